"""Plain FP64 CPU oracle of the NOLSM hot path.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute this module; only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it. It shares no code with the HIP path.

What it computes, step by step (Schade et al., Sec. III-B.2, "The Submatrix
Method" and "The Non-Orthogonal Local Submatrix Method"):

  1. validate the block-CSR patterns of K (the Hamiltonian H_0) and S;
  2. merge the two patterns: block row I belongs to the submatrix of column
     block J iff K_IJ or S_IJ is stored (NOLSM generation step);
  3. gather the dense submatrices T_J(K), T_J(S) on the sorted index list N(J);
  4. Cholesky S_J = L L^T (a non-positive pivot means "not SPD");
  5. A_J = S_J^-1 K_J - mu I and Y_J = S_J^-1 E_cJ (the molecule's columns);
  6. scale by c_J = 1 / ||A_J||_inf so that the sign iteration converges
     (the paper only says the matrix is rescaled before the iteration);
  7. Newton-Schulz sign iteration (Eq. NS1-NS2): X_0 = c A,
     X_{k+1} = X_k (3I - X_k^2) / 2, stopped at the first X_k with
     ||X_k^2 - I||_F < tol;
  8. the owned columns of the purified submatrix (Eq. purification_submatrix):
     T_J(D)[:, cJ] = (I - sign(A_J)) S_J^-1 E_cJ / 2 = (Y_J - X Y_J) / 2;
  9. write-back of those columns into D, which keeps the merged pattern;
 10. per-molecule traces N_J = sum_c (S_J Dcols)[cJ_c, c] and
     E_J = sum_c (K_J Dcols)[cJ_c, c] (Eq. e_elec restricted to column J).

Readings where the paper is silent: rows of T_J are kept in ascending global
block order; absent blocks inside a submatrix are gathered as zeros; D is the
orbital projector with no spin factor; D is not symmetrised.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

OK = 0
NOT_SPD = 1
NOCONV = 2


class PatternError(ValueError):
    pass


# --------------------------------------------------------------------------
# 1-2: validation and merge (Sec. III-B.2, NOLSM generation step)
# --------------------------------------------------------------------------

def validate_pattern(nb, row_ptr, col_idx):
    """Rows monotone, columns strictly increasing and in range, diagonal block
    present, pattern symmetric. Raises PatternError."""
    row_ptr = np.asarray(row_ptr)
    col_idx = np.asarray(col_idx)
    if row_ptr.shape[0] != nb + 1 or row_ptr[0] != 0 or row_ptr[-1] != col_idx.shape[0]:
        raise PatternError("row_ptr shape/limits")
    if np.any(np.diff(row_ptr) < 0):
        raise PatternError("row_ptr not monotone")
    pairs = set()
    for i in range(nb):
        cols = col_idx[row_ptr[i]:row_ptr[i + 1]]
        if len(cols) and (cols.min() < 0 or cols.max() >= nb):
            raise PatternError("column out of range")
        if np.any(np.diff(cols) <= 0):
            raise PatternError("columns not strictly increasing")
        if i not in set(cols.tolist()):
            raise PatternError("diagonal block missing")
        for c in cols.tolist():
            pairs.add((i, c))
    for (i, c) in pairs:
        if (c, i) not in pairs:
            raise PatternError("pattern not symmetric")


def merge(nb, K_row_ptr, K_col_idx, S_row_ptr, S_col_idx):
    """Merged pattern P = pat(K) u pat(S). Returns, per column block J, the
    sorted list N(J) = {I : (I, J) in P}, and J's position p_J in it.

    Since both patterns are symmetric, N(J) is also row J of P."""
    lists = []
    self_pos = np.empty(nb, dtype=np.int64)
    for J in range(nb):
        a = set(np.asarray(K_col_idx[K_row_ptr[J]:K_row_ptr[J + 1]]).tolist())
        b = set(np.asarray(S_col_idx[S_row_ptr[J]:S_row_ptr[J + 1]]).tolist())
        nj = sorted(a | b)
        lists.append(np.array(nj, dtype=np.int64))
        self_pos[J] = nj.index(J)
    return lists, self_pos


def plan_arrays(nb, K_row_ptr, K_col_idx, S_row_ptr, S_col_idx):
    """Integer arrays of the merged plan, for exact comparison with the
    library's plan: sub_ptr, sub_blk, self_pos, and the pattern of D
    (D_row_ptr, D_col_idx, which is P itself) with scatter_pos[sub_ptr[J]+a]
    = index in D's block-CSR of block (N(J)_a, J)."""
    lists, self_pos = merge(nb, K_row_ptr, K_col_idx, S_row_ptr, S_col_idx)
    sub_ptr = np.zeros(nb + 1, dtype=np.int64)
    for J in range(nb):
        sub_ptr[J + 1] = sub_ptr[J] + len(lists[J])
    sub_blk = np.concatenate(lists) if nb else np.zeros(0, dtype=np.int64)
    # D pattern: row I holds column J iff I in N(J)
    rows = [[] for _ in range(nb)]
    for J in range(nb):
        for I in lists[J].tolist():
            rows[I].append(J)
    D_row_ptr = np.zeros(nb + 1, dtype=np.int64)
    for I in range(nb):
        rows[I].sort()
        D_row_ptr[I + 1] = D_row_ptr[I] + len(rows[I])
    D_col_idx = np.array([c for r in rows for c in r], dtype=np.int64)
    scatter_pos = np.empty(sub_ptr[-1], dtype=np.int64)
    for J in range(nb):
        for a, I in enumerate(lists[J].tolist()):
            scatter_pos[sub_ptr[J] + a] = D_row_ptr[I] + rows[I].index(J)
    return dict(sub_ptr=sub_ptr, sub_blk=sub_blk, self_pos=self_pos,
                D_row_ptr=D_row_ptr, D_col_idx=D_col_idx, scatter_pos=scatter_pos)


# --------------------------------------------------------------------------
# 3: gather (Sec. III-B.2, submatrix construction T_j)
# --------------------------------------------------------------------------

def find_block(row_ptr, col_idx, I, J):
    lo, hi = int(row_ptr[I]), int(row_ptr[I + 1])
    k = lo + int(np.searchsorted(col_idx[lo:hi], J))
    if k < hi and col_idx[k] == J:
        return k
    return -1


def gather(idx, bs, row_ptr, col_idx, val):
    """Dense submatrix on block indices idx (ascending): block (a, b) is the
    stored block (idx[a], idx[b]) or zero."""
    m = len(idx)
    out = np.zeros((m * bs, m * bs), dtype=np.float64)
    for a, I in enumerate(idx):
        for b, J in enumerate(idx):
            k = find_block(row_ptr, col_idx, int(I), int(J))
            if k >= 0:
                out[a * bs:(a + 1) * bs, b * bs:(b + 1) * bs] = val[k]
    return out


def gather_vectorized(idx, bs, row_ptr, col_idx, val):
    """Same result as gather(), with the block lookups done by one sorted
    search per row (for label generation on large submatrices)."""
    idx = np.asarray(idx)
    m = len(idx)
    out = np.zeros((m, bs, m, bs))
    for a, I in enumerate(idx):
        lo, hi = int(row_ptr[I]), int(row_ptr[I + 1])
        cols = col_idx[lo:hi]
        pos = np.searchsorted(idx, cols)
        pos_c = np.minimum(pos, m - 1)
        hit = idx[pos_c] == cols
        out[a, :, pos_c[hit], :] = val[lo:hi][hit]
    return out.reshape(m * bs, m * bs)


# --------------------------------------------------------------------------
# 4-8: per-submatrix purification (Eq. purification_submatrix, Eq. NS1-NS2)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class SubResult:
    status: int
    Dcols: np.ndarray | None     # (n_J, bs)
    X: np.ndarray | None         # converged sign iterate (n_J, n_J)
    A: np.ndarray | None
    iters: int
    resid: float
    scale: float
    N_J: float
    E_J: float
    Wcols: np.ndarray | None = None   # (n_J, bs), only when asked for


def newton_schulz_sign(A, c, tol=1e-10, max_iter=100, restart_at=None):
    """X_0 = c A; X_{k+1} = X_k (3I - X_k^2)/2 (Eq. NS1); returns the first
    X_k with ||X_k^2 - I||_F < tol, the number of updates taken, and that
    residual. Reaching max_iter means no convergence.
    restart_at = k (the injected stall of the divergence guard, not in the
    paper): after the residual of X_k, X_{k+1} = c A instead of the update,
    the guard's restart from the initial scale; the sign reached is the same."""
    n = A.shape[0]
    I = np.eye(n)
    X = c * A
    r = np.inf
    for k in range(max_iter):
        T = X @ X
        r = float(np.linalg.norm(T - I, "fro"))
        if k == restart_at:
            X = c * A
            continue
        if r < tol:
            return X, k, r, True
        X = 0.5 * (X @ (3.0 * I - T))
    return X, max_iter, r, False


def coupled_ns_inverse(S, c, tol=1e-12, max_iter=100):
    """Inverse of an SPD submatrix by the coupled Newton-Schulz iteration
    (Eq. inv1-inv3): Y_0 = c S, Z_0 = I, V_k = Z_k Y_k,
    Y_{k+1} = Y_k (3I - V_k) / 2, Z_{k+1} = (3I - V_k) Z_k / 2; Z_k tends to
    (c S)^(-1/2), so S^-1 = c Z^2. Returns (S^-1, iterations, ||V - I||_F,
    converged); stops at the first k with ||V_k - I||_F < tol. c must put the
    spectrum of c S inside (0, 2) (here: c = 1 / max row sum of |S|)."""
    n = S.shape[0]
    I = np.eye(n)
    Y = c * S
    Z = I.copy()
    r = np.inf
    for k in range(max_iter):
        V = Z @ Y
        r = float(np.linalg.norm(V - I, "fro"))
        if r < tol:
            return c * (Z @ Z), k, r, True
        T = 3.0 * I - V
        Y, Z = 0.5 * (Y @ T), 0.5 * (T @ Z)
    return c * (Z @ Z), max_iter, r, False


def solve_submatrix(KJ, SJ, p, bs, mu, tol=1e-10, max_iter=100, scale=None, want_w=False,
                    inverse="cholesky", restart_at=None):
    """Everything inside one submatrix, for the molecule at block position p.
    inverse="coupled_ns" applies T_J(S)^-1 from the coupled Newton-Schulz
    iteration (Eq. inv1-inv3, FP64, converged to 1e-12) instead of the
    Cholesky factor; both give the same D up to rounding.
    With want_w, also the owned columns of the energy-weighted density
    matrix T_J(W) = T_J(D) T_J(K) T_J(D) (Sec. III-B.2), from the full
    T_J(D) = (I - X) T_J(S)^-1 / 2."""
    n = KJ.shape[0]
    try:
        L = np.linalg.cholesky(SJ)
    except np.linalg.LinAlgError:
        return SubResult(NOT_SPD, None, None, None, 0, np.nan, np.nan, np.nan, np.nan)
    if not np.all(np.diag(L) > 0):
        return SubResult(NOT_SPD, None, None, None, 0, np.nan, np.nan, np.nan, np.nan)
    if inverse == "coupled_ns":
        Sinv, _, _, ok = coupled_ns_inverse(SJ, 1.0 / np.abs(SJ).sum(axis=1).max())
        if not ok:
            return SubResult(NOT_SPD, None, None, None, 0, np.nan, np.nan, np.nan, np.nan)

        def s_inv(B):
            return Sinv @ B
    else:
        def s_inv(B):
            W = sla.solve_triangular(L, B, lower=True)
            return sla.solve_triangular(L.T, W, lower=False)
    A = s_inv(KJ) - mu * np.eye(n)
    E = np.zeros((n, bs))
    E[p * bs:(p + 1) * bs, :] = np.eye(bs)
    Y = s_inv(E)
    c = 1.0 / np.abs(A).sum(axis=1).max() if scale is None else scale
    X, iters, r, conv = newton_schulz_sign(A, c, tol, max_iter, restart_at)
    Dcols = 0.5 * (Y - X @ Y)
    rows = slice(p * bs, (p + 1) * bs)
    N_J = float(np.trace(SJ[rows, :] @ Dcols))
    E_J = float(np.trace(KJ[rows, :] @ Dcols))
    Wcols = None
    if want_w:
        DJ = 0.5 * (np.eye(n) - X) @ s_inv(np.eye(n))
        Wcols = DJ @ (KJ @ Dcols)
    return SubResult(OK if conv else NOCONV, Dcols, X, A, iters, r, c, N_J, E_J, Wcols)


# --------------------------------------------------------------------------
# 9-10: whole batch, write-back and diagnostics (Sec. III-B.2 write-back)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class BatchResult:
    plan: dict
    Dcols: list            # per J, (n_J, bs)
    D_val: np.ndarray      # (nnzb(D), bs, bs) on D's block-CSR = merged pattern
    status: np.ndarray
    iters: np.ndarray
    resid: np.ndarray
    scale: np.ndarray
    N: np.ndarray          # per-molecule Tr(S D) share
    E: np.ndarray          # per-molecule Tr(K D) share
    Wcols: list | None = None     # per J, (n_J, bs), with want_w
    W_val: np.ndarray | None = None   # W on D's block-CSR, with want_w


def nolsm(system, mu=None, tol=1e-10, max_iter=100, molecules=None, keep_x=False, want_w=False):
    """The NOLSM density matrix of a synth.System (or anything with the same
    K/S block-CSR fields). `molecules` restricts the solve to a subset of
    column blocks (the remaining Dcols entries are None). With want_w, also
    the energy-weighted density matrix W, written back like D."""
    K, S = system.K, system.S
    nb, bs = K.nb, K.bs
    mu = system.mu if mu is None else mu
    plan = plan_arrays(nb, K.row_ptr, K.col_idx, S.row_ptr, S.col_idx)
    sub_ptr, sub_blk = plan["sub_ptr"], plan["sub_blk"]
    todo = range(nb) if molecules is None else molecules
    Dcols = [None] * nb
    D_val = np.zeros((plan["D_col_idx"].shape[0], bs, bs))
    status = np.full(nb, -1, dtype=np.int64)
    iters = np.zeros(nb, dtype=np.int64)
    resid = np.full(nb, np.nan)
    scale = np.full(nb, np.nan)
    N = np.full(nb, np.nan)
    E = np.full(nb, np.nan)
    Wcols = [None] * nb if want_w else None
    W_val = np.zeros_like(D_val) if want_w else None
    xs = {}
    for J in todo:
        idx = sub_blk[sub_ptr[J]:sub_ptr[J + 1]]
        p = int(plan["self_pos"][J])
        KJ = gather(idx, bs, K.row_ptr, K.col_idx, K.val)
        SJ = gather(idx, bs, S.row_ptr, S.col_idx, S.val)
        r = solve_submatrix(KJ, SJ, p, bs, mu, tol, max_iter, want_w=want_w)
        status[J], iters[J], resid[J], scale[J] = r.status, r.iters, r.resid, r.scale
        if r.Dcols is None:
            continue
        Dcols[J] = r.Dcols
        N[J], E[J] = r.N_J, r.E_J
        for a in range(len(idx)):
            D_val[plan["scatter_pos"][sub_ptr[J] + a]] = r.Dcols[a * bs:(a + 1) * bs, :]
        if want_w:
            Wcols[J] = r.Wcols
            for a in range(len(idx)):
                W_val[plan["scatter_pos"][sub_ptr[J] + a]] = r.Wcols[a * bs:(a + 1) * bs, :]
        if keep_x:
            xs[J] = (r.X, r.A)
    res = BatchResult(plan, Dcols, D_val, status, iters, resid, scale, N, E, Wcols, W_val)
    if keep_x:
        res.xs = xs
    return res


def nolsm_groups(system, groups, mu=None, tol=1e-10, max_iter=100):
    """NOLSM on combined submatrices (Sec. III-B, submatrix combination):
    `groups` = (grp_ptr, grp_blk, own_ptr, own_J) as from
    oracle.combine.combine_groups. Each group's submatrix T_g is built on
    its row blocks R_g; one sign iteration serves every molecule J it owns,
    whose columns are T_g(D)[:, cJ] = (Y_J - X Y_J) / 2 with
    Y_J = T_g(S)^-1 E_cJ. Only the rows N(J) are written back, so D keeps
    the merged pattern of K and S. Returns a BatchResult (Dcols per
    molecule on N(J); iters/resid/scale repeated for every owned molecule)."""
    K, S = system.K, system.S
    nb, bs = K.nb, K.bs
    mu = system.mu if mu is None else mu
    plan = plan_arrays(nb, K.row_ptr, K.col_idx, S.row_ptr, S.col_idx)
    sub_ptr, sub_blk = plan["sub_ptr"], plan["sub_blk"]
    grp_ptr, grp_blk, own_ptr, own_J = groups
    Dcols = [None] * nb
    D_val = np.zeros((plan["D_col_idx"].shape[0], bs, bs))
    status = np.full(nb, -1, dtype=np.int64)
    iters = np.zeros(nb, dtype=np.int64)
    resid = np.full(nb, np.nan)
    scale = np.full(nb, np.nan)
    N = np.full(nb, np.nan)
    E = np.full(nb, np.nan)
    for g in range(len(grp_ptr) - 1):
        rows = grp_blk[grp_ptr[g]:grp_ptr[g + 1]]
        where = {int(b): a for a, b in enumerate(rows)}
        KG = gather(rows, bs, K.row_ptr, K.col_idx, K.val)
        SG = gather(rows, bs, S.row_ptr, S.col_idx, S.val)
        n = KG.shape[0]
        owned = own_J[own_ptr[g]:own_ptr[g + 1]]
        try:
            L = np.linalg.cholesky(SG)
            ok = bool(np.all(np.diag(L) > 0))
        except np.linalg.LinAlgError:
            ok = False
        if not ok:
            for J in owned:
                status[J] = NOT_SPD
            continue
        def s_inv(B):
            W = sla.solve_triangular(L, B, lower=True)
            return sla.solve_triangular(L.T, W, lower=False)
        A = s_inv(KG) - mu * np.eye(n)
        c = 1.0 / np.abs(A).sum(axis=1).max()
        X, it, r, conv = newton_schulz_sign(A, c, tol, max_iter)
        for J in owned:
            J = int(J)
            q = where[J]
            Ec = np.zeros((n, bs))
            Ec[q * bs:(q + 1) * bs, :] = np.eye(bs)
            Y = s_inv(Ec)
            Dfull = 0.5 * (Y - X @ Y)
            idx = sub_blk[sub_ptr[J]:sub_ptr[J + 1]]
            sel = np.concatenate([np.arange(where[int(I)] * bs, where[int(I)] * bs + bs) for I in idx])
            Dcols[J] = Dfull[sel, :]
            qrows = slice(q * bs, (q + 1) * bs)
            N[J] = float(np.trace(SG[qrows, :] @ Dfull))
            E[J] = float(np.trace(KG[qrows, :] @ Dfull))
            status[J], iters[J], resid[J], scale[J] = (OK if conv else NOCONV), it, r, c
            for a in range(len(idx)):
                D_val[plan["scatter_pos"][sub_ptr[J] + a]] = Dcols[J][a * bs:(a + 1) * bs, :]
    return BatchResult(plan, Dcols, D_val, status, iters, resid, scale, N, E)


def neighbour_lists(system):
    """N(J) lists and p_J of a system, merged once and cached on it."""
    cache = getattr(system, "_oracle_lists", None)
    if cache is None:
        K, S = system.K, system.S
        cache = merge(K.nb, K.row_ptr, K.col_idx, S.row_ptr, S.col_idx)
        system._oracle_lists = cache
    return cache


def submatrix(system, J, mu=None):
    """Dense K_J, S_J, the block list N(J) and p_J (for tests and labels)."""
    K, S = system.K, system.S
    lists, self_pos = neighbour_lists(system)
    idx = lists[J]
    KJ = gather(idx, K.bs, K.row_ptr, K.col_idx, K.val)
    SJ = gather(idx, S.bs, S.row_ptr, S.col_idx, S.val)
    return KJ, SJ, idx, int(self_pos[J])


def solve_molecule(system, J, mu=None, tol=1e-10, max_iter=100, want_w=False, inverse="cholesky",
                   restart_at=None):
    """Steps 3-8 and 10 for one column block J, without assembling D (for
    sampled checks on systems too large for the whole-batch oracle)."""
    mu = system.mu if mu is None else mu
    KJ, SJ, idx, p = submatrix(system, J)
    return solve_submatrix(KJ, SJ, p, system.K.bs, mu, tol, max_iter, want_w=want_w, inverse=inverse,
                           restart_at=restart_at)


def dense(csr):
    """The full dense matrix of a block-CSR (small systems only)."""
    nb, bs = csr.nb, csr.bs
    out = np.zeros((nb * bs, nb * bs))
    for I in range(nb):
        for k in range(csr.row_ptr[I], csr.row_ptr[I + 1]):
            J = csr.col_idx[k]
            out[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs] = csr.val[k]
    return out


def dense_from_pattern(nb, bs, row_ptr, col_idx, val):
    out = np.zeros((nb * bs, nb * bs))
    for I in range(nb):
        for k in range(row_ptr[I], row_ptr[I + 1]):
            J = col_idx[k]
            out[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs] = val[k]
    return out


def gershgorin(A):
    """Row and column Gershgorin intervals [lo, hi] enclosing the spectrum."""
    d = np.diag(A)
    off = np.abs(A) - np.diag(np.abs(d))
    rr = off.sum(axis=1)
    cr = off.sum(axis=0)
    row = (float((d - rr).min()), float((d + rr).max()))
    col = (float((d - cr).min()), float((d + cr).max()))
    return row, col
