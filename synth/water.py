"""Seeded synthetic water-like inputs for the NOLSM hot path.

This module only *constructs inputs*: molecule positions, the block-sparse
overlap matrix S and Kohn-Sham-like matrix K in block-CSR form. It holds none
of the method's arithmetic (no inversion, no sign iteration, no write-back),
so both the CPU oracle and the GPU path may consume what it produces.

The paper's workloads (Sec. IV-A: liquid water built from a 32-molecule cell,
one atom-group per submatrix; an inhomogeneous solvated system) are not
available here, so the systems below stand in for them with the same shape:
molecules at liquid-water density, a few localized basis functions per
molecule, distance-truncated blocks, and submatrix sizes in the few-hundred
to ~1500 range the paper reports (Sec. III-A, Sec. V-A).

Recipe (all lengths in nm):
  * positions: random sequential addition (RSA) in a periodic box with a
    minimum-image separation of at least 0.25 nm between molecule centres;
  * 6 basis functions per molecule, each centred at the molecule centre plus
    an independent N(0, 0.03^2) offset per axis;
  * pattern: block (I, J) is stored iff the minimum-image distance between
    molecule centres is strictly below the cutoff r_c (diagonal blocks always);
  * S_ij = exp(-r_ij^2 / 0.02) over stored blocks, plus 0.1 on the diagonal;
  * K_ii = onsite energy (functions 0-3 ~ U(-1.1, -0.9), functions 4-5 ~
    U(0.9, 1.1)); K_ij = 0.2 exp(-r_ij / 0.1) for every other pair inside a
    stored block (intra-molecular pairs included);
  * r_ij is the minimum-image distance between basis-function centres.
Seeds: SeedSequence(20210417 + config_id).spawn(4) -> streams for positions,
jitter, onsite energies and sampling.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.spatial import cKDTree

BS = 6                   # basis functions per molecule
DENSITY = 33.4           # molecules / nm^3 (liquid water)
MIN_SEP = 0.25           # nm, minimum molecule-centre separation
JITTER = 0.03            # nm, std-dev of basis-centre offsets
S_WIDTH = 0.02           # nm^2, Gaussian overlap width
S_SHIFT = 0.1            # diagonal shift of S
K_HOP = 0.2              # hopping prefactor
K_DECAY = 0.1            # nm, hopping decay length
SEED_BASE = 20210417


@dataclasses.dataclass
class BlockCSR:
    """Square block-sparse matrix pattern (+ optional values), bs x bs blocks.

    row_ptr[nb+1], col_idx[nnzb] (int32, strictly increasing per row);
    values, if present, are float64 of shape (nnzb, bs, bs), blocks row-major.
    """
    nb: int
    bs: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray | None = None

    @property
    def nnzb(self) -> int:
        return int(self.col_idx.shape[0])


@dataclasses.dataclass
class System:
    box: np.ndarray          # (3,) periodic box lengths
    r_c: float
    centres: np.ndarray      # (N, 3) molecule centres
    basis: np.ndarray        # (N, BS, 3) basis-function centres
    onsite: np.ndarray       # (N, BS) onsite energies (diagonal of K)
    K: BlockCSR
    S: BlockCSR
    mu: float = 0.0
    sample_rng: np.random.Generator | None = None

    @property
    def nmol(self) -> int:
        return int(self.centres.shape[0])


def streams(config_id: int):
    ss = np.random.SeedSequence(SEED_BASE + int(config_id))
    return [np.random.default_rng(s) for s in ss.spawn(4)]


def min_image(d: np.ndarray, box: np.ndarray) -> np.ndarray:
    return d - box * np.round(d / box)


def _conflicts_existing(tree, cand, box):
    if tree is None:
        return np.zeros(len(cand), dtype=bool)
    dist, _ = tree.query(cand, k=1, distance_upper_bound=MIN_SEP)
    return np.isfinite(dist)


def rsa_region(rng, count, box, lo, hi, placed, max_reject_factor=1000):
    """Random sequential addition of `count` centres, uniform in the region
    lo <= x < hi of the periodic `box`, keeping every centre at least MIN_SEP
    (minimum image) from all centres placed so far (including `placed`).

    Candidates are drawn in batches; a candidate is accepted iff it clears all
    previously accepted centres and every earlier accepted candidate of its
    own batch (processed in draw order), which keeps the result a function of
    the seed alone."""
    box = np.asarray(box, dtype=np.float64)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    pts = [p for p in placed] if placed is not None and len(placed) else []
    out = []
    rejected = 0
    while len(out) < count:
        need = count - len(out)
        batch = int(min(max(2 * need, 64), 65536))
        cand = lo + (hi - lo) * rng.random((batch, 3))
        allp = np.array(pts + out) if (pts or out) else None
        tree = cKDTree(np.mod(allp, box), boxsize=box) if allp is not None else None
        ok = ~_conflicts_existing(tree, np.mod(cand, box), box)
        cand_ok = cand[ok]
        rejected += int((~ok).sum())
        # resolve conflicts inside the batch, first-drawn wins
        if len(cand_ok) > 1:
            ctree = cKDTree(np.mod(cand_ok, box), boxsize=box)
            pairs = ctree.query_pairs(MIN_SEP, output_type="ndarray")
            keep = np.ones(len(cand_ok), dtype=bool)
            if len(pairs):
                nbrs = [[] for _ in range(len(cand_ok))]
                for a, b in pairs:
                    lo_i, hi_i = (a, b) if a < b else (b, a)
                    nbrs[hi_i].append(lo_i)
                for i in range(len(cand_ok)):
                    for j in nbrs[i]:
                        if keep[j]:
                            keep[i] = False
                            break
            rejected += int((~keep).sum())
            cand_ok = cand_ok[keep]
        out.extend(list(cand_ok[:need]))
        if rejected > max_reject_factor * max(count, 1):
            raise RuntimeError("random sequential addition: too many rejections")
    return np.array(out, dtype=np.float64).reshape(-1, 3)


def neighbour_pairs(centres, box, r_c):
    """All molecule pairs (I < J) with minimum-image centre distance < r_c."""
    n = centres.shape[0]
    box = np.asarray(box, dtype=np.float64)
    if n <= 2048 or r_c >= 0.5 * box.min():
        d = min_image(centres[:, None, :] - centres[None, :, :], box)
        r = np.sqrt((d * d).sum(-1))
        iu, ju = np.triu_indices(n, k=1)
        m = r[iu, ju] < r_c
        return iu[m].astype(np.int64), ju[m].astype(np.int64)
    tree = cKDTree(np.mod(centres, box), boxsize=box)
    pairs = tree.query_pairs(r_c, output_type="ndarray").astype(np.int64)
    a = np.minimum(pairs[:, 0], pairs[:, 1])
    b = np.maximum(pairs[:, 0], pairs[:, 1])
    d = min_image(centres[a] - centres[b], box)
    r = np.sqrt((d * d).sum(-1))
    m = r < r_c
    a, b = a[m], b[m]
    order = np.lexsort((b, a))
    return a[order], b[order]


def pattern_from_pairs(n, iu, ju):
    rows = np.concatenate([iu, ju, np.arange(n)])
    cols = np.concatenate([ju, iu, np.arange(n)])
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return row_ptr.astype(np.int32), cols.astype(np.int32), rows


def block_values(basis, onsite, box, rows, cols, chunk=200_000):
    """Dense 6x6 values of K and S for the listed blocks (rows[k], cols[k])."""
    nnzb = rows.shape[0]
    K = np.empty((nnzb, BS, BS), dtype=np.float64)
    S = np.empty((nnzb, BS, BS), dtype=np.float64)
    eye = np.eye(BS, dtype=bool)
    for s in range(0, nnzb, chunk):
        r_ = rows[s:s + chunk]
        c_ = cols[s:s + chunk]
        d = basis[r_][:, :, None, :] - basis[c_][:, None, :, :]
        d = min_image(d, box)
        r2 = (d * d).sum(-1)
        r = np.sqrt(r2)
        sv = np.exp(-r2 / S_WIDTH)
        kv = K_HOP * np.exp(-r / K_DECAY)
        diag = r_ == c_
        if diag.any():
            idx = np.nonzero(diag)[0]
            sv[idx] += S_SHIFT * eye
            kv[idx[:, None], np.arange(BS)[None, :], np.arange(BS)[None, :]] = onsite[r_[idx]]
        S[s:s + chunk] = sv
        K[s:s + chunk] = kv
    return K, S


def build_system(centres, box, r_c, jitter_rng, onsite_rng, sample_rng=None, basis=None, onsite=None):
    box = np.asarray(box, dtype=np.float64)
    n = centres.shape[0]
    if basis is None:
        basis = centres[:, None, :] + JITTER * jitter_rng.standard_normal((n, BS, 3))
    if onsite is None:
        onsite = np.concatenate([onsite_rng.uniform(-1.1, -0.9, (n, 4)),
                                 onsite_rng.uniform(0.9, 1.1, (n, 2))], axis=1)
    iu, ju = neighbour_pairs(centres, box, r_c)
    # values for the upper triangle + diagonal, mirrored exactly for the lower
    up_r = np.concatenate([iu, np.arange(n)])
    up_c = np.concatenate([ju, np.arange(n)])
    Ku, Su = block_values(basis, onsite, box, up_r, up_c)
    row_ptr, col_idx, rows = pattern_from_pairs(n, iu, ju)
    # map each stored block to its upper-triangle source (transposed if lower)
    key_up = up_r * n + up_c
    order_up = np.argsort(key_up)
    lo = np.minimum(rows, col_idx)
    hi = np.maximum(rows, col_idx)
    src = order_up[np.searchsorted(key_up[order_up], lo * n + hi)]
    transpose = rows > col_idx
    Kv = Ku[src]
    Sv = Su[src]
    Kv[transpose] = np.swapaxes(Kv[transpose], 1, 2)
    Sv[transpose] = np.swapaxes(Sv[transpose], 1, 2)
    Kc = BlockCSR(n, BS, row_ptr, col_idx, np.ascontiguousarray(Kv))
    Sc = BlockCSR(n, BS, row_ptr.copy(), col_idx.copy(), np.ascontiguousarray(Sv))
    return System(box=box, r_c=float(r_c), centres=centres, basis=basis, onsite=onsite,
                  K=Kc, S=Sc, mu=0.0, sample_rng=sample_rng)


def truncate(csr, centres, box, r_cut):
    """The blocks of `csr` whose molecule centres lie strictly closer than
    r_cut (minimum image); diagonal blocks always stay. Values are copied."""
    rows = np.repeat(np.arange(csr.nb), np.diff(csr.row_ptr))
    cols = csr.col_idx.astype(np.int64)
    d = min_image(centres[rows] - centres[cols], np.asarray(box, dtype=np.float64))
    keep = (np.sqrt((d * d).sum(-1)) < r_cut) | (rows == cols)
    row_ptr = np.zeros(csr.nb + 1, dtype=np.int64)
    np.add.at(row_ptr, rows[keep] + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    val = None if csr.val is None else np.ascontiguousarray(csr.val[keep])
    return BlockCSR(csr.nb, csr.bs, row_ptr, csr.col_idx[keep].copy(), val)


def two_cutoffs(system, r_k=None, r_s=None):
    """The same system with K (or S) truncated at a smaller cutoff than the
    other matrix, so that the two block patterns differ: with r_k < r_c the
    pattern of S strictly contains that of K, with r_s < r_c the reverse."""
    K = truncate(system.K, system.centres, system.box, r_k) if r_k is not None else system.K
    S = truncate(system.S, system.centres, system.box, r_s) if r_s is not None else system.S
    return dataclasses.replace(system, K=K, S=S)


def cubic_box(nmol, density=DENSITY):
    L = (nmol / density) ** (1.0 / 3.0)
    return np.array([L, L, L])


def water_cube(nmol, r_c, config_id, density=DENSITY):
    """Homogeneous cubic box at the given density."""
    pos_rng, jit_rng, ons_rng, smp_rng = streams(config_id)
    box = cubic_box(nmol, density)
    centres = rsa_region(pos_rng, nmol, box, np.zeros(3), box, None)
    return build_system(centres, box, r_c, jit_rng, ons_rng, smp_rng)


SLAB_BOX = np.array([8.0, 8.0, 16.632])
SLAB_DENSE_Z = 3.832


def water_slab(config_id=4, r_c=1.2, n_dense=8192, n_dilute=8192, box=SLAB_BOX,
               z_split=SLAB_DENSE_Z):
    """Periodic slab: a liquid-density layer (z < z_split) and a dilute layer
    (10 molecules/nm^3 for the default sizes), separation enforced globally."""
    pos_rng, jit_rng, ons_rng, smp_rng = streams(config_id)
    box = np.asarray(box, dtype=np.float64)
    dense = rsa_region(pos_rng, n_dense, box, np.zeros(3),
                       np.array([box[0], box[1], z_split]), None)
    dilute = rsa_region(pos_rng, n_dilute, box, np.array([0.0, 0.0, z_split]), box, dense)
    centres = np.concatenate([dense, dilute], axis=0)
    return build_system(centres, box, r_c, jit_rng, ons_rng, smp_rng)


def trajectory(nframes=10, nmol=4096, r_c=0.9, config_id=5, step=0.01):
    """Frame 0: a fresh homogeneous box; frame f: frame f-1 with every molecule
    moved by N(0, step^2) per axis (cumulative, basis offsets rigid, onsite
    energies fixed, pattern recomputed per frame)."""
    pos_rng, jit_rng, ons_rng, smp_rng = streams(config_id)
    box = cubic_box(nmol)
    centres = rsa_region(pos_rng, nmol, box, np.zeros(3), box, None)
    offsets = JITTER * jit_rng.standard_normal((nmol, BS, 3))
    onsite = np.concatenate([ons_rng.uniform(-1.1, -0.9, (nmol, 4)),
                             ons_rng.uniform(0.9, 1.1, (nmol, 2))], axis=1)
    frames = []
    for f in range(nframes):
        if f > 0:
            centres = centres + step * pos_rng.standard_normal(centres.shape)
        basis = centres[:, None, :] + offsets
        frames.append(build_system(centres, box, r_c, None, None, smp_rng,
                                   basis=basis, onsite=onsite))
    return frames


# The five workloads, by id. Sizes follow the submatrix-size ranges of the
# paper's water and solvated-capsid benchmarks (Sec. IV-A, Sec. V-A).
CONFIGS = {
    1: dict(kind="cube", nmol=64, r_c=0.6),
    2: dict(kind="cube", nmol=4096, r_c=0.9),
    3: dict(kind="cube", nmol=32768, r_c=0.9),
    4: dict(kind="slab", nmol=16384, r_c=1.2),
    5: dict(kind="trajectory", nmol=4096, r_c=0.9, nframes=10),
}


def make_config(config_id: int):
    c = CONFIGS[config_id]
    if c["kind"] == "cube":
        return water_cube(c["nmol"], c["r_c"], config_id)
    if c["kind"] == "slab":
        return water_slab(config_id, c["r_c"])
    return trajectory(c["nframes"], c["nmol"], c["r_c"], config_id)
