// Plan / index build of the NOLSM hot path (host work).
//
// Sec. III-B.2 (NOLSM generation step, Fig. 2 b-c): the row indices of a
// column's submatrix are the union of the rows where K (H_0) or S has a
// stored block in that column. Both inputs are symmetric block patterns, so
// the index list N(J) of column block J is the merged block row J. The result
// matrix D keeps the merged pattern (the submatrix approximation has the
// sparsity of its input).
#include <algorithm>
#include <queue>
#include <iterator>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "plan.h"

static thread_local std::string g_last_error;
void nolsm_set_last_error(const std::string &s) { g_last_error = s; }

static inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Newton-Schulz tile edge of a submatrix with np rows: FP64/FP32 use 64;
// FP16/BF16 use 128 unless bit (np/64 - 1) of small_mask asks for 64.
int nolsm_ns_tile_for(int32_t prec, int32_t np, uint64_t small_mask) {
    if (prec != NOLSM_FP16 && prec != NOLSM_BF16) return 64;
    const int b = np / 64 - 1;
    return (b >= 0 && b < 64 && ((small_mask >> b) & 1u)) ? 64 : 128;
}
int nolsm_elem_for(int32_t prec) {
    switch (prec) {
        case NOLSM_FP64: return 8;
        case NOLSM_FP32: return 4;
        default: return 2;
    }
}

// Residual below which the 16-bit sign iteration hands over to the FP32
// finishing iterations (a tol < 0 asks for it; tol >= 0 is used as given).
// One Newton-Schulz step maps e = 1 - x^2 of every eigenvalue x to
// 3/4 e^2 + 1/4 e^3, and ||X^2 - I||_F bounds every |e|, so f FP32 steps
// from a residual r leave 3/4 r^2 (f = 1) or 27/64 r^4 (f = 2) to leading
// order. The switch point puts that below a tenth of the unit roundoff u of
// the 16-bit format (2^-11 FP16, 2^-8 BF16), under the rounding the 16-bit
// iterate itself carries: FP16 0.104, BF16 0.174 with f = 2. Without
// finishing steps only the stagnation test stops the iteration.
extern "C" double nolsm_switch_tol(int32_t prec, int32_t n_final_fp32, double tol) {
    if (tol >= 0.0) return tol;
    if (prec == NOLSM_FP64) return 1e-10;
    if (prec == NOLSM_FP32) return 1e-5;
    const double u = (prec == NOLSM_FP16) ? std::ldexp(1.0, -11) : std::ldexp(1.0, -8);
    if (n_final_fp32 >= 2) return std::pow(u / 10.0 * 64.0 / 27.0, 0.25);
    if (n_final_fp32 == 1) return std::sqrt(u / 10.0 * 4.0 / 3.0);
    return 0.0;
}

size_t nolsm_slot_bytes(int32_t np, int32_t ns_tile, int32_t elem, int32_t max_iter, int32_t inverse,
                        int32_t nown, int32_t sym) {
    const size_t n = (size_t)np;
    const size_t P = n / NOLSM_TILE;
    const size_t nt = (n + ns_tile - 1) / ns_tile;
    size_t b = 0;
    b += align256(n * n * 8);                 // L / X0
    // K / W / A|Y: FP32 when the substitution runs in FP32 arithmetic
    const bool kf32 = inverse == NOLSM_INV_CHOLESKY_FP32 || inverse == NOLSM_INV_CHOLESKY_APPLY_FP32;
    b += align256(n * (n + 64) * (kf32 ? 4 : 8));
    b += align256(P * 64 * 64 * 8);           // Dinv
    b += align256((P + 1) * n * 8);           // row partials
    b += align256((n + 64) * 8);              // col sums + frob partials
    const size_t ldx = nt * (size_t)ns_tile;   // X0 (in the L buffer) also fits: ldx <= np + 64
    b += align256(ldx * ldx * (size_t)elem);  // X1
    b += align256(ldx * ldx * (size_t)elem);  // R
    b += align256((size_t)NOLSM_NVEC * n * 6 * 8 * nown);  // finishing vectors per owned molecule
    b += align256((size_t)max_iter * nt * nt * 8);  // residual partials
    if (inverse == NOLSM_INV_COUPLED_NS) b += 4 * align256(ldx * ldx * (size_t)elem);  // Y, Z ping-pong
    if (sym) b += align256(ldx * ldx * (size_t)elem);   // X0 beside L (kept to the end)
    if (inverse == NOLSM_INV_CHOLESKY_APPLY_FP32)         // FP32 copies of L and Dinv
        b += align256(n * n * 4) + align256(P * 64 * 64 * 4);
    return b;
}

static int validate(const nolsm_pattern *p, const char *name) {
    if (!p || !p->row_ptr || (p->nnzb > 0 && !p->col_idx) || p->nb < 1) {
        nolsm_set_last_error(std::string(name) + ": null or empty pattern");
        return NOLSM_E_ARG;
    }
    const int32_t nb = p->nb;
    if (p->row_ptr[0] != 0 || (int64_t)p->row_ptr[nb] != p->nnzb) {
        nolsm_set_last_error(std::string(name) + ": row_ptr limits");
        return NOLSM_E_PATTERN;
    }
    for (int32_t i = 0; i < nb; ++i) {
        const int32_t lo = p->row_ptr[i], hi = p->row_ptr[i + 1];
        if (hi < lo) { nolsm_set_last_error(std::string(name) + ": row_ptr not monotone"); return NOLSM_E_PATTERN; }
        bool diag = false;
        for (int32_t e = lo; e < hi; ++e) {
            const int32_t c = p->col_idx[e];
            if (c < 0 || c >= nb) { nolsm_set_last_error(std::string(name) + ": column out of range"); return NOLSM_E_PATTERN; }
            if (e > lo && c <= p->col_idx[e - 1]) { nolsm_set_last_error(std::string(name) + ": columns not strictly increasing"); return NOLSM_E_PATTERN; }
            if (c == i) diag = true;
        }
        if (!diag) { nolsm_set_last_error(std::string(name) + ": diagonal block missing"); return NOLSM_E_PATTERN; }
    }
    // symmetry: (i, c) stored => (c, i) stored (binary search in row c)
    for (int32_t i = 0; i < nb; ++i) {
        for (int32_t e = p->row_ptr[i]; e < p->row_ptr[i + 1]; ++e) {
            const int32_t c = p->col_idx[e];
            const int32_t *b = p->col_idx + p->row_ptr[c], *en = p->col_idx + p->row_ptr[c + 1];
            if (!std::binary_search(b, en, i)) {
                nolsm_set_last_error(std::string(name) + ": pattern not symmetric");
                return NOLSM_E_PATTERN;
            }
        }
    }
    return NOLSM_OK;
}

// Submatrix combination (Sec. III-B, Eq. combination_criterion), greedy:
// the valid pair with the fewest blocks added to one side is merged first
// (ties: larger cubic drop, then lower ids); stale queue entries are skipped
// by version. Candidates of group a are the groups owning a block of R_a
// (patterns are symmetric, so the relation is too).
namespace {
struct PairKey {
    int64_t add, neg_drop;
    int32_t a, b;
    uint32_t va, vb;
    bool operator>(const PairKey &o) const {
        if (add != o.add) return add > o.add;
        if (neg_drop != o.neg_drop) return neg_drop > o.neg_drop;
        if (a != o.a) return a > o.a;
        return b > o.b;
    }
};

static int64_t common_blocks(const std::vector<int32_t> &x, const std::vector<int32_t> &y) {
    int64_t c = 0;
    size_t i = 0, j = 0;
    while (i < x.size() && j < y.size()) {
        if (x[i] < y[j]) ++i;
        else if (y[j] < x[i]) ++j;
        else { ++c; ++i; ++j; }
    }
    return c;
}

static void combine_groups(nolsm_plan *pl, int32_t max_own) {
    const int32_t nb = pl->nb;
    std::vector<std::vector<int32_t>> rows(nb), owned(nb);
    std::vector<int32_t> owner(nb);
    std::vector<uint32_t> ver(nb, 0);
    std::vector<char> alive(nb, 1);
    for (int32_t J = 0; J < nb; ++J) {
        rows[J].assign(pl->sub_blk.begin() + pl->sub_ptr[J], pl->sub_blk.begin() + pl->sub_ptr[J + 1]);
        owned[J].assign(1, J);
        owner[J] = J;
    }
    std::priority_queue<PairKey, std::vector<PairKey>, std::greater<PairKey>> q;
    auto consider = [&](int32_t a, int32_t b) {   // a < b, both alive
        if ((int32_t)(owned[a].size() + owned[b].size()) > max_own) return;
        const int64_t mi = (int64_t)rows[a].size(), mj = (int64_t)rows[b].size();
        const int64_t mij = common_blocks(rows[a], rows[b]);
        const int64_t mu = mi + mj - mij;
        const int64_t drop = mi * mi * mi + mj * mj * mj - mu * mu * mu;
        if (drop <= 0) return;
        q.push(PairKey{std::min(mj - mij, mi - mij), -drop, a, b, ver[a], ver[b]});
    };
    std::vector<int32_t> cand;
    auto candidates = [&](int32_t a) {
        cand.clear();
        for (int32_t blk : rows[a]) {
            const int32_t g = owner[blk];
            if (g != a) cand.push_back(g);
        }
        std::sort(cand.begin(), cand.end());
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    };
    for (int32_t a = 0; a < nb; ++a) {
        candidates(a);
        for (int32_t b : cand)
            if (b > a) consider(a, b);
    }
    while (!q.empty()) {
        const PairKey k = q.top();
        q.pop();
        if (!alive[k.a] || !alive[k.b] || ver[k.a] != k.va || ver[k.b] != k.vb) continue;
        const int32_t a = k.a, b = k.b;
        std::vector<int32_t> u;
        u.reserve(rows[a].size() + rows[b].size());
        std::set_union(rows[a].begin(), rows[a].end(), rows[b].begin(), rows[b].end(), std::back_inserter(u));
        rows[a].swap(u);
        std::vector<int32_t>().swap(rows[b]);
        std::vector<int32_t> o;
        std::merge(owned[a].begin(), owned[a].end(), owned[b].begin(), owned[b].end(), std::back_inserter(o));
        owned[a].swap(o);
        for (int32_t J : owned[a]) owner[J] = a;
        std::vector<int32_t>().swap(owned[b]);
        alive[b] = 0;
        ++ver[a];
        candidates(a);
        for (int32_t c : cand) consider(std::min(a, c), std::max(a, c));
    }
    // groups ordered by their smallest molecule (= their id)
    pl->grp_ptr.assign(1, 0);
    pl->own_ptr.assign(1, 0);
    pl->grp_blk.clear();
    pl->own_J.clear();
    for (int32_t g = 0; g < nb; ++g) {
        if (!alive[g]) continue;
        pl->grp_blk.insert(pl->grp_blk.end(), rows[g].begin(), rows[g].end());
        pl->grp_ptr.push_back((int32_t)pl->grp_blk.size());
        pl->own_J.insert(pl->own_J.end(), owned[g].begin(), owned[g].end());
        pl->own_ptr.push_back((int32_t)pl->own_J.size());
    }
}
}  // namespace

// Positions of owned molecules and of their N(J) rows inside their groups,
// and the group size statistics.
static void finish_groups(nolsm_plan *pl) {
    const int32_t ng = (int32_t)pl->grp_ptr.size() - 1;
    pl->own_pos.assign(pl->own_J.size(), -1);
    pl->rowpos.assign(pl->sub_blk.size(), -1);
    pl->g_m_max = 0;
    pl->sum_gn3 = 0.0;
    for (int32_t g = 0; g < ng; ++g) {
        const int32_t *lb = pl->grp_blk.data() + pl->grp_ptr[g], *le = pl->grp_blk.data() + pl->grp_ptr[g + 1];
        const int32_t m = (int32_t)(le - lb);
        pl->g_m_max = std::max(pl->g_m_max, m);
        const double n = (double)m * pl->bs;
        pl->sum_gn3 += n * n * n;
        for (int32_t o = pl->own_ptr[g]; o < pl->own_ptr[g + 1]; ++o) {
            const int32_t J = pl->own_J[o];
            pl->own_pos[o] = (int32_t)(std::lower_bound(lb, le, J) - lb);
            for (int32_t e = pl->sub_ptr[J]; e < pl->sub_ptr[J + 1]; ++e)
                pl->rowpos[e] = (int32_t)(std::lower_bound(lb, le, pl->sub_blk[e]) - lb);
        }
    }
}

extern "C" int nolsm_build_submatrices(const nolsm_pattern *K, const nolsm_pattern *S,
                                       int32_t flags, nolsm_plan **out) {
    if (!out) { nolsm_set_last_error("plan out-pointer is null"); return NOLSM_E_ARG; }
    if (flags & ~NOLSM_PLAN_COMBINE) { nolsm_set_last_error("unknown plan flag"); return NOLSM_E_ARG; }
    *out = nullptr;
    if (!K || !S) { nolsm_set_last_error("null pattern"); return NOLSM_E_ARG; }
    if (K->nb != S->nb || K->bs != S->bs) { nolsm_set_last_error("K and S disagree on nb/bs"); return NOLSM_E_ARG; }
    if (K->bs < 1 || K->bs > 6) { nolsm_set_last_error("bs must be 1..6"); return NOLSM_E_ARG; }
    int rc = validate(K, "K");
    if (rc) return rc;
    rc = validate(S, "S");
    if (rc) return rc;
    nolsm_plan *pl = new (std::nothrow) nolsm_plan();
    if (!pl) return NOLSM_E_NOMEM;
    try {
        const int32_t nb = K->nb;
        pl->nb = nb;
        pl->bs = K->bs;
        pl->Krp.assign(K->row_ptr, K->row_ptr + nb + 1);
        pl->Kci.assign(K->col_idx, K->col_idx + K->nnzb);
        pl->Srp.assign(S->row_ptr, S->row_ptr + nb + 1);
        pl->Sci.assign(S->col_idx, S->col_idx + S->nnzb);
        // merged pattern: row J of pat(K) u pat(S), sorted (set union of two
        // sorted lists)
        pl->sub_ptr.assign(nb + 1, 0);
        pl->sub_blk.reserve((size_t)std::max<int64_t>(K->nnzb, S->nnzb));
        pl->self_pos.assign(nb, -1);
        for (int32_t J = 0; J < nb; ++J) {
            const int32_t *a = K->col_idx + K->row_ptr[J], *ae = K->col_idx + K->row_ptr[J + 1];
            const int32_t *b = S->col_idx + S->row_ptr[J], *be = S->col_idx + S->row_ptr[J + 1];
            const size_t start = pl->sub_blk.size();
            std::set_union(a, ae, b, be, std::back_inserter(pl->sub_blk));
            pl->sub_ptr[J + 1] = (int32_t)pl->sub_blk.size();
            const int32_t *lb = pl->sub_blk.data() + start, *le = pl->sub_blk.data() + pl->sub_blk.size();
            pl->self_pos[J] = (int32_t)(std::lower_bound(lb, le, J) - lb);
        }
        // D keeps the merged pattern: D_row_ptr = sub_ptr, D_col_idx = sub_blk
        // (P is symmetric). scatter_pos: block (N(J)_a, J) lives in row
        // I = N(J)_a at the position of J in N(I).
        const size_t sum_m = pl->sub_blk.size();
        pl->scatter_pos.assign(sum_m, -1);
        pl->m_min = 1 << 30;
        pl->m_max = 0;
        pl->sum_n3 = 0.0;
        for (int32_t J = 0; J < nb; ++J) {
            const int32_t m = pl->sub_ptr[J + 1] - pl->sub_ptr[J];
            pl->m_min = std::min(pl->m_min, m);
            pl->m_max = std::max(pl->m_max, m);
            const double n = (double)m * pl->bs;
            pl->sum_n3 += n * n * n;
            for (int32_t a = 0; a < m; ++a) {
                const int32_t I = pl->sub_blk[pl->sub_ptr[J] + a];
                const int32_t *lb = pl->sub_blk.data() + pl->sub_ptr[I];
                const int32_t *le = pl->sub_blk.data() + pl->sub_ptr[I + 1];
                const int32_t *q = std::lower_bound(lb, le, J);
                pl->scatter_pos[pl->sub_ptr[J] + a] = (int32_t)(q - pl->sub_blk.data());
            }
        }
        if (flags & NOLSM_PLAN_COMBINE) {
            combine_groups(pl, 64 / pl->bs);
        } else {
            pl->grp_ptr = pl->sub_ptr;
            pl->grp_blk = pl->sub_blk;
            pl->own_ptr.resize(nb + 1);
            pl->own_J.resize(nb);
            for (int32_t J = 0; J <= nb; ++J) pl->own_ptr[J] = J;
            for (int32_t J = 0; J < nb; ++J) pl->own_J[J] = J;
        }
        finish_groups(pl);
    } catch (...) {
        delete pl;
        return NOLSM_E_NOMEM;
    }
    *out = pl;
    return NOLSM_OK;
}

extern "C" void nolsm_default_opts(nolsm_solve_opts *o, int32_t prec) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->prec = prec;
    o->n_final_fp32 = (prec == NOLSM_FP16 || prec == NOLSM_BF16) ? 2 : 0;
    // FP16/BF16: negative = the switch point derived from the precision and
    // the finishing iterations at configure time (nolsm_switch_tol)
    o->tol = (prec == NOLSM_FP64) ? 1e-10 : (prec == NOLSM_FP32 ? 1e-5 : -1.0);
    o->max_iter = (prec == NOLSM_FP64) ? 48 : 40;
    o->fixed_iters = 0;
    o->switch_theta = 0.7;
    o->switch_rmax = 0.5;
    o->bounds = NOLSM_BOUNDS_GERSHGORIN;
    o->mlp_safety = 1.05f;
    o->sched = NOLSM_SCHED_GRAPH;
    o->debug_poison_mol = -1;
    o->ns_small_tile_mask = 0x5;   // 64 and 192 rows: 128-row tiles would waste work
    o->inverse = NOLSM_INV_CHOLESKY;
    o->inv_max_iter = 40;
    o->sym_sign = 0;
    o->finish_rows = 0;
    o->debug_force_stall = -1;
    o->subst_fp32 = 0;
}

extern "C" int nolsm_plan_info(const nolsm_plan *p, nolsm_plan_sizes *o) {
    if (!p || !o) return NOLSM_E_ARG;
    std::memset(o, 0, sizeof(*o));
    o->nb = p->nb;
    o->bs = p->bs;
    o->sum_m = (int64_t)p->sub_blk.size();
    o->m_min = p->m_min;
    o->m_max = p->m_max;
    o->sum_n3 = p->sum_n3;
    if (p->configured) {
        o->nchunks = (int32_t)p->chunks.size();
        o->meta_bytes = p->image.size();
        o->ws_min_bytes = p->ws_min;
        o->ws_full_bytes = p->ws_full;
    }
    o->ngroups = (int32_t)p->grp_ptr.size() - 1;
    o->g_m_max = p->g_m_max;
    o->sum_gm = (int64_t)p->grp_blk.size();
    o->sum_gn3 = p->sum_gn3;
    return NOLSM_OK;
}

extern "C" int nolsm_plan_groups(const nolsm_plan *p, int32_t *grp_ptr, int32_t *grp_blk, int32_t *own_ptr,
                                 int32_t *own_J) {
    if (!p) return NOLSM_E_ARG;
    if (grp_ptr) std::memcpy(grp_ptr, p->grp_ptr.data(), p->grp_ptr.size() * 4);
    if (grp_blk) std::memcpy(grp_blk, p->grp_blk.data(), p->grp_blk.size() * 4);
    if (own_ptr) std::memcpy(own_ptr, p->own_ptr.data(), p->own_ptr.size() * 4);
    if (own_J) std::memcpy(own_J, p->own_J.data(), p->own_J.size() * 4);
    return NOLSM_OK;
}

extern "C" int nolsm_plan_export(const nolsm_plan *p, int32_t *sub_ptr, int32_t *sub_blk,
                                 int32_t *self_pos, int32_t *D_row_ptr, int32_t *D_col_idx,
                                 int32_t *scatter_pos) {
    if (!p) return NOLSM_E_ARG;
    const size_t nb = (size_t)p->nb, sm = p->sub_blk.size();
    if (sub_ptr) std::memcpy(sub_ptr, p->sub_ptr.data(), (nb + 1) * 4);
    if (sub_blk) std::memcpy(sub_blk, p->sub_blk.data(), sm * 4);
    if (self_pos) std::memcpy(self_pos, p->self_pos.data(), nb * 4);
    if (D_row_ptr) std::memcpy(D_row_ptr, p->sub_ptr.data(), (nb + 1) * 4);
    if (D_col_idx) std::memcpy(D_col_idx, p->sub_blk.data(), sm * 4);
    if (scatter_pos) std::memcpy(scatter_pos, p->scatter_pos.data(), sm * 4);
    return NOLSM_OK;
}

// Append a task list padded to a multiple of 8: kernels remap workgroup b to
// list entry (b % 8) * (G / 8) + b / 8, so that consecutive entries (the
// tiles of one submatrix) run on the same XCD and share its L2.
static void pad8(std::vector<uint32_t> &v) {
    while (v.size() % 8) v.push_back(NOLSM_TASK_NONE);
    if (v.empty()) for (int i = 0; i < 8; ++i) v.push_back(NOLSM_TASK_NONE);
}

template <class T>
static size_t put(std::vector<char> &img, const T *src, size_t count) {
    const size_t off = align256(img.size());
    img.resize(off + count * sizeof(T));
    if (count) std::memcpy(img.data() + off, src, count * sizeof(T));
    return off;
}

extern "C" int nolsm_plan_configure(nolsm_plan *pl, const nolsm_solve_opts *opts,
                                    size_t ws_bytes, size_t *meta_bytes) {
    if (!pl || !opts) { nolsm_set_last_error("configure: null argument"); return NOLSM_E_ARG; }
    if (opts->prec < NOLSM_FP64 || opts->prec > NOLSM_BF16) { nolsm_set_last_error("bad precision"); return NOLSM_E_ARG; }
    if (opts->max_iter < 2 || opts->max_iter > NOLSM_MAX_ITER_CAP) { nolsm_set_last_error("max_iter must be 2..128"); return NOLSM_E_ARG; }
    if (opts->sched < NOLSM_SCHED_GRAPH || opts->sched > NOLSM_SCHED_PIPELINE) { nolsm_set_last_error("bad schedule"); return NOLSM_E_ARG; }
    if (opts->inverse < NOLSM_INV_CHOLESKY || opts->inverse > NOLSM_INV_CHOLESKY_APPLY_FP32) { nolsm_set_last_error("bad inverse"); return NOLSM_E_ARG; }
    if ((opts->inverse == NOLSM_INV_CHOLESKY_FP32 || opts->inverse == NOLSM_INV_CHOLESKY_APPLY_FP32) &&
        opts->prec != NOLSM_FP16 && opts->prec != NOLSM_BF16) {
        nolsm_set_last_error("the FP32 Cholesky routes serve the FP16/BF16 sign iterations only");
        return NOLSM_E_ARG;
    }
    if (opts->sym_sign && ((opts->prec != NOLSM_FP16 && opts->prec != NOLSM_BF16) ||
                           opts->inverse == NOLSM_INV_COUPLED_NS)) {
        nolsm_set_last_error("the symmetric sign iteration needs FP16/BF16 and a Cholesky route");
        return NOLSM_E_ARG;
    }
    if (opts->inverse == NOLSM_INV_COUPLED_NS) {
        if (opts->prec != NOLSM_FP16 && opts->prec != NOLSM_BF16) {
            nolsm_set_last_error("the coupled Newton-Schulz inverse runs in FP16/BF16 only");
            return NOLSM_E_ARG;
        }
        if (opts->inv_max_iter < 2 || opts->inv_max_iter > NOLSM_MAX_ITER_CAP) {
            nolsm_set_last_error("inv_max_iter must be 2..128");
            return NOLSM_E_ARG;
        }
    }
    try {
        pl->configured = false;
        pl->bound = false;
        pl->chunks.clear();
        pl->prec = opts->prec;
        pl->sched = opts->sched;
        pl->max_iter = opts->max_iter;
        pl->inverse = opts->inverse;
        pl->sym = opts->sym_sign ? 1 : 0;
        pl->inv_max_iter = opts->inverse == NOLSM_INV_COUPLED_NS ? opts->inv_max_iter : 0;
        // residual partial slots serve both iterations, one after the other
        const int32_t res_slots = std::max(pl->max_iter, pl->inv_max_iter);
        pl->elem = nolsm_elem_for(opts->prec);
        // slots are submatrices: groups of molecules (one per molecule
        // unless the plan was built with NOLSM_PLAN_COMBINE)
        const int32_t bs = pl->bs, ng = (int32_t)pl->grp_ptr.size() - 1;
        auto np_of = [&](int32_t g) {
            const int32_t n = bs * (pl->grp_ptr[g + 1] - pl->grp_ptr[g]);
            return (n + NOLSM_TILE - 1) / NOLSM_TILE * NOLSM_TILE;
        };
        const uint64_t mask = opts->ns_small_tile_mask;
        auto tile_of = [&](int32_t J) { return nolsm_ns_tile_for(opts->prec, np_of(J), mask); };
        if ((size_t)pl->g_m_max * bs > NOLSM_MAX_ROWS) {
            nolsm_set_last_error("submatrices above " + std::to_string(NOLSM_MAX_ROWS) + " rows are not supported");
            return NOLSM_E_ARG;
        }
        // order: decreasing np (largest-first keeps the tail short), then J
        std::vector<int32_t> order(ng);
        for (int32_t g = 0; g < ng; ++g) order[g] = g;
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return np_of(a) > np_of(b); });
        const size_t ctl_bytes =
            align256(sizeof(SubCtl)) + (pl->inverse == NOLSM_INV_COUPLED_NS ? align256(sizeof(InvCtl)) : 0);
        // queue counters of the persistent launches, per chunk
        const size_t nqueue = (size_t)pl->max_iter * 2 * 2 * 8;
        const size_t qbytes = align256(nqueue * sizeof(int32_t));
        pl->ws_min = 0;
        pl->ws_full = 0;
        auto slot_bytes = [&](int32_t g) {
            return nolsm_slot_bytes(np_of(g), tile_of(g), pl->elem, res_slots, pl->inverse,
                                    pl->own_ptr[g + 1] - pl->own_ptr[g], pl->sym) + ctl_bytes;
        };
        for (int32_t J = 0; J < ng; ++J) {
            const size_t sb = slot_bytes(J);
            pl->ws_min = std::max(pl->ws_min, sb);
            pl->ws_full += sb;
        }
        pl->ws_full += 256 + qbytes;
        // the pipeline schedule keeps two chunks resident: half the
        // workspace each
        const bool pipe = pl->sched == NOLSM_SCHED_PIPELINE;
        const size_t region = pipe ? (ws_bytes / 2) & ~(size_t)255 : ws_bytes;
        if (region < pl->ws_min + 256 + qbytes) {
            nolsm_set_last_error("workspace smaller than the largest submatrix needs");
            return NOLSM_E_WORKSPACE;
        }
        pl->ws_bytes = ws_bytes;
        // greedy chunks in decreasing size. The per-bucket schedule also cuts
        // at bucket changes (buckets of 64 rows, i.e. equal np); the others
        // cut where np falls below 4/5 of the chunk's largest, because the
        // serial setup launches (Cholesky panels, right-solve row blocks) of
        // a chunk run to the depth of its largest submatrix while smaller
        // ones idle
        size_t i = 0;
        while (i < order.size()) {
            HostChunk ch;
            size_t used = 0;
            std::vector<int32_t> js;
            const int32_t bucket = np_of(order[i]);
            while (i < order.size() && js.size() < 65535) {
                const int32_t J = order[i];
                if (pl->sched == NOLSM_SCHED_PER_BUCKET && np_of(J) != bucket) break;
                if (pl->sched != NOLSM_SCHED_PER_BUCKET && 5 * np_of(J) < 4 * bucket) break;
                const size_t sb = slot_bytes(J);
                if (used + sb + 256 + qbytes > region) break;
                used += sb;
                js.push_back(J);
                ++i;
            }
            // layout: SubCtl array first, then the slots
            // layout: workspace header, SubCtl array, InvCtl array (coupled
            // inverse only), queue counters, slots
            ch.off_ctl = NOLSM_WS_HEADER;
            ch.off_ictl = 0;
            ch.off_q = NOLSM_WS_HEADER + align256(js.size() * sizeof(SubCtl));
            if (pl->inverse == NOLSM_INV_COUPLED_NS) {
                ch.off_ictl = ch.off_q;
                ch.off_q += align256(js.size() * sizeof(InvCtl));
            }
            size_t off = ch.off_q + qbytes;
            for (size_t s = 0; s < js.size(); ++s) {
                const int32_t g = js[s];
                SubMeta m;
                std::memset(&m, 0, sizeof(m));
                m.J = pl->own_J[pl->own_ptr[g]];
                m.m = pl->grp_ptr[g + 1] - pl->grp_ptr[g];
                m.n = bs * m.m;
                m.np = np_of(g);
                m.p = pl->own_pos[pl->own_ptr[g]];
                m.P = m.np / NOLSM_TILE;
                m.sub_off = pl->grp_ptr[g];
                m.own_off = pl->own_ptr[g];
                m.nown = pl->own_ptr[g + 1] - pl->own_ptr[g];
                m.pmin = m.p;
                for (int32_t o = pl->own_ptr[g]; o < pl->own_ptr[g + 1]; ++o)
                    m.pmin = std::min(m.pmin, pl->own_pos[o]);
                const int32_t T = tile_of(g);
                const int32_t nt = (m.np + T - 1) / T;
                m.ntile_ns = nt * nt;
                const size_t n = (size_t)m.np;
                m.offL = (int64_t)off; off += align256(n * n * 8);
                m.kf32 = (pl->inverse == NOLSM_INV_CHOLESKY_FP32 || pl->inverse == NOLSM_INV_CHOLESKY_APPLY_FP32) ? 1 : 0;
                m.pad_ = 0;
                m.offK = (int64_t)off; off += align256(n * (n + 64) * (m.kf32 ? 4 : 8));
                m.offDinv = (int64_t)off; off += align256((size_t)m.P * 4096 * 8);
                m.offRow = (int64_t)off; off += align256((size_t)(m.P + 1) * n * 8);
                m.offCol = (int64_t)off; off += align256((n + 64) * 8);
                m.ldx = nt * T;
                const size_t ldx = (size_t)m.ldx;
                m.offX1 = (int64_t)off; off += align256(ldx * ldx * pl->elem);
                m.offB = (int64_t)off; off += align256(ldx * ldx * pl->elem);
                m.offVec = (int64_t)off; off += align256((size_t)NOLSM_NVEC * n * 6 * 8 * m.nown);
                m.offX0 = m.offL;
                if (pl->sym) { m.offX0 = (int64_t)off; off += align256(ldx * ldx * pl->elem); }
                m.offRes = (int64_t)off; off += align256((size_t)res_slots * m.ntile_ns * 8);
                if (pl->inverse == NOLSM_INV_COUPLED_NS) {
                    m.offY0 = (int64_t)off; off += align256(ldx * ldx * pl->elem);
                    m.offY1 = (int64_t)off; off += align256(ldx * ldx * pl->elem);
                    m.offZ0 = (int64_t)off; off += align256(ldx * ldx * pl->elem);
                    m.offZ1 = (int64_t)off; off += align256(ldx * ldx * pl->elem);
                }
                if (pl->inverse == NOLSM_INV_CHOLESKY_APPLY_FP32) {
                    m.offL32 = (int64_t)off; off += align256(n * n * 4);
                    m.offDinv32 = (int64_t)off; off += align256((size_t)m.P * 4096 * 4);
                }
                ch.meta.push_back(m);
                ch.max_m = std::max(ch.max_m, m.m);
                ch.max_np = std::max(ch.max_np, m.np);
                ch.max_own = std::max(ch.max_own, m.nown);
                for (int32_t c = 0; c <= m.P; ++c) ch.t_subst.push_back(NOLSM_TASK(s, c, 0));
                // X_0 tiles: the symmetric route converts the upper ones (each
                // also writes its mirror)
                for (int32_t a = 0; a < m.P; ++a)
                    for (int32_t b = pl->sym ? a : 0; b < m.P; ++b) ch.t_conv.push_back(NOLSM_TASK(s, a, b));
                // FP16/BF16 slots with 64-row tiles get their own list
                std::vector<uint32_t> &tl =
                    (T == 64 && (pl->prec == NOLSM_FP16 || pl->prec == NOLSM_BF16)) ? ch.t_ns64 : ch.t_ns;
                // symmetric route: upper tiles only, each mirrors itself
                const bool sym = pl->sym != 0;
                for (int32_t a = 0; a < nt; ++a)
                    for (int32_t b = sym ? a : 0; b < nt; ++b) tl.push_back(NOLSM_TASK(s, a, b));
                // (slot, 256-row block, owned molecule): the molecules of one row
                // block are adjacent, so they run together on one XCD and share
                // the streamed rows through its L2
                for (int32_t a = 0; a < (m.P + 3) / 4; ++a)
                    for (int32_t o = 0; o < m.nown; ++o) ch.t_rows.push_back(NOLSM_TASK(s, a, o));
            }
            ch.ws_used = off;
            ch.n_ns_real = ch.t_ns.size();
            ch.n_ns64_real = ch.t_ns64.size();
            pad8(ch.t_subst);
            pad8(ch.t_conv);
            pad8(ch.t_ns);
            pad8(ch.t_ns64);
            pad8(ch.t_rows);
            ch.base = (pipe && (pl->chunks.size() & 1)) ? region : 0;
            pl->chunks.push_back(std::move(ch));
        }
        // metadata image
        pl->image.clear();
        pl->o_Krp = put(pl->image, pl->Krp.data(), pl->Krp.size());
        pl->o_Kci = put(pl->image, pl->Kci.data(), pl->Kci.size());
        pl->o_Srp = put(pl->image, pl->Srp.data(), pl->Srp.size());
        pl->o_Sci = put(pl->image, pl->Sci.data(), pl->Sci.size());
        pl->o_sub_ptr = put(pl->image, pl->sub_ptr.data(), pl->sub_ptr.size());
        pl->o_sub_blk = put(pl->image, pl->sub_blk.data(), pl->sub_blk.size());
        pl->o_self = put(pl->image, pl->self_pos.data(), pl->self_pos.size());
        pl->o_scatter = put(pl->image, pl->scatter_pos.data(), pl->scatter_pos.size());
        pl->o_grp_blk = put(pl->image, pl->grp_blk.data(), pl->grp_blk.size());
        pl->o_own_J = put(pl->image, pl->own_J.data(), pl->own_J.size());
        pl->o_own_pos = put(pl->image, pl->own_pos.data(), pl->own_pos.size());
        pl->o_rowpos = put(pl->image, pl->rowpos.data(), pl->rowpos.size());
        for (auto &ch : pl->chunks) {
            ch.o_meta = put(pl->image, ch.meta.data(), ch.meta.size());
            ch.o_subst = put(pl->image, ch.t_subst.data(), ch.t_subst.size());
            ch.o_conv = put(pl->image, ch.t_conv.data(), ch.t_conv.size());
            ch.o_ns = put(pl->image, ch.t_ns.data(), ch.t_ns.size());
            ch.o_ns64 = put(pl->image, ch.t_ns64.data(), ch.t_ns64.size());
            ch.o_rows = put(pl->image, ch.t_rows.data(), ch.t_rows.size());
        }
        pl->image.resize(align256(pl->image.size()));
        pl->configured = true;
        if (meta_bytes) *meta_bytes = pl->image.size();
    } catch (...) {
        return NOLSM_E_NOMEM;
    }
    return NOLSM_OK;
}

extern "C" const char *nolsm_strerror(int code) {
    static thread_local std::string msg;
    const char *base = "unknown error";
    switch (code) {
        case NOLSM_OK: base = "ok"; break;
        case NOLSM_E_ARG: base = "invalid argument"; break;
        case NOLSM_E_PATTERN: base = "invalid block pattern"; break;
        case NOLSM_E_WORKSPACE: base = "workspace or metadata buffer too small"; break;
        case NOLSM_E_HIP: base = "HIP runtime error"; break;
        case NOLSM_E_STATE: base = "plan not configured/bound for these options"; break;
        case NOLSM_E_NOT_SPD: base = "a submatrix of S is not positive definite"; break;
        case NOLSM_E_NOCONV: base = "a sign iteration did not converge"; break;
        case NOLSM_E_NOMEM: base = "host allocation failed"; break;
    }
    msg = base;
    if (!g_last_error.empty()) msg += std::string(": ") + g_last_error;
    return msg.c_str();
}
