// Setup of every submatrix: gather, Cholesky, substitution, bounds, X_0.
//
// Sec. III-B.2 (NOLSM generation step and Eq. purification_submatrix): the
// submatrices T_J(K), T_J(S) are dense on the index list N(J); the sign
// iteration acts on A_J = T_J(S)^-1 T_J(K) - mu I, and the owned columns of
// T_J(D) need Y_J = T_J(S)^-1 E_cJ. Here T_J(S)^-1 is applied through an FP64
// Cholesky factor (the paper's inverse is iterative; the FP64 factorisation
// is this library's choice, for accuracy at these sizes), with FP64 or, on
// the 16-bit routes that ask for it, FP32 arithmetic in the substitutions
// (on the symmetric route by default as split FP16 products, split16.h);
// the K buffer (K, then W, then A or A~ and Y) is stored in the type of that
// arithmetic.
#include "dev_common.h"
#include "kernels.h"
#include "split16.h"

// ---------------------------------------------------------------------------
// Gather (Sec. III-B.2, submatrix construction): block row a of T_J(K) and
// T_J(S) from the block-CSR rows of N(J)_a, absent blocks as zeros. The K
// buffer gets 64 extra columns holding E_cJ (identity on the molecule's own
// bs rows), which the substitution turns into Y_J. Padding rows/columns
// n..np-1: S = I, K = 0.
// One workgroup per (block row a, submatrix). Each stored block (I, C) of
// row I = N(J)_a is located in N(J) by one binary search, giving the inverse
// map pos[b] = CSR entry of block column N(J)_b (or -1); the 6 x np stripes
// are then written straight to HBM, coalesced along the row.
// grid (max_m, nsub), 256 threads; dynamic LDS: 3 m ints.
// ---------------------------------------------------------------------------
#define GATHER_BSMAX 6   // largest block size (the plan refuses larger)
__global__ __launch_bounds__(256) void k_gather(ChunkDev cd, char *ws, GatherArgs ga) {
    extern __shared__ int gsm[];
    const int s = blockIdx.y, a = blockIdx.x;
    if (s >= cd.nsub) return;
    const SubMeta M = cd.meta[s];
    if (a >= M.m) return;
    const int bs = ga.bs, np = M.np, n = M.n, m = M.m, t = threadIdx.x;
    int *list = gsm;                 // N(J)
    int *posK = gsm + cd.max_m;      // block column b -> CSR entry in K's row I, or -1
    int *posS = gsm + 2 * cd.max_m;  // the same for S
    const int *nlist = ga.grp_blk + M.sub_off;
    for (int i = t; i < m; i += 256) {
        list[i] = nlist[i];
        posK[i] = -1;
        posS[i] = -1;
    }
    const int I = nlist[a];   // from global memory: `list` is complete only after the barrier
    __syncthreads();
    for (int which = 0; which < 2; ++which) {
        const int *rp = which ? ga.Srp : ga.Krp;
        const int *ci = which ? ga.Sci : ga.Kci;
        int *pos = which ? posS : posK;
        const int lo = rp[I], hi = rp[I + 1];
        for (int e = lo + t; e < hi; e += 256) {
            const int C = ci[e];
            int l = 0, h = m - 1;
            while (l <= h) {
                const int mid = (l + h) >> 1;
                const int v = list[mid];
                if (v == C) { pos[mid] = e; break; }
                if (v < C) l = mid + 1; else h = mid - 1;
            }
        }
    }
    __syncthreads();
    double *Kd = (double *)(ws + M.offK);   // T_J(K) in FP64, or
    float *Kf = (float *)(ws + M.offK);     // in FP32 when the substitution runs in FP32
    auto put_k = [&](int64_t idx, double v) {
        if (M.kf32) Kf[idx] = (float)v;
        else Kd[idx] = v;
    };
    double *Sd = (double *)(ws + M.offL);   // T_J(S) in FP64, or
    float *Sf = (float *)(ws + M.offL);     // in FP32 for the FP32 Cholesky route
    auto put_s = [&](int64_t idx, double v) {
        if (ga.s_fp32) Sf[idx] = (float)v;
        else Sd[idx] = v;
    };
    const int64_t ldk = np + 64, lds = np;
    const int bb = bs * bs;
    // debug: a negative pivot in the submatrix that owns poison_J
    bool poison = false;
    for (int o = 0; o < M.nown; ++o)
        poison |= (a == 0 && ga.own_J[M.own_off + o] == ga.poison_J);
    // thread t takes columns t, t + 256, ..: the block column and the CSR
    // entries are found once per column, then its bs rows follow
    double kmx = 0.0;   // largest |K| entry this thread stores
    for (int c = t; c < np; c += 256) {
        int ek = -1, es = -1, cc = 0;
        if (c < n) {
            const int b = c / bs;
            cc = c - b * bs;
            ek = posK[b];
            es = posS[b];
        }
        const int tc = c >> 6;
        // all loads of the column first (the stores below may not move above
        // them), then the stores; 64-tile row and column of each entry: the
        // tiles that nothing downstream reads are not written
        double vk[GATHER_BSMAX], vs[GATHER_BSMAX];
#pragma unroll
        for (int r = 0; r < GATHER_BSMAX; ++r) {
            vk[r] = vs[r] = 0.0;
            if (r < bs) {
                const int tr = (a * bs + r) >> 6;
                const bool wk = !ga.k_upper || tc >= tr, ws_ = !ga.s_lower || tc <= tr;
                if (wk && ek >= 0) vk[r] = ga.Kval[(int64_t)ek * bb + r * bs + cc];
                if (ws_ && es >= 0) vs[r] = ga.Sval[(int64_t)es * bb + r * bs + cc];
            }
        }
        if (poison && c == 0) vs[0] = -1.0;
#pragma unroll
        for (int r = 0; r < GATHER_BSMAX; ++r) kmx = fmax(kmx, fabs(vk[r]));
#pragma unroll
        for (int r = 0; r < GATHER_BSMAX; ++r) {
            if (r < bs) {
                const int tr = (a * bs + r) >> 6;
                const bool wk = !ga.k_upper || tc >= tr, ws_ = !ga.s_lower || tc <= tr;
                if (wk) put_k((int64_t)(a * bs + r) * ldk + c, vk[r]);
                if (ws_) put_s((int64_t)(a * bs + r) * lds + c, vs[r]);
            }
        }
    }
    // max |T_J(K)| over the submatrix, as FP32 bits (non-negative floats
    // order like their bit patterns): one atomic per wave
    {
        float v = (float)kmx;
        for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
        if ((t & 63) == 0) atomicMax(&cd.ctl[s].kmax, __float_as_uint(v));
    }
    // E tile: columns np..np+63 of the K buffer; owned molecule o (block
    // position q_o in the rows) has its unit columns at o bs .. o bs + bs - 1
    int own_here = -1;
    for (int o = 0; o < M.nown; ++o)
        if (ga.own_pos[M.own_off + o] == a) own_here = o;
    for (int i = t; i < bs * 64; i += 256) {
        const int r = i / 64, c = i % 64;
        put_k((int64_t)(a * bs + r) * ldk + np + c, (own_here >= 0 && c == own_here * bs + r) ? 1.0 : 0.0);
    }
    // padding rows (one workgroup per submatrix does it)
    if (a == 0 && np > n) {
        const int rows = np - n;
        for (int i = t; i < rows * np; i += 256) {
            const int r = n + i / np, c = i % np;
            put_s((int64_t)r * np + c, (r == c) ? 1.0 : 0.0);
        }
        for (int i = t; i < rows * (np + 64); i += 256) {
            const int r = n + i / (np + 64), c = i % (np + 64);
            put_k((int64_t)r * (np + 64) + c, 0.0);
        }
    }
}

// ---------------------------------------------------------------------------
// Cholesky S_J = L L^T, left-looking by 64-column panels: per panel, one
// launch factors and inverts the diagonal tiles (one workgroup per
// submatrix) and one launch forms the tiles below them in parallel. The
// inverses of the diagonal tiles are kept (the substitution applies them as
// GEMMs). A non-positive pivot marks the molecule NOT_SPD.
// ---------------------------------------------------------------------------
// Cholesky of the 64x64 diagonal tile in LDS (lower part read), right-looking
// by columns with the entries in registers: thread t holds column q = t % 64,
// rows r = w + 4i (w = t / 64, i = 0..15). After step c the owners of column
// c + 1 publish it (updated through step c) in cb[(c + 1) % 2], so one
// barrier per column suffices: a buffer is rewritten only after every thread
// has passed the barrier that follows its last read. The factor L (zeros
// above the diagonal) is written back to D. A non-positive pivot sets *fail.
template <typename T> __device__ void potrf64_reg(T (*D)[LDP], T (*cb)[64], int *fail) {
    // w in a scalar register: the row tests below are branches, not masks
    const int t = threadIdx.x, q = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);
    T v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = D[w + 4 * i][q];
    if (q == 0)
#pragma unroll
        for (int i = 0; i < 16; ++i) cb[0][w + 4 * i] = v[i];
    __syncthreads();
    for (int c = 0; c < 64; ++c) {
        const T *col = cb[c & 1];
        const T d = col[c];
        if (t == 0 && !(d > (T)0)) *fail = 1;
        const T piv = sqrt(fmax(d, (T)(sizeof(T) == 8 ? 1e-300 : 1e-30)));
        const T rp = (T)1 / piv;
        const T lq = col[q] * rp;   // L[q][c] for q > c
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int r = w + 4 * i;
            if (r < c) continue;   // finished rows; r is uniform in a wave: no divergence
            const T lr = col[r] * rp;
            if (q == c) {
                if (r > c) v[i] = lr;
                else v[i] = piv;
            } else if (q > c && r >= q) {
                v[i] -= lr * lq;
            }
        }
        if (q == c + 1)
#pragma unroll
            for (int i = 0; i < 16; ++i) cb[(c + 1) & 1][w + 4 * i] = v[i];
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int r = w + 4 * i;
        D[r][q] = (q <= r) ? v[i] : (T)0;
    }
    __syncthreads();
}

// Di = L^-1 for the lower-triangular 64x64 L in LDS: forward substitution
// against the identity, all 64 columns at once, by pivot rows q. Thread t
// holds column c = t % 64, rows r = w + 4i of the right-hand side B; at step q
// the owners of row q scale it by 1/L[q][q] (final row q of Di) and publish
// it, then every row r > q takes off L[r][q] times it. Entries above the
// diagonal stay exact zeros. The result goes straight from registers to the
// global 64x64 row-major Dg (row r of a wave's lanes is 512 contiguous
// bytes). rd: 64 values of LDS, xb: 2 x 64.
template <typename T> __device__ void trinv64_reg(const T (*Lt)[LDP], T *Dg, T *rd, T (*xb)[64], float *Df = nullptr) {
    const int t = threadIdx.x, c = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);
    if (t < 64) rd[t] = (T)1 / Lt[t][t];
    T b[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) b[i] = (w + 4 * i == c) ? (T)1 : (T)0;
    __syncthreads();
    for (int q = 0; q < 64; ++q) {
        const int iq = q >> 2;
        if (w == (q & 3)) {
            const T s = rd[q];
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (i == iq) {
                    b[i] *= s;
                    xb[q & 1][c] = b[i];
                }
        }
        __syncthreads();
        const T xq = xb[q & 1][c];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int r = w + 4 * i;   // uniform in a wave: rows above q are skipped without divergence
            if (r > q) b[i] -= Lt[r][q] * xq;
        }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) Dg[(w + 4 * i) * 64 + c] = b[i];
    if (Df)
#pragma unroll
        for (int i = 0; i < 16; ++i) Df[(w + 4 * i) * 64 + c] = (float)b[i];
}

// FP64 Cholesky and inverse of the 64x64 tile in LDS by 16x16 blocks,
// right-looking. For block column b: wave 0 factors the diagonal block and
// inverts it in registers (M_b = L_bb^-1; a chain of 16 steps whose
// exchanges are lane shuffles, with no workgroup barrier); the blocks below
// become L_ib = A_ib M_b^T (one wave each), then the trailing blocks take
// A_ij -= L_ib L_jb^T (round robin over the waves), all on the FP64 matrix
// cores (v_mfma_f64_16x16x4). The inverse of L follows by block columns, one
// wave each: (L^-1)_bb = M_b, (L^-1)_ib = -M_i sum_{b<=k<i} L_ik (L^-1)_kb.
// A block in registers uses the accumulator layout of the FP64 16x16x4
// product: lane l, element e holds row (l >> 4) + 4e, column l & 15. That is
// also the layout of a B operand chunk (rows 4kk + (l >> 4) in element kk),
// so a block in registers multiplies from the right without staging. The
// upper blocks of the tile (zero in L) keep M_0..M_3 until the end. The
// factor (zeros above the diagonal) is left in sA; the inverse goes from
// registers to the global 64x64 row-major Dg (and its FP32 copy to Df). A
// non-positive pivot sets *fail.
__device__ __forceinline__ void mblk_pos(int b, int &bi, int &bj) {
    bi = (b == 3) ? 1 : 0;
    bj = (b == 3) ? 2 : b + 1;
}
__device__ void chol16_wave(double v[4], int &bad) {
    const int l = threadIdx.x & 63, g = l >> 4, q = l & 15;
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        const double d = __shfl(v[c >> 2], c + 16 * (c & 3), 64);   // A[c][c]
        bad |= !(d > 0.0);
        const double piv = sqrt(fmax(d, 1e-300));
        const double rp = 1.0 / piv;
        double colr[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) colr[e] = __shfl(v[e], c + 16 * g, 64);   // A[g + 4e][c]
        // A[c][q], equal to A[q][c]: the trailing matrix is updated on both
        // sides of its diagonal, so it stays symmetric
        const double lq = __shfl(v[c >> 2], q + 16 * (c & 3), 64) * rp;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = g + 4 * e;
            const double lr = colr[e] * rp;
            if (q == c) {
                if (r > c) v[e] = lr;
                else if (r == c) v[e] = piv;
            } else if (q > c && r > c) {
                v[e] -= lr * lq;
            }
        }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
        if (g + 4 * e < q) v[e] = 0.0;
}
// M = L^-1 for the lower-triangular 16x16 L in registers: M = I, then for
// each pivot row p, row p of M is scaled by 1 / L[p][p] (final) and taken
// off the rows below it, L[r][p] times.
__device__ void inv16_wave(const double v[4], double m[4]) {
    const int l = threadIdx.x & 63, g = l >> 4, q = l & 15;
#pragma unroll
    for (int e = 0; e < 4; ++e) m[e] = (g + 4 * e == q) ? 1.0 : 0.0;
#pragma unroll
    for (int p = 0; p < 16; ++p) {
        const double lpp = __shfl(v[p >> 2], p + 16 * (p & 3), 64);
        if (g == (p & 3)) m[p >> 2] /= lpp;
        const double xq = __shfl(m[p >> 2], q + 16 * (p & 3), 64);   // M[p][q], final
        double lrp[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) lrp[e] = __shfl(v[e], p + 16 * g, 64);   // L[g + 4e][p]
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (g + 4 * e > p) m[e] -= lrp[e] * xq;
    }
}
__device__ void chol_inv64_blocked(double (*sA)[LDP], double *Dg, float *Df, int *fail) {
    const int t = threadIdx.x, w = __builtin_amdgcn_readfirstlane(t >> 6), l = t & 63, g = l >> 4, q = l & 15;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        if (w == 0) {
            double v[4], m[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = sA[16 * b + g + 4 * e][16 * b + q];
            int bad = 0;
            chol16_wave(v, bad);
            inv16_wave(v, m);
            int bi, bj;
            mblk_pos(b, bi, bj);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                sA[16 * b + g + 4 * e][16 * b + q] = v[e];
                sA[16 * bi + g + 4 * e][16 * bj + q] = m[e];
            }
            if (bad && l == 0) *fail = 1;
        }
        __syncthreads();
        if (b == 3) break;
        {
            // L_ib = A_ib M_b^T: B[k][q] = M_b[q][k]
            const int i = b + 1 + w;
            if (i < 4) {
                int bi, bj;
                mblk_pos(b, bi, bj);
                v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int k = 4 * kk + g;
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sA[16 * i + q][16 * b + k],
                                                               sA[16 * bi + q][16 * bj + k], acc, 0, 0, 0);
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) sA[16 * i + g + 4 * e][16 * b + q] = acc[e];
            }
        }
        __syncthreads();
        {
            // A_ij -= L_ib L_jb^T, b < j <= i: B[k][q] = L_jb[q][k]
            int task = 0;
#pragma unroll
            for (int i = b + 1; i < 4; ++i)
#pragma unroll
                for (int j = b + 1; j <= i; ++j, ++task) {
                    if ((task & 3) != w) continue;
                    v4d acc;
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc[e] = sA[16 * i + g + 4 * e][16 * j + q];
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        const int k = 4 * kk + g;
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-sA[16 * i + q][16 * b + k],
                                                                   sA[16 * j + q][16 * b + k], acc, 0, 0, 0);
                    }
#pragma unroll
                    for (int e = 0; e < 4; ++e) sA[16 * i + g + 4 * e][16 * j + q] = acc[e];
                }
        }
        __syncthreads();
    }
    {
        // block column w of L^-1, kept in registers
        v4d X[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) X[i] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            if (b != w) continue;
            int bi, bj;
            mblk_pos(b, bi, bj);
#pragma unroll
            for (int e = 0; e < 4; ++e) X[b][e] = sA[16 * bi + g + 4 * e][16 * bj + q];
#pragma unroll
            for (int i = b + 1; i < 4; ++i) {
                v4d s = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int k = b; k < i; ++k)
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk)
                        s = __builtin_amdgcn_mfma_f64_16x16x4f64(sA[16 * i + q][16 * k + 4 * kk + g], X[k][kk], s,
                                                                 0, 0, 0);
                int ni, nj;
                mblk_pos(i, ni, nj);
                v4d r = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    r = __builtin_amdgcn_mfma_f64_16x16x4f64(-sA[16 * ni + q][16 * nj + 4 * kk + g], s[kk], r, 0, 0, 0);
                X[i] = r;
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = 16 * i + g + 4 * e, col = 16 * w + q;
                const double x = (i >= w) ? X[i][e] : 0.0;
                Dg[row * 64 + col] = x;
                if (Df) Df[row * 64 + col] = (float)x;
            }
    }
    __syncthreads();
    // the upper blocks are zero in L
    for (int f = t; f < 6 * 256; f += 256) {
        const int blk = f >> 8, e = f & 255;
        const int bi = (blk < 3) ? 0 : (blk < 5 ? 1 : 2);
        const int bj = (blk < 3) ? blk + 1 : (blk < 5 ? blk - 1 : 3);
        sA[16 * bi + (e >> 4)][16 * bj + (e & 15)] = 0.0;
    }
    __syncthreads();
}

// Panel j, diagonal tile: L_jj L_jj^T = S_jj - sum_{k<j} L_jk L_jk^T, and
// its inverse. One workgroup per submatrix with P > j. A non-positive pivot
// marks the submatrix NOT_SPD; its later launches then skip it.
template <typename T>
__global__ __launch_bounds__(256, 4) void k_chol_diag(ChunkDev cd, char *ws, int j) {
    // one tile (33 KB in FP64) plus small buffers, and at most 128 VGPRs:
    // four workgroups share a CU, so that the serial chains of one (the
    // diagonal blocks) hide behind the others
    __shared__ T sA[64][LDP];
    __shared__ T cb[2][64];
    __shared__ T rd[64];
    __shared__ int fail;
    const int s = blockIdx.x;
    if (s >= cd.nsub) return;
    const SubMeta M = cd.meta[s];
    SubCtl *ctl = cd.ctl + s;
    if (j >= M.P || ctl->status != NOLSM_MOL_OK) return;
    T *L = (T *)(ws + M.offL);         // S, factored in place (FP32 route: FP32)
    T *Dinv = (T *)(ws + M.offDinv);
    const int64_t ld = M.np;
    auto Lt = [&](int r, int c) { return L + (int64_t)(r * 64) * ld + c * 64; };
    if (threadIdx.x == 0) fail = 0;
    AccT<T> acc;
    g2acc(acc, Lt(j, j), ld);
    // - L_jk L_jk^T over k < j, tile k + 1 loaded into registers while
    // tile k is multiplied
    RegTile<T> pl;
    if (j > 0) g2r_tile(pl, Lt(j, 0), ld);
    for (int k = 0; k < j; ++k) {
        r2s_tile(sA, pl);
        __syncthreads();
        if (k + 1 < j) g2r_tile(pl, Lt(j, k + 1), ld);
        mma64<false, true>(acc, sA, sA, -1.0);
        __syncthreads();
    }
    acc2s(sA, acc);
    __syncthreads();
    // FP64 factor applied in FP32: the tile and its inverse also in FP32
    float *L32 = M.offL32 ? (float *)(ws + M.offL32) : nullptr;
    float *D32 = M.offDinv32 ? (float *)(ws + M.offDinv32) + (int64_t)j * 4096 : nullptr;
    if constexpr (sizeof(T) == 8) {
        chol_inv64_blocked(sA, Dinv + (int64_t)j * 4096, D32, &fail);
        if (fail) {
            if (threadIdx.x == 0) { ctl->status = NOLSM_MOL_NOT_SPD; ctl->done = 1; }
            return;
        }
    } else {
        potrf64_reg(sA, cb, &fail);
        if (fail) {
            if (threadIdx.x == 0) { ctl->status = NOLSM_MOL_NOT_SPD; ctl->done = 1; }
            return;
        }
        trinv64_reg(sA, Dinv + (int64_t)j * 4096, rd, cb, D32);
    }
    s2g_tile(Lt(j, j), ld, sA);
    if (L32) s2g_tile(L32 + (int64_t)(j * 64) * ld + j * 64, ld, sA);
}

// Panel j below the diagonal: L_ij = (S_ij - sum_{k<j} L_ik L_jk^T) L_jj^-T
// for CHOL_PR row tiles i per workgroup, which share each L_jk load; the
// row tiles of a panel run in parallel. Grid: (submatrix, block of rows).
#define CHOL_PR 4
template <typename T, int OCC>
__global__ __launch_bounds__(256, OCC) void k_chol_panel(ChunkDev cd, char *ws, int j) {
    __shared__ T sA[64][LDP];
    __shared__ T sB[64][LDP];
    const int s = blockIdx.x;
    if (s >= cd.nsub) return;
    const SubMeta M = cd.meta[s];
    const int P = M.P, i0 = j + 1 + (int)blockIdx.y * CHOL_PR;
    if (i0 >= P || cd.ctl[s].status != NOLSM_MOL_OK) return;
    T *L = (T *)(ws + M.offL);
    const T *Dinv = (const T *)(ws + M.offDinv);
    const int64_t ld = M.np;
    auto Lt = [&](int r, int c) { return L + (int64_t)(r * 64) * ld + c * 64; };
    const int nr = min(CHOL_PR, P - i0);
    AccT<T> acc[CHOL_PR];
#pragma unroll
    for (int r = 0; r < CHOL_PR; ++r)
        if (r < nr) g2acc(acc[r], Lt(i0 + r, j), ld);
    // - L_ik L_jk^T over k < j: the row-j tile per k, and the row tiles one
    // (k, r) step ahead in registers while the current one is multiplied
    RegTile<T> pl;
    if (j > 0) g2r_tile(pl, Lt(i0, 0), ld);
    for (int k = 0; k < j; ++k) {
        g2s_tile(sB, Lt(j, k), ld);
        r2s_tile(sA, pl);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < CHOL_PR; ++r) {
            if (r < nr) {
                const bool last_r = (r + 1 == nr);
                const int kn = last_r ? k + 1 : k, rn = last_r ? 0 : r + 1;
                if (kn < j) g2r_tile(pl, Lt(i0 + rn, kn), ld);
                mma64<false, true>(acc[r], sA, sB, -1.0);
                __syncthreads();
                if (!last_r) {
                    r2s_tile(sA, pl);
                    __syncthreads();
                }
            }
        }
    }
    g2s_tile(sB, Dinv + (int64_t)j * 4096, 64);
#pragma unroll
    for (int r = 0; r < CHOL_PR; ++r) {
        if (r < nr) {
            acc2s(sA, acc[r]);
            __syncthreads();
            AccT<T> o;
            acc_zero(o);
            mma64<false, true>(o, sA, sB);   // acc L_jj^-T
            __syncthreads();
            acc2s(sA, o);
            __syncthreads();
            s2g_tile(Lt(i0 + r, j), ld, sA);
            if (M.offL32) s2g_tile((float *)(ws + M.offL32) + (int64_t)((i0 + r) * 64) * ld + j * 64, ld, sA);
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Substitution for SC consecutive 64-column tiles cc .. cc + SC - 1 of
// [K | E] (tile P is the E tile): W = L^-1 B (forward), then [A | Y] = L^-T W
// (backward), in place in the K buffer; mu is taken off A's diagonal once
// its column tile is complete (the backward recursion needs the unshifted
// rows). For every column tile < P it also emits the |A| row sums of the
// tile, the complete |A| column sums and a partial Frobenius sum (bounds
// inputs). Task list: (slot, cc), cc = 0..P; tasks with cc % SC != 0 return.
// SR row tiles are solved per pass with their accumulators in registers: each
// L tile is read once per pass and task, and each finished tile of the
// column once per pass (the tasks of a submatrix are adjacent in the task
// list and share L through one XCD's L2 while they run together).
// ---------------------------------------------------------------------------
template <typename T, int SR, int SC, int OCC, bool FWD_ONLY>
__global__ __launch_bounds__(256, OCC) void k_subst(ChunkDev cd, char *ws) {
    const double mu = ((const WsHeader *)ws)->mu;
    __shared__ T sA[64][LDP];
    __shared__ T sB[SC][64][LDP];
    __shared__ double red[256];
    const uint32_t task = xcd_task(cd.t_subst);
    if (task == NOLSM_TASK_NONE) return;
    const int s = task_slot(task), cc = task_a(task);
    if (cc % SC) return;
    const SubMeta M = cd.meta[s];
    if (cd.ctl[s].status != NOLSM_MOL_OK) return;
    const int P = M.P, np = M.np, n = M.n;
    const int nc = min(SC, P + 1 - cc);   // column tiles of this task
    const int64_t ldl = np, ldk = np + 64;
    // FP32 arithmetic reads the FP32 copy of an FP64 factor when there is one
    const bool l32 = sizeof(T) == 4 && M.offL32;
    const T *L = (const T *)(ws + (l32 ? M.offL32 : M.offL));
    const T *Dinv = (const T *)(ws + (l32 ? M.offDinv32 : M.offDinv));
    // the K buffer is stored in the arithmetic type (SubMeta::kf32 <=> FP32)
    T *Kb = (T *)(ws + M.offK);
    auto Lt = [&](int r, int c) { return L + (int64_t)(r * 64) * ldl + c * 64; };
    auto Bt = [&](int c, int r) {   // row tile r of this task's column c
        const int col0 = (cc + c < P) ? (cc + c) * 64 : np;
        return Kb + (int64_t)(r * 64) * ldk + col0;
    };
    // forward: W_i = Dinv_i (B_i - sum_{k<i} L_ik W_k). Row i needs only the
    // rows above it, and the symmetric route's right solve reads W only on
    // and above the diagonal (W_ij, j >= i: the rest of A~ comes from its
    // upper tiles), so there the column tiles stop at their diagonal row; the
    // E tile (y = L^-1 E) takes every row.
    const int Pr = (FWD_ONLY && cc + nc <= P) ? cc + nc : P;
    // The E tile alone: its rows above the first owned block are zero in
    // E and stay zero in L^-1 E (L is lower triangular), so the solve
    // starts at that block's row tile and sums only from there.
    const int i1 = (cc == P) ? (M.pmin * (n / M.m)) / 64 : 0;
    for (int i0 = i1; i0 < Pr; i0 += SR) {
        const int nr = min(SR, Pr - i0);
        AccT<T> acc[SR][SC];
#pragma unroll
        for (int r = 0; r < SR; ++r)
#pragma unroll
            for (int c = 0; c < SC; ++c)
                if (r < nr && c < nc) g2acc(acc[r][c], Bt(c, i0 + r), ldk);
        // the updates from the finished rows k < i0, one (k, r) step at a
        // time: the tiles of the next step are loaded into registers while
        // this step multiplies from LDS
        if (i0 > i1) {
            RegTile<T> pl;
            g2r_tile(pl, Lt(i0, i1), ldl);
            r2s_tile(sA, pl);
            for (int k = i1; k < i0; ++k) {
#pragma unroll
                for (int c = 0; c < SC; ++c)
                    if (c < nc) g2s_tile(sB[c], Bt(c, k), ldk);
                __syncthreads();
#pragma unroll
                for (int r = 0; r < SR; ++r) {
                    if (r < nr) {
                        const bool last_r = (r + 1 == nr);
                        const int kn = last_r ? k + 1 : k, rn = last_r ? 0 : r + 1;
                        const bool more = kn < i0;
                        if (more) g2r_tile(pl, Lt(i0 + rn, kn), ldl);
#pragma unroll
                        for (int c = 0; c < SC; ++c)
                            if (c < nc) mma64<false, false>(acc[r][c], sA, sB[c], -1.0);
                        __syncthreads();
                        if (more) r2s_tile(sA, pl);
                        if (!last_r) __syncthreads();
                    }
                }
            }
            __syncthreads();
        }
        // the diagonal block of the pass, in order
#pragma unroll
        for (int r = 0; r < SR; ++r) {
            if (r < nr) {
                const int i = i0 + r;
                g2s_tile(sA, Dinv + (int64_t)i * 4096, 64);
#pragma unroll
                for (int c = 0; c < SC; ++c)
                    if (c < nc) acc2s(sB[c], acc[r][c]);
                __syncthreads();
#pragma unroll
                for (int c = 0; c < SC; ++c) {
                    if (c < nc) {
                        AccT<T> o;
                        acc_zero(o);
                        mma64<false, false>(o, sA, sB[c]);
                        __syncthreads();
                        acc2s(sB[c], o);
                    }
                }
                __syncthreads();
#pragma unroll
                for (int c = 0; c < SC; ++c)
                    if (c < nc) s2g_tile(Bt(c, i), ldk, sB[c]);   // W_i, kept in sB for the rows below
#pragma unroll
                for (int r2 = r + 1; r2 < SR; ++r2) {
                    if (r2 < nr) {
                        g2s_tile(sA, Lt(i0 + r2, i), ldl);
                        __syncthreads();
#pragma unroll
                        for (int c = 0; c < SC; ++c)
                            if (c < nc) mma64<false, false>(acc[r2][c], sA, sB[c], -1.0);
                        __syncthreads();
                    }
                }
                __syncthreads();
            }
        }
    }
    // symmetric route: [W | y] = L^-1 [K | E] is all this kernel forms
    if constexpr (FWD_ONLY) return;
    // backward: A_i = Dinv_i^T (W_i - sum_{k>i} L_ki^T A_k), passes from the bottom
    double colsum[SC], frob[SC];
#pragma unroll
    for (int c = 0; c < SC; ++c) colsum[c] = frob[c] = 0.0;
    for (int i1 = P - 1; i1 >= 0; i1 -= SR) {
        const int nr = min(SR, i1 + 1);   // rows i1 - r, r < nr
        AccT<T> acc[SR][SC];
#pragma unroll
        for (int r = 0; r < SR; ++r)
#pragma unroll
            for (int c = 0; c < SC; ++c)
                if (r < nr && c < nc) g2acc(acc[r][c], Bt(c, i1 - r), ldk);
        for (int k = i1 + 1; k < P; ++k) {
#pragma unroll
            for (int c = 0; c < SC; ++c)
                if (c < nc) g2s_tile(sB[c], Bt(c, k), ldk);   // A_k, unshifted
#pragma unroll
            for (int r = 0; r < SR; ++r) {
                if (r < nr) {
                    g2s_tile(sA, Lt(k, i1 - r), ldl);
                    __syncthreads();
#pragma unroll
                    for (int c = 0; c < SC; ++c)
                        if (c < nc) mma64<true, false>(acc[r][c], sA, sB[c], -1.0);
                    __syncthreads();
                }
            }
        }
#pragma unroll
        for (int r = 0; r < SR; ++r) {
            if (r < nr) {
                const int i = i1 - r;
                g2s_tile(sA, Dinv + (int64_t)i * 4096, 64);
#pragma unroll
                for (int c = 0; c < SC; ++c)
                    if (c < nc) acc2s(sB[c], acc[r][c]);
                __syncthreads();
#pragma unroll
                for (int c = 0; c < SC; ++c) {
                    if (c < nc) {
                        AccT<T> o;
                        acc_zero(o);
                        mma64<true, false>(o, sA, sB[c]);
                        __syncthreads();
                        acc2s(sB[c], o);
                    }
                }
                __syncthreads();
#pragma unroll
                for (int c = 0; c < SC; ++c) {
                    const int ccol = cc + c;
                    if (c < nc && ccol < P) {
                        // bounds inputs of A_J - mu I; the tile itself is
                        // stored without the shift, since the rows above
                        // still use it
                        auto a = [&](int rr, int q) {
                            return (double)sB[c][rr][q] - ((i == ccol && rr == q) ? mu : 0.0);
                        };
                        const int t = threadIdx.x;
                        if (t < 64) {
                            const int gr = i * 64 + t;
                            double rs = 0.0;
                            for (int q = 0; q < 64; ++q)
                                if (ccol * 64 + q < n) rs += fabs(a(t, q));
                            double *rowp = (double *)(ws + M.offRow);
                            rowp[(int64_t)ccol * np + gr] = (gr < n) ? rs : 0.0;
                        } else if (t < 128) {
                            const int q = t - 64;
                            for (int rr = 0; rr < 64; ++rr)
                                if (i * 64 + rr < n) colsum[c] += fabs(a(rr, q));
                        }
                        // Frobenius partial: 16 entries per thread
                        double fs = 0.0;
                        for (int f = t; f < 4096; f += 256) {
                            const int rr = f >> 6, q = f & 63;
                            if (i * 64 + rr < n && ccol * 64 + q < n) fs += a(rr, q) * a(rr, q);
                        }
                        frob[c] += fs;
                    }
                }
#pragma unroll
                for (int c = 0; c < SC; ++c)
                    if (c < nc) s2g_tile(Bt(c, i), ldk, sB[c]);   // A_i, kept in sB for the rows above
#pragma unroll
                for (int r2 = r + 1; r2 < SR; ++r2) {
                    if (r2 < nr) {
                        g2s_tile(sA, Lt(i, i1 - r2), ldl);
                        __syncthreads();
#pragma unroll
                        for (int c = 0; c < SC; ++c)
                            if (c < nc) mma64<true, false>(acc[r2][c], sA, sB[c], -1.0);
                        __syncthreads();
                    }
                }
                __syncthreads();
            }
        }
    }
#pragma unroll
    for (int c = 0; c < SC; ++c) {
        const int ccol = cc + c;
        if (c < nc && ccol < P) {
            // the whole column tile is final: take mu off the diagonal of A_J
            const int t = threadIdx.x;
            if (t < 64) Kb[(int64_t)(ccol * 64 + t) * ldk + ccol * 64 + t] -= mu;
            double *colp = (double *)(ws + M.offCol);
            if (t >= 64 && t < 128) {
                const int q = t - 64;
                colp[ccol * 64 + q] = (ccol * 64 + q < n) ? colsum[c] : 0.0;
            }
            const double fsum = block_sum(frob[c], red);
            if (t == 0) colp[np + ccol] = fsum;
        }
    }
}

// ---------------------------------------------------------------------------
// Symmetric sign iteration, second half of the setup: with W = L^-1 K_J in the K
// buffer (from the forward-only substitution), A~ = W L^-T = L^-1 K_J L^-T,
// row block i per launch (one workgroup per submatrix), in place:
// X_ij = (W_ij - sum_{k<j} X_ik L_jk^T) Dinv_j^T over the column tiles
// j >= i in order. The tiles left of the diagonal are not solved again:
// A~ is symmetric, so X_ik = X_ki^T for k < i, final since the launch of row
// block k, which saves a third of the right solve's products; they are read
// transposed from the upper triangle and never stored below it (nothing after
// this kernel reads A~ below its diagonal tiles). A~ - mu I has the spectrum
// of A_J. Bounds inputs in the layout of k_subst: each tile writes the row
// sums of its rows, and an off-diagonal tile also its column sums, which are
// the row sums of its mirror X_ji; the Frobenius partial of row block i
// counts every off-diagonal tile twice. Being symmetric, the matrix's column
// sums are its row sums, which the bounds kernel takes from the row sums. mu
// is taken off the diagonal once the row block is complete. RR column tiles
// per pass with their accumulators in registers.
// ---------------------------------------------------------------------------
template <typename T, int RR, int OCC>
__global__ __launch_bounds__(256, OCC) void k_rsolve(ChunkDev cd, char *ws, int i) {
    const double mu = ((const WsHeader *)ws)->mu;
    __shared__ T sX[64][LDP];
    __shared__ T sL[64][LDP];
    __shared__ double red[256];
    const int s = blockIdx.x;
    if (s >= cd.nsub) return;
    const SubMeta M = cd.meta[s];
    if (cd.ctl[s].status != NOLSM_MOL_OK) return;
    const int P = M.P, np = M.np, n = M.n;
    if (i >= P) return;
    const int64_t ldl = np, ldk = np + 64;
    // FP32 arithmetic reads the FP32 copy of an FP64 factor when there is one
    const bool l32 = sizeof(T) == 4 && M.offL32;
    const T *L = (const T *)(ws + (l32 ? M.offL32 : M.offL));
    const T *Dinv = (const T *)(ws + (l32 ? M.offDinv32 : M.offDinv));
    T *Kb = (T *)(ws + M.offK);   // in the arithmetic type (SubMeta::kf32 <=> FP32)
    double *rowp = (double *)(ws + M.offRow);
    auto Lt = [&](int r, int c) { return L + (int64_t)(r * 64) * ldl + c * 64; };
    auto Xt = [&](int j) { return Kb + (int64_t)(i * 64) * ldk + j * 64; };   // tile (i, j), j >= i
    auto Ut = [&](int k) { return Kb + (int64_t)(k * 64) * ldk + i * 64; };   // tile (k, i) = X_ik^T
    // X_ik into LDS: the tile itself on and right of the diagonal, the
    // transpose of X_ki left of it
    auto load_x = [&](int k) {
        if (k < i) g2s_tile_t(sX, Ut(k), ldk);
        else g2s_tile(sX, Xt(k), ldk);
    };
    const int t = threadIdx.x;
    double frob = 0.0;
    for (int j0 = i; j0 < P; j0 += RR) {
        const int nr = min(RR, P - j0);
        AccT<T> acc[RR];
#pragma unroll
        for (int r = 0; r < RR; ++r)
            if (r < nr) g2acc(acc[r], Xt(j0 + r), ldk);
        // - X_ik L_jk^T for the finished tiles k < j0, one (k, r) step at a
        // time: the tiles of the next step are loaded into registers while
        // this step multiplies from LDS
        if (j0 > 0) {
            RegTile<T> pl;
            g2r_tile(pl, Lt(j0, 0), ldl);
            r2s_tile(sL, pl);
            for (int k = 0; k < j0; ++k) {
                load_x(k);
                __syncthreads();
#pragma unroll
                for (int r = 0; r < RR; ++r) {
                    if (r < nr) {
                        const bool last_r = (r + 1 == nr);
                        const int kn = last_r ? k + 1 : k, rn = last_r ? 0 : r + 1;
                        const bool more = kn < j0;
                        if (more) g2r_tile(pl, Lt(j0 + rn, kn), ldl);
                        mma64<false, true>(acc[r], sX, sL, -1.0);
                        __syncthreads();
                        if (more) r2s_tile(sL, pl);
                        if (!last_r) __syncthreads();
                    }
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            if (r < nr) {
                const int j = j0 + r;
                g2s_tile(sL, Dinv + (int64_t)j * 4096, 64);
                acc2s(sX, acc[r]);
                __syncthreads();
                AccT<T> o;
                acc_zero(o);
                mma64<false, true>(o, sX, sL);   // acc Dinv_j^T
                __syncthreads();
                acc2s(sX, o);
                __syncthreads();
                {
                    // bounds inputs of A~ - mu I (stored unshifted: later
                    // tiles of this row block still use it)
                    auto a = [&](int rr, int q) { return (double)sX[rr][q] - ((i == j && rr == q) ? mu : 0.0); };
                    if (t < 64) {
                        const int gr = i * 64 + t;
                        double rs = 0.0;
                        for (int q = 0; q < 64; ++q)
                            if (j * 64 + q < n) rs += fabs(a(t, q));
                        rowp[(int64_t)j * np + gr] = (gr < n) ? rs : 0.0;
                    } else if (t < 128 && j > i) {
                        // row sums of the mirror tile X_ji over column tile i
                        const int gc = j * 64 + t - 64;
                        double cs = 0.0;
                        for (int rr = 0; rr < 64; ++rr)
                            if (i * 64 + rr < n) cs += fabs(a(rr, t - 64));
                        rowp[(int64_t)i * np + gc] = (gc < n) ? cs : 0.0;
                    }
                    double fs = 0.0;
                    for (int f = t; f < 4096; f += 256) {
                        const int rr = f >> 6, q = f & 63;
                        if (i * 64 + rr < n && j * 64 + q < n) fs += a(rr, q) * a(rr, q);
                    }
                    frob += (j > i) ? 2.0 * fs : fs;
                }
                s2g_tile(Xt(j), ldk, sX);   // X_ij, kept in sX for the tiles to its right
#pragma unroll
                for (int r2 = r + 1; r2 < RR; ++r2) {
                    if (r2 < nr) {
                        g2s_tile(sL, Lt(j0 + r2, j), ldl);
                        __syncthreads();
                        mma64<false, true>(acc[r2], sX, sL, -1.0);
                        __syncthreads();
                    }
                }
                __syncthreads();
            }
        }
    }
    // the row block is final: take mu off its diagonal
    if (t < 64) Kb[(int64_t)(i * 64 + t) * ldk + i * 64 + t] -= mu;
    const double fsum = block_sum(frob, red);
    if (t == 0) ((double *)(ws + M.offCol))[np + i] = fsum;
}

// ---------------------------------------------------------------------------
// k_subst's forward pass and k_rsolve for the symmetric route with FP32
// arithmetic, with their tile products on the FP16 matrix cores as split
// hi + lo operands (split16.h; about 2^-22 relative per operand, and the
// result feeds an FP16 iterate). The FP32 accumulators are written out
// through an FP32 LDS tile. The K columns are operands scaled by the power
// of two sc of max |T_J(K)| (sc max |K| in [1, 2)), which W = L^-1 K and A~
// carry until they are stored; the E tile (entries 0 and 1) is not scaled.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void acc_mul(AccT<float> &a, float f) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) a.c[i][j][e] *= f;
}

// [W | y] = L^-1 [K | E], column tile cc of one submatrix per task, the
// column tiles of K to their diagonal row
template <int SR, int OCC>
__global__ __launch_bounds__(256, OCC) void k_subst_hl(ChunkDev cd, char *ws) {
    __shared__ __attribute__((aligned(16))) HLTile sA;   // L_ik (negated) or Dinv_i: A[m][k]
    __shared__ __attribute__((aligned(16))) HLTile sB;   // W_k, k-major: B[k][n] = sB(n, k)
    __shared__ float sF[64][LDP];
    const uint32_t task = xcd_task(cd.t_subst);
    if (task == NOLSM_TASK_NONE) return;
    const int s = task_slot(task), cc = task_a(task);
    const SubMeta M = cd.meta[s];
    if (cd.ctl[s].status != NOLSM_MOL_OK) return;
    const int P = M.P, np = M.np, n = M.n;
    const int64_t ldl = np, ldk = np + 64;
    const float *L = (const float *)(ws + (M.offL32 ? M.offL32 : M.offL));
    const float *Dinv = (const float *)(ws + (M.offL32 ? M.offDinv32 : M.offDinv));
    float *Kb = (float *)(ws + M.offK);
    float sc = 1.0f, inv = 1.0f;
    if (cc < P) hl_scale(__uint_as_float(cd.ctl[s].kmax), sc, inv);
    auto Lt = [&](int r, int c) { return L + (int64_t)(r * 64) * ldl + c * 64; };
    const int col0 = (cc < P) ? cc * 64 : np;
    auto Bt = [&](int r) { return Kb + (int64_t)(r * 64) * ldk + col0; };
    // a column tile of K stops at its diagonal row; the E tile starts at the
    // row tile of its first owned block (the rows above stay zero)
    const int Pr = (cc < P) ? cc + 1 : P;
    const int i1 = (cc == P) ? (M.pmin * (n / M.m)) / 64 : 0;
    for (int i0 = i1; i0 < Pr; i0 += SR) {
        const int nr = min(SR, Pr - i0);
        AccT<float> acc[SR];
#pragma unroll
        for (int r = 0; r < SR; ++r)
            if (r < nr) {
                g2acc(acc[r], Bt(i0 + r), ldk);
                acc_mul(acc[r], sc);
            }
        if (i0 > i1) {
            RegTile<float> pl;
            g2r_tile(pl, Lt(i0, i1), ldl);
            r2hl(sA, pl, -1.0f);
            for (int k = i1; k < i0; ++k) {
                g2hl_t(sB, Bt(k), ldk, sc);
                __syncthreads();
#pragma unroll
                for (int r = 0; r < SR; ++r) {
                    if (r < nr) {
                        const bool last_r = (r + 1 == nr);
                        const int kn = last_r ? k + 1 : k, rn = last_r ? 0 : r + 1;
                        const bool more = kn < i0;
                        if (more) g2r_tile(pl, Lt(i0 + rn, kn), ldl);
                        mma64_hl(acc[r], sA, sB);
                        __syncthreads();
                        if (more) r2hl(sA, pl, -1.0f);
                        if (!last_r) __syncthreads();
                    }
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < SR; ++r) {
            if (r < nr) {
                const int i = i0 + r;
                g2hl(sA, Dinv + (int64_t)i * 4096, 64, 1.0f);
                acc2hl_t(sB, acc[r], 1.0f);
                __syncthreads();
                AccT<float> o;
                acc_zero(o);
                mma64_hl(o, sA, sB);   // sc W_i
                __syncthreads();
                acc2hl_t(sB, o, 1.0f);   // kept for the rows below
                acc_mul(o, inv);
                acc2s(sF, o);
                __syncthreads();
                s2g_tile(Bt(i), ldk, sF);
#pragma unroll
                for (int r2 = r + 1; r2 < SR; ++r2) {
                    if (r2 < nr) {
                        g2hl(sA, Lt(i0 + r2, i), ldl, -1.0f);
                        __syncthreads();
                        mma64_hl(acc[r2], sA, sB);
                        __syncthreads();
                    }
                }
                __syncthreads();
            }
        }
    }
}

// A~ = W L^-T, two row blocks (i, i + 1) per launch: every tile of the factor
// that the launch reads serves both rows, so the factor's lower triangle is
// read half as often as with one row block per launch. First the three
// tiles (i, i), (i, i + 1), (i + 1, i + 1), in that order (row i + 1 needs
// X_{i+1,i} = X_{i,i+1}^T); then passes of RC column tiles j >= i + 2 with
// both rows' accumulators in registers.
template <int RC, int OCC>
__global__ __launch_bounds__(256, OCC) void k_rsolve2_hl(ChunkDev cd, char *ws, int i) {
    const double mu = ((const WsHeader *)ws)->mu;
    __shared__ __attribute__((aligned(16))) HLTile sXa;   // operands of row i
    __shared__ __attribute__((aligned(16))) HLTile sXb;   // operands of row i + 1
    __shared__ __attribute__((aligned(16))) HLTile sL;    // L_jk or Dinv_j: B[k][n] = sL(n, k)
    __shared__ float sF[64][LDP];
    __shared__ double red[256];
    const int s = blockIdx.x;
    if (s >= cd.nsub) return;
    const SubMeta M = cd.meta[s];
    if (cd.ctl[s].status != NOLSM_MOL_OK) return;
    const int P = M.P, np = M.np, n = M.n;
    if (i >= P) return;
    const bool two = i + 1 < P;
    const int64_t ldl = np, ldk = np + 64;
    const float *L = (const float *)(ws + (M.offL32 ? M.offL32 : M.offL));
    const float *Dinv = (const float *)(ws + (M.offL32 ? M.offDinv32 : M.offDinv));
    float *Kb = (float *)(ws + M.offK);
    double *rowp = (double *)(ws + M.offRow);
    float sc, inv;
    hl_scale(__uint_as_float(cd.ctl[s].kmax), sc, inv);
    auto Lt = [&](int r, int c) { return L + (int64_t)(r * 64) * ldl + c * 64; };
    auto Dt = [&](int j) { return Dinv + (int64_t)j * 4096; };
    auto Xt = [&](int r, int j) { return Kb + (int64_t)(r * 64) * ldk + j * 64; };   // stored for j >= r
    // -sc X_{r,k} as an A operand: the stored tile, or for k < r the
    // transpose of the stored tile (k, r)
    auto load_x = [&](HLTile &dst, int r, int k) {
        if (k < r) g2hl_t(dst, Xt(k, r), ldk, -sc);
        else g2hl(dst, Xt(r, k), ldk, -sc);
    };
    const int t = threadIdx.x;
    double frob0 = 0.0, frob1 = 0.0;
    // a final tile o = sc X_{r,j} (accumulator layout): the bounds inputs of
    // A~ - mu I as in k_rsolve, and the FP32 store
    auto emit = [&](const AccT<float> &o, int r, int j, double &frob) {
        __syncthreads();
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int e = 0; e < 4; ++e) sF[acc_row<float>(bi, e)][acc_col(bj)] = o.c[bi][bj][e] * inv;
        __syncthreads();
        auto a = [&](int rr, int q) { return (double)sF[rr][q] - ((r == j && rr == q) ? mu : 0.0); };
        if (t < 64) {
            const int gr = r * 64 + t;
            double rs = 0.0;
            for (int q = 0; q < 64; ++q)
                if (j * 64 + q < n) rs += fabs(a(t, q));
            rowp[(int64_t)j * np + gr] = (gr < n) ? rs : 0.0;
        } else if (t < 128 && j > r) {
            const int gc = j * 64 + t - 64;
            double cs = 0.0;
            for (int rr = 0; rr < 64; ++rr)
                if (r * 64 + rr < n) cs += fabs(a(rr, t - 64));
            rowp[(int64_t)r * np + gc] = (gc < n) ? cs : 0.0;
        }
        double fs = 0.0;
        for (int f = t; f < 4096; f += 256) {
            const int rr = f >> 6, q = f & 63;
            if (r * 64 + rr < n && j * 64 + q < n) fs += a(rr, q) * a(rr, q);
        }
        frob += (j > r) ? 2.0 * fs : fs;
        s2g_tile(Xt(r, j), ldk, sF);
    };
    // o = acc Dinv_j^T with acc staged in sXa
    auto diag = [&](AccT<float> &o, const AccT<float> &acc, int j) {
        g2hl(sL, Dt(j), 64, 1.0f);
        acc2hl(sXa, acc, 1.0f);
        __syncthreads();
        acc_zero(o);
        mma64_hl(o, sXa, sL);
        __syncthreads();
    };
    {
        AccT<float> a00, a01, a11, o;
        g2acc(a00, Xt(i, i), ldk);
        acc_mul(a00, sc);
        if (two) {
            g2acc(a01, Xt(i, i + 1), ldk);
            acc_mul(a01, sc);
            g2acc(a11, Xt(i + 1, i + 1), ldk);
            acc_mul(a11, sc);
        }
        for (int k = 0; k < i; ++k) {
            load_x(sXa, i, k);
            if (two) load_x(sXb, i + 1, k);
            g2hl(sL, Lt(i, k), ldl, 1.0f);
            __syncthreads();
            mma64_hl(a00, sXa, sL);
            __syncthreads();
            if (two) {
                g2hl(sL, Lt(i + 1, k), ldl, 1.0f);
                __syncthreads();
                mma64_hl(a01, sXa, sL);
                mma64_hl(a11, sXb, sL);
                __syncthreads();
            }
        }
        diag(o, a00, i);
        emit(o, i, i, frob0);
        if (two) {
            acc2hl(sXa, o, -1.0f);
            g2hl(sL, Lt(i + 1, i), ldl, 1.0f);
            __syncthreads();
            mma64_hl(a01, sXa, sL);   // - X_ii L_{i+1,i}^T
            __syncthreads();
            diag(o, a01, i + 1);
            emit(o, i, i + 1, frob0);
            acc2hl_t(sXb, o, -1.0f);   // -sc X_{i+1,i} = -sc X_{i,i+1}^T
            g2hl(sL, Lt(i + 1, i), ldl, 1.0f);
            __syncthreads();
            mma64_hl(a11, sXb, sL);
            __syncthreads();
            diag(o, a11, i + 1);
            emit(o, i + 1, i + 1, frob1);
        }
    }
    if (two) {
        for (int j0 = i + 2; j0 < P; j0 += RC) {
            const int nr = min(RC, P - j0);
            AccT<float> a0[RC], a1[RC];
#pragma unroll
            for (int r = 0; r < RC; ++r)
                if (r < nr) {
                    g2acc(a0[r], Xt(i, j0 + r), ldk);
                    acc_mul(a0[r], sc);
                    g2acc(a1[r], Xt(i + 1, j0 + r), ldk);
                    acc_mul(a1[r], sc);
                }
            {
                __syncthreads();
                RegTile<float> pl;
                g2r_tile(pl, Lt(j0, 0), ldl);
                r2hl(sL, pl, 1.0f);
                for (int k = 0; k < j0; ++k) {
                    load_x(sXa, i, k);
                    load_x(sXb, i + 1, k);
                    __syncthreads();
#pragma unroll
                    for (int r = 0; r < RC; ++r) {
                        if (r < nr) {
                            const bool last_r = (r + 1 == nr);
                            const int kn = last_r ? k + 1 : k, rn = last_r ? 0 : r + 1;
                            const bool more = kn < j0;
                            if (more) g2r_tile(pl, Lt(j0 + rn, kn), ldl);
                            mma64_hl(a0[r], sXa, sL);
                            mma64_hl(a1[r], sXb, sL);
                            __syncthreads();
                            if (more) r2hl(sL, pl, 1.0f);
                            if (!last_r) __syncthreads();
                        }
                    }
                }
                __syncthreads();
            }
#pragma unroll
            for (int r = 0; r < RC; ++r) {
                if (r < nr) {
                    const int j = j0 + r;
                    AccT<float> o0, o1;
                    g2hl(sL, Dt(j), 64, 1.0f);
                    acc2hl(sXa, a0[r], 1.0f);
                    acc2hl(sXb, a1[r], 1.0f);
                    __syncthreads();
                    acc_zero(o0);
                    acc_zero(o1);
                    mma64_hl(o0, sXa, sL);
                    mma64_hl(o1, sXb, sL);
                    __syncthreads();
                    acc2hl(sXa, o0, -1.0f);   // read by the next products only after emit's barriers
                    emit(o0, i, j, frob0);
                    acc2hl(sXb, o1, -1.0f);
                    emit(o1, i + 1, j, frob1);
#pragma unroll
                    for (int r2 = r + 1; r2 < RC; ++r2) {
                        if (r2 < nr) {
                            g2hl(sL, Lt(j0 + r2, j), ldl, 1.0f);
                            __syncthreads();
                            mma64_hl(a0[r2], sXa, sL);
                            mma64_hl(a1[r2], sXb, sL);
                            __syncthreads();
                        }
                    }
                    __syncthreads();
                }
            }
        }
    }
    // the row blocks are final: take mu off their diagonals
    __syncthreads();
    if (t < 64) {
        Kb[(int64_t)(i * 64 + t) * ldk + i * 64 + t] -= mu;
        if (two) Kb[(int64_t)((i + 1) * 64 + t) * ldk + (i + 1) * 64 + t] -= mu;
    }
    const double f0 = block_sum(frob0, red);
    const double f1 = block_sum(frob1, red);
    if (t == 0) {
        ((double *)(ws + M.offCol))[np + i] = f0;
        if (two) ((double *)(ws + M.offCol))[np + i + 1] = f1;
    }
}

// ---------------------------------------------------------------------------
// Bounds and scale (one workgroup per submatrix). Row and column Gershgorin
// intervals of A_J; their intersection [G_lo, G_hi] encloses the (real)
// spectrum, so c_G = 1/max(|G_lo|, |G_hi|) puts it inside [-1, 1], which
// satisfies the convergence condition of the sign iteration (Sec. III-B.2,
// after Eq. NS2: the matrix is rescaled before the iteration). With learned
// bounds, an MLP predicts the normalised extremes; c = 1/(safety*rho_hat),
// never below c_G. Also writes the 12 features.
// ---------------------------------------------------------------------------
__device__ float silu_f(float z) { return z / (1.0f + expf(-z)); }

__global__ __launch_bounds__(256) void k_bounds(ChunkDev cd, char *ws, BoundsArgs ba) {
    __shared__ double red[256];
    __shared__ float feat[NOLSM_NFEAT];
    __shared__ float h1[64], h2[64], outp[2];
    const int s = blockIdx.x;
    if (s >= cd.nsub) return;
    const SubMeta M = cd.meta[s];
    SubCtl *ctl = cd.ctl + s;
    if (ctl->status != NOLSM_MOL_OK) return;
    const int n = M.n, np = M.np, P = M.P, t = threadIdx.x;
    const double *rowp = (const double *)(ws + M.offRow);
    const double *colp = (const double *)(ws + M.offCol);
    const int64_t ldk = np + 64;
    double dsum = 0, dsq = 0, dmin = 1e300, dmax = -1e300;
    double rsum = 0, rmax = -1e300, rlo = 1e300, rhi = -1e300, clo = 1e300, chi = -1e300;
    for (int r = t; r < n; r += 256) {
        const double d = kbuf_get(M, ws, (int64_t)r * ldk + r);
        double rs = 0;
        for (int c = 0; c < P; ++c) rs += rowp[(int64_t)c * np + r];
        const double R = rs - fabs(d);
        // symmetric route: the column sums are the row sums
        const double C = (ba.sym ? rs : colp[r]) - fabs(d);
        dsum += d; dsq += d * d; dmin = fmin(dmin, d); dmax = fmax(dmax, d);
        rsum += R; rmax = fmax(rmax, R);
        rlo = fmin(rlo, d - R); rhi = fmax(rhi, d + R);
        clo = fmin(clo, d - C); chi = fmax(chi, d + C);
    }
    double fr = 0;
    for (int c = t; c < P; c += 256) fr += colp[np + c];
    dsum = block_sum(dsum, red);
    dsq = block_sum(dsq, red);
    dmin = block_min(dmin, red);
    dmax = block_max(dmax, red);
    rsum = block_sum(rsum, red);
    rmax = block_max(rmax, red);
    rlo = block_min(rlo, red);
    rhi = block_max(rhi, red);
    clo = block_min(clo, red);
    chi = block_max(chi, red);
    fr = block_sum(fr, red);
    const double mean = dsum / n;
    const double glo = fmax(rlo, clo), ghi = fmin(rhi, chi);
    const double rho_g = fmax(fabs(glo), fabs(ghi));
    const double cg = 1.0 / rho_g;
    if (t == 0) {
        double f[NOLSM_NFEAT] = {log((double)n), mean, sqrt(fmax(dsq / n - mean * mean, 0.0)), dmin, dmax,
                                 rsum / n, rmax, rlo, rhi, clo, chi, sqrt(fr / n)};
        for (int i = 0; i < NOLSM_NFEAT; ++i) feat[i] = (float)f[i];
        if (ba.d_features)
            for (int o = 0; o < M.nown; ++o) {
                const int64_t Jo = ba.own_J[M.own_off + o];
                for (int i = 0; i < NOLSM_NFEAT; ++i) ba.d_features[Jo * NOLSM_NFEAT + i] = (float)f[i];
            }
    }
    __syncthreads();
    double c = cg;
    if (ba.learned && ba.d_mlp) {
        // forward of the 12-64-64-2 perceptron in FP32 (weights packed [out][in])
        const float *W1 = ba.d_mlp, *b1 = W1 + 64 * 12, *W2 = b1 + 64, *b2 = W2 + 64 * 64,
                    *W3 = b2 + 64, *b3 = W3 + 2 * 64;
        if (t < 64) {
            float z = b1[t];
            for (int i = 0; i < 12; ++i) z += W1[t * 12 + i] * ((feat[i] - ba.d_norm[i]) / ba.d_norm[12 + i]);
            h1[t] = silu_f(z);
        }
        __syncthreads();
        if (t < 64) {
            float z = b2[t];
            for (int i = 0; i < 64; ++i) z += W2[t * 64 + i] * h1[i];
            h2[t] = silu_f(z);
        }
        __syncthreads();
        if (t < 2) {
            float z = b3[t];
            for (int i = 0; i < 64; ++i) z += W3[t * 64 + i] * h2[i];
            outp[t] = z;
        }
        __syncthreads();
        const double rho_hat = fmax(fabs((double)outp[0] * glo), fabs((double)outp[1] * ghi));
        // c in [c_G, 1.7 c_G]: since rho(A) <= rho_G, c rho(A) <= 1.7 < sqrt(3)
        // whatever the prediction, so no eigenvalue can be mapped past the
        // point where the iteration would converge to the wrong sign
        if (rho_hat > 0 && isfinite(rho_hat)) c = fmin(fmax(1.0 / ((double)ba.safety * rho_hat), cg), 1.7 * cg);
    }
    if (ba.scale_mult != 0.0) c *= ba.scale_mult;
    if (t == 0) {
        ctl->scale = c;
        ctl->scale_g = cg;
        ctl->restart_at = -1;
    }
}

// ---------------------------------------------------------------------------
// X_0 = c_J A_J in the Newton-Schulz precision, identity on the padding
// (sign(diag(A, I)) = diag(sign(A), I): the padding never mixes with A).
// Task list: (slot, 64x64 tile i, j).
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ T cvt(double x);
template <> __device__ __forceinline__ double cvt<double>(double x) { return x; }
template <> __device__ __forceinline__ float cvt<float>(double x) { return (float)x; }
template <> __device__ __forceinline__ _Float16 cvt<_Float16>(double x) { return (_Float16)(float)x; }
template <> __device__ __forceinline__ __bf16 cvt<__bf16>(double x) { return (__bf16)(float)x; }

// SYM (the symmetric iteration on A~ = L^-1 K L^-T - mu I, 16-bit): only
// tiles ti <= tj read A~ (the task list holds no others); an off-diagonal
// tile also writes its transpose (staged in LDS), and a diagonal tile takes
// its lower half from its upper half, so X_0 is exactly symmetric and the
// tiles below the diagonal are never read. The off-diagonal tiles go 8
// consecutive values per thread and access (wide loads and 16-byte stores);
// every value is c a rounded through FP32 as in the element loop.
template <typename T, bool SYM>
__global__ __launch_bounds__(256) void k_convert(ChunkDev cd, char *ws, int use_scale_g) {
    __shared__ __attribute__((aligned(16))) T tt[SYM ? 64 : 1][SYM ? 72 : 1];
    const uint32_t task = xcd_task(cd.t_conv);
    if (task == NOLSM_TASK_NONE) return;
    const int s = task_slot(task), ti = task_a(task), tj = task_b(task);
    if (SYM && ti > tj) return;
    const SubMeta M = cd.meta[s];
    const SubCtl *ctl = cd.ctl + s;
    if (ctl->status != NOLSM_MOL_OK) return;
    const double c = use_scale_g ? ctl->scale_g : ctl->scale;
    const int n = M.n, np = M.np;
    T *X = (T *)(ws + M.offX0);
    const int64_t ldk = np + 64;
    if constexpr (SYM && sizeof(T) == 2) {
        if (ti < tj) {   // uniform per workgroup; every entry has r < q
            const int t = threadIdx.x;
            // both halves' loads first (the stores below may not move above them)
            double a2[2][8];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int rr = t >> 2, q0 = ((t & 3) + 4 * h) * 8;
                const int64_t off = (int64_t)(ti * 64 + rr) * ldk + tj * 64 + q0;
                double *a = a2[h];
                if (M.kf32) {
                    const float4 *p = (const float4 *)((const float *)(ws + M.offK) + off);
                    const float4 u = p[0], v = p[1];
                    a[0] = u.x; a[1] = u.y; a[2] = u.z; a[3] = u.w; a[4] = v.x; a[5] = v.y; a[6] = v.z; a[7] = v.w;
                } else {
                    const double2 *p = (const double2 *)((const double *)(ws + M.offK) + off);
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const double2 u = p[k];
                        a[2 * k] = u.x;
                        a[2 * k + 1] = u.y;
                    }
                }
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int rr = t >> 2, q0 = ((t & 3) + 4 * h) * 8;
                const int r = ti * 64 + rr, qb = tj * 64 + q0;
                const double *a = a2[h];
                uint16_t o[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const double v = (r < n && qb + k < n) ? c * a[k] : 0.0;
                    const T x = cvt<T>(v);
                    o[k] = __builtin_bit_cast(uint16_t, x);
                    tt[q0 + k][rr] = x;
                }
                *(uint4 *)(X + (int64_t)r * M.ldx + qb) =
                    make_uint4(o[0] | ((uint32_t)o[1] << 16), o[2] | ((uint32_t)o[3] << 16),
                               o[4] | ((uint32_t)o[5] << 16), o[6] | ((uint32_t)o[7] << 16));
            }
            __syncthreads();
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int qq = t >> 2, r0 = ((t & 3) + 4 * h) * 8;
                *(uint4 *)(X + (int64_t)(tj * 64 + qq) * M.ldx + ti * 64 + r0) = *(const uint4 *)&tt[qq][r0];
            }
            return;
        }
    }
    // the 16 loads of a thread first (the stores into the workspace below
    // may not move above them), then the conversions and stores
    double a[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int f = threadIdx.x + 256 * k;
        const int r = ti * 64 + (f >> 6), q = tj * 64 + (f & 63);
        const int ra = (SYM && r > q) ? q : r, qa = (SYM && r > q) ? r : q;
        a[k] = (r < n && q < n) ? kbuf_get(M, ws, (int64_t)ra * ldk + qa) : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int f = threadIdx.x + 256 * k;
        const int r = ti * 64 + (f >> 6), q = tj * 64 + (f & 63);
        const double v = (r < n && q < n) ? c * a[k] : (r == q ? 1.0 : 0.0);
        const T x = cvt<T>(v);
        X[(int64_t)r * M.ldx + q] = x;
        if constexpr (SYM) tt[f & 63][f >> 6] = x;
    }
    if constexpr (SYM) {
        if (ti == tj) return;   // uniform per workgroup
        __syncthreads();
        for (int f = threadIdx.x; f < 4096; f += 256)
            X[(int64_t)(tj * 64 + (f >> 6)) * M.ldx + ti * 64 + (f & 63)] = tt[f >> 6][f & 63];
    }
}

// init of the per-slot control blocks and residual partials of a chunk
__global__ void k_init_ctl(ChunkDev cd) {
    const int s = blockIdx.x;
    if (s >= cd.nsub) return;
    SubCtl *c = cd.ctl + s;
    if (threadIdx.x == 0) {
        c->done = 0; c->iters = 0; c->status = NOLSM_MOL_OK; c->fallback = 0; c->restart_at = -1;
        c->scale = 0; c->scale_g = 0; c->resid = 0; c->kmax = 0;
    }
    for (int i = threadIdx.x; i < NOLSM_MAX_ITER_CAP; i += blockDim.x) c->rhist[i] = 0.0;
    if (s == 0)
        for (int i = threadIdx.x; i < cd.nqueue; i += blockDim.x) cd.queues[i] = 0;
}

// ----------------------------------------------------------------- launchers
#define LAUNCH_CHECK() do { hipError_t e_ = hipGetLastError(); if (e_ != hipSuccess) return e_; } while (0)

hipError_t launch_gather(const ChunkDev &cd, char *ws, const GatherArgs &ga, hipStream_t st) {
    hipLaunchKernelGGL(k_init_ctl, dim3(cd.nsub), dim3(64), 0, st, cd);
    LAUNCH_CHECK();
    const size_t lds = (size_t)cd.max_m * 3 * sizeof(int);
    hipLaunchKernelGGL(k_gather, dim3(cd.max_m, cd.nsub), dim3(256), lds, st, cd, ws, ga);
    return hipGetLastError();
}
// Cholesky of every submatrix of the chunk, left-looking by 64-column panels:
// per panel a diagonal launch and a launch of the tiles below it.
hipError_t launch_chol(const ChunkDev &cd, char *ws, bool fp32, hipStream_t st) {
    const int pmax = cd.max_np / 64;
    for (int j = 0; j < pmax; ++j) {
        if (fp32) hipLaunchKernelGGL(k_chol_diag<float>, dim3(cd.nsub), dim3(256), 0, st, cd, ws, j);
        else hipLaunchKernelGGL(k_chol_diag<double>, dim3(cd.nsub), dim3(256), 0, st, cd, ws, j);
        LAUNCH_CHECK();
        const int rows = pmax - 1 - j;
        if (rows <= 0) continue;
        const dim3 grid(cd.nsub, (rows + CHOL_PR - 1) / CHOL_PR);
        if (fp32) hipLaunchKernelGGL((k_chol_panel<float, 3>), grid, dim3(256), 0, st, cd, ws, j);
        else hipLaunchKernelGGL((k_chol_panel<double, 2>), grid, dim3(256), 0, st, cd, ws, j);
        LAUNCH_CHECK();
    }
    return hipSuccess;
}
hipError_t launch_subst_sym(const ChunkDev &cd, char *ws, bool fp32, bool split16, hipStream_t st) {
    const bool hl = fp32 && split16;
    // split products: two row tiles per pass fit three workgroups per CU
    // without spills (faster than four at two per CU). The right solve takes
    // two row blocks per launch at two workgroups per CU (it spills a little
    // there; at one per CU without spills the phase took 32% longer); with
    // one row block per launch it read the factor twice as often and the
    // phase took 9% longer.
    if (hl) {
        hipLaunchKernelGGL((k_subst_hl<2, 3>), dim3(cd.n_subst), dim3(256), 0, st, cd, ws);
    } else if (fp32) {
        hipLaunchKernelGGL((k_subst<float, 4, 1, 3, true>), dim3(cd.n_subst), dim3(256), 0, st, cd, ws);
    } else {
        hipLaunchKernelGGL((k_subst<double, 4, 1, 2, true>), dim3(cd.n_subst), dim3(256), 0, st, cd, ws);
    }
    LAUNCH_CHECK();
    // row blocks in order: block i reads the finished blocks k < i
    const int pmax = cd.max_np / 64;
    if (hl) {
        for (int i = 0; i < pmax; i += 2) {
            hipLaunchKernelGGL((k_rsolve2_hl<2, 2>), dim3(cd.nsub), dim3(256), 0, st, cd, ws, i);
            LAUNCH_CHECK();
        }
        return hipSuccess;
    }
    for (int i = 0; i < pmax; ++i) {
        if (fp32) hipLaunchKernelGGL((k_rsolve<float, 4, 3>), dim3(cd.nsub), dim3(256), 0, st, cd, ws, i);
        else hipLaunchKernelGGL((k_rsolve<double, 4, 2>), dim3(cd.nsub), dim3(256), 0, st, cd, ws, i);
        LAUNCH_CHECK();
    }
    return hipSuccess;
}
hipError_t launch_subst(const ChunkDev &cd, char *ws, bool fp32, hipStream_t st) {
    // one column tile per task keeps enough tasks in flight (two per task
    // halved the concurrency and ran 1.7x slower); FP32 fits three
    // workgroups per CU
    if (fp32) hipLaunchKernelGGL((k_subst<float, 4, 1, 3, false>), dim3(cd.n_subst), dim3(256), 0, st, cd, ws);
    else hipLaunchKernelGGL((k_subst<double, 4, 1, 2, false>), dim3(cd.n_subst), dim3(256), 0, st, cd, ws);
    return hipGetLastError();
}
hipError_t launch_bounds(const ChunkDev &cd, char *ws, const BoundsArgs &ba, int prec, hipStream_t st) {
    hipLaunchKernelGGL(k_bounds, dim3(cd.nsub), dim3(256), 0, st, cd, ws, ba);
    LAUNCH_CHECK();
    return launch_convert(cd, ws, prec, 0, ba.sym, st);
}

hipError_t launch_convert(const ChunkDev &cd, char *ws, int prec, int use_scale_g, int sym, hipStream_t st) {
    const bool sy = sym != 0;
    switch (prec) {
        case 0: hipLaunchKernelGGL((k_convert<double, false>), dim3(cd.n_conv), dim3(256), 0, st, cd, ws, use_scale_g); break;
        case 1: hipLaunchKernelGGL((k_convert<float, false>), dim3(cd.n_conv), dim3(256), 0, st, cd, ws, use_scale_g); break;
        case 2:
            if (sy) hipLaunchKernelGGL((k_convert<_Float16, true>), dim3(cd.n_conv), dim3(256), 0, st, cd, ws, use_scale_g);
            else hipLaunchKernelGGL((k_convert<_Float16, false>), dim3(cd.n_conv), dim3(256), 0, st, cd, ws, use_scale_g);
            break;
        default:
            if (sy) hipLaunchKernelGGL((k_convert<__bf16, true>), dim3(cd.n_conv), dim3(256), 0, st, cd, ws, use_scale_g);
            else hipLaunchKernelGGL((k_convert<__bf16, false>), dim3(cd.n_conv), dim3(256), 0, st, cd, ws, use_scale_g);
            break;
    }
    return hipGetLastError();
}

// Raises the dynamic-LDS limit of the kernels whose LDS grows with the
// largest submatrix. A refusal is not an error: launches that fit the
// default limit still work, larger ones report the launch failure.
hipError_t nolsm_kernels_init() {
    (void)hipFuncSetAttribute((const void *)k_gather, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)nolsm_finish_init();
    (void)hipGetLastError();
    return hipSuccess;
}
