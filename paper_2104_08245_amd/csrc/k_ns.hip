// Newton-Schulz sign iteration on the matrix cores (Sec. III-B.2, Eq. NS1-NS2;
// Sec. III-C.3: the iteration runs as GEMMs in mixed precision).
//
// One iteration is two batched GEMM launches over the tiles of every active
// submatrix of a chunk:
//   mode 1: T = X_k X_k; epilogue: partial sums of ||T - I||_F^2 per tile and
//           R = I - T stored in the iteration precision;
//   mode 2: every workgroup of a submatrix reads the finished residual
//           r_k = ||X_k^2 - I||_F, takes the same stop/continue/restart
//           decision, and if continuing writes X_{k+1} = X_k + X_k R / 2,
//           which equals X_k (3I - X_k^2) / 2 of Eq. NS1.
// X ping-pongs between two buffers (X_k in buffer k % 2). Precisions:
// FP64 / FP32 use 64x64 tiles on v_mfma_f64_16x16x4 / v_mfma_f32_16x16x4;
// FP16 / BF16 use 128x128 (or 64x64) tiles on v_mfma_f32_32x32x16_{f16,bf16}
// with FP32 accumulation.
#include "dev_common.h"
#include "kernels.h"
#include "lp_gemm.h"

enum { ACT_STOP = 0, ACT_UPDATE = 1, ACT_RESTART = 2 };

// Decision of mode 2 at iteration `it`. Computed by thread 0 of every
// workgroup of the submatrix from data that is final before this launch
// (the residual partials of mode 1 and rhist[0..it-1]); the tile-0
// workgroup records it.
__device__ int ns_decide(const NsArgs &na, const SubMeta &M, SubCtl *ctl, const char *ws, int it,
                         int tile) {
    const double *res = (const double *)(ws + M.offRes) + (int64_t)it * M.ntile_ns;
    double ssum = 0.0;
    for (int i = 0; i < M.ntile_ns; ++i) ssum += res[i];
    const double r = sqrt(ssum);
    const double rprev = it > 0 ? ctl->rhist[it - 1] : INFINITY;
    bool stop;
    if (na.fixed_iters > 0)
        stop = it >= na.fixed_iters;
    else if (na.prec == NOLSM_FP64)
        stop = r < na.tol;
    else
        stop = (na.tol > 0.0 && r < na.tol) || (it >= 1 && r < na.rmax && r > na.theta * rprev);
    // a stall injected from the host for one molecule counts as divergence
    // at one iteration, so that the restart path can be checked (every
    // workgroup of the submatrix takes the same decision from `it` alone;
    // restart_at may already hold it + 1 from the tile-0 workgroup)
    const bool forced = na.force_stall >= 0 && M.J == na.force_stall && it == NOLSM_STALL_IT;
    const bool diverge = forced || !isfinite(r) || (it >= 1 && r > 2.0 * rprev && r > 1.0);
    const int ra = ctl->restart_at;
    int act;
    bool noconv = false;
    if (diverge && na.allow_restart && (ra < 0 || ra == it + 1)) {
        act = ACT_RESTART;
    } else if (diverge) {
        act = ACT_STOP;
        noconv = true;
    } else if (stop) {
        act = ACT_STOP;
    } else if (it + 1 >= na.max_iter) {
        act = ACT_STOP;
        noconv = na.fixed_iters <= 0;
    } else {
        act = ACT_UPDATE;
    }
    if (tile == 0) {
        ctl->rhist[it] = r;
        if (act == ACT_STOP) {
            ctl->iters = it;
            ctl->resid = r;
            // a status set earlier (NOT_SPD) is never overwritten
            if (noconv && ctl->status == NOLSM_MOL_OK) ctl->status = NOLSM_MOL_NOCONV;
            ctl->done = 1;
        } else if (act == ACT_RESTART) {
            ctl->fallback = 1;
            ctl->restart_at = it + 1;
            ctl->scale = ctl->scale_g;
        }
    }
    return act;
}

template <typename T> __device__ __forceinline__ T to_t(float x);
template <> __device__ __forceinline__ double to_t<double>(float x) { return x; }
template <> __device__ __forceinline__ float to_t<float>(float x) { return x; }
template <typename T> __device__ __forceinline__ T to_t_d(double x) { return (T)x; }

// X_{k+1} tile <- c_G A on [0,n)^2, identity on the padding (restart);
// sym: from the upper triangle of A, so that the restart is exactly symmetric
template <typename T, typename Cvt>
__device__ void restart_tile(const SubMeta &M, const SubCtl *ctl, const char *ws, T *Xn, int r0, int c0,
                             int rows, int cols, Cvt cvt, bool sym = false) {
    const int64_t ldk = M.np + 64;
    const double c = ctl->scale_g;
    for (int f = threadIdx.x; f < rows * cols; f += blockDim.x) {
        const int r = r0 + f / cols, q = c0 + f % cols;
        if (r >= M.np || q >= M.np) continue;
        const int ra = sym ? min(r, q) : r, qa = sym ? max(r, q) : q;
        const double v = (r < M.n && q < M.n) ? c * kbuf_get(M, ws, (int64_t)ra * ldk + qa) : (r == q ? 1.0 : 0.0);
        Xn[(int64_t)r * M.ldx + q] = cvt(v);
    }
}

// ------------------------------------------------------------ FP64 / FP32
template <typename T> struct Mma16;
// Output row of element e in lane group lk = l/16 (column is l%16 for both).
template <> struct Mma16<double> {
    typedef v4d acc_t;
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int e) { return lk + 4 * e; }
};
template <> struct Mma16<float> {
    typedef v4f acc_t;
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int e) { return 4 * lk + e; }
};

template <typename T>
__device__ __forceinline__ void g2s_t(T (*s)[LDP], const T *g, int64_t ld) {
    const int t = threadIdx.x;
    const int c4 = (t & 15) * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = i * 16 + (t >> 4);
        const T *p = g + (int64_t)r * ld + c4;
#pragma unroll
        for (int e = 0; e < 4; ++e) s[r][c4 + e] = p[e];
    }
}

// One 64x64 output tile of one half-iteration (body shared by the
// one-workgroup-per-tile launch and the persistent queue launch).
template <typename T>
__device__ __forceinline__ void ns64_tile(const ChunkDev &cd, uint32_t task, char *ws, const NsArgs &na, int it,
                                          int mode) {
    typedef typename Mma16<T>::acc_t acc_t;
    __shared__ T sA[64][LDP];
    __shared__ T sB[64][LDP];
    __shared__ double red[256];
    __shared__ int act_s;
    if (task == NOLSM_TASK_NONE) return;
    const int s = task_slot(task), ti = task_a(task), tj = task_b(task);
    const SubMeta M = cd.meta[s];
    SubCtl *ctl = cd.ctl + s;
    const int np = M.np, nt = np / 64, tile = ti * nt + tj;
    T *Xc = (T *)(ws + ((it & 1) ? M.offX1 : M.offX0));
    T *Xn = (T *)(ws + ((it & 1) ? M.offX0 : M.offX1));
    T *Bb = (T *)(ws + M.offB);
    // one thread reads the control state and decides for the whole workgroup
    if (threadIdx.x == 0) act_s = ctl->done ? ACT_STOP : (mode == 2 ? ns_decide(na, M, ctl, ws, it, tile) : ACT_UPDATE);
    __syncthreads();
    {
        const int act = act_s;
        if (act == ACT_STOP) return;
        if (act == ACT_RESTART) {
            restart_tile(M, ctl, ws, Xn, ti * 64, tj * 64, 64, 64, [](double v) { return (T)v; });
            return;
        }
    }
    const T *Bop = (mode == 1) ? Xc : Bb;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32;
    const int li = l & 15, lk = l >> 4;
    acc_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = (acc_t){0, 0, 0, 0};
    for (int kt = 0; kt < nt; ++kt) {
        g2s_t(sA, Xc + (int64_t)(ti * 64) * np + kt * 64, np);
        g2s_t(sB, Bop + (int64_t)(kt * 64) * np + tj * 64, np);
        __syncthreads();
#pragma unroll 4
        for (int k0 = 0; k0 < 64; k0 += 4) {
            const int k = k0 + lk;
            T a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = sA[r0 + i * 16 + li][k];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = sB[k][c0 + j * 16 + li];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = Mma16<T>::mma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
    double part = 0.0;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gr = ti * 64 + r0 + i * 16 + Mma16<T>::row(lk, e);
                const int gc = tj * 64 + c0 + j * 16 + li;
                const T v = acc[i][j][e];
                const int64_t o = (int64_t)gr * np + gc;
                if (mode == 1) {
                    // R = I - X^2; the update below is X + X R / 2 = X (3I - X^2) / 2
                    const T rr = (gr == gc ? (T)1 : (T)0) - v;
                    part += (double)rr * (double)rr;
                    Bb[o] = rr;
                } else {
                    Xn[o] = Xc[o] + (T)0.5 * v;
                }
            }
    if (mode == 1) {
        const double sum = block_sum(part, red);
        if (threadIdx.x == 0) ((double *)(ws + M.offRes))[(int64_t)it * M.ntile_ns + tile] = sum;
    }
}

// Persistent launches: a fixed grid whose workgroups pop entries from the
// task-list segment of their XCD through an atomic counter (one counter per
// XCD, per launch, zeroed at chunk start). No workgroup ever waits for
// another one, so every wave exits once its segment is drained.
__device__ __forceinline__ int queue_pop(int *q, int *slot) {
    __syncthreads();
    if (threadIdx.x == 0) *slot = atomicAdd(q, 1);
    __syncthreads();
    return *slot;
}

template <typename T>
__global__ __launch_bounds__(256) void k_ns64(ChunkDev cd, char *ws, NsArgs na, int it, int mode) {
    ns64_tile<T>(cd, xcd_task(cd.t_ns), ws, na, it, mode);
}

template <typename T>
__global__ __launch_bounds__(256) void k_ns64_pq(ChunkDev cd, int ntask, int *q, char *ws, NsArgs na, int it,
                                                 int mode) {
    __shared__ int idx_s;
    const int x = blockIdx.x & 7, seg = ntask >> 3;
    for (;;) {
        const int i = queue_pop(q + x, &idx_s);
        if (i >= seg) break;
        ns64_tile<T>(cd, cd.t_ns[x * seg + i], ws, na, it, mode);
    }
}

// ------------------------------------------------------------ FP16 / BF16
// Symmetric sign iteration: the output tile (16-bit values) is staged
// transposed in the operand LDS of lp_tile_product (free once it returns):
// BM rows of BM values, 16-byte chunks swizzled by row, entry (r, c) of the
// tile at row c, column r. Each lane holds 4 consecutive rows of one column
// per group of 4 accumulator elements: one 8-byte store each.
template <int BM> __device__ __forceinline__ int sym_idx(int row, int col) {
    return row * BM + ((((col >> 3) ^ row ^ (row >> 3)) & (BM / 8 - 1)) << 3) + (col & 7);
}
template <int BM, typename Val> __device__ __forceinline__ void sym_stage(Val val) {
    constexpr int WT = BM / 2, NB = WT / 32;
    uint16_t *st = lp_lds<BM>();
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, wm = w >> 1, wn = w & 1;
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int rl = wm * WT + i * 32 + q * 8 + (l >> 5) * 4, cl = wn * WT + j * 32 + (l & 31);
                const uint32_t lo = (uint32_t)val(i, j, 4 * q) | ((uint32_t)val(i, j, 4 * q + 1) << 16);
                const uint32_t hi = (uint32_t)val(i, j, 4 * q + 2) | ((uint32_t)val(i, j, 4 * q + 3) << 16);
                *(uint2 *)(st + sym_idx<BM>(cl, rl)) = make_uint2(lo, hi);
            }
}
// off-diagonal tile (ti, tj): its transpose goes to tile (tj, ti), 16-byte
// row stores from the staged copy
template <int BM> __device__ __forceinline__ void sym_store_mirror(uint16_t *X, int ldx, int row0, int col0) {
    constexpr int NCH = BM / 8;
    const uint16_t *st = lp_lds<BM>();
    for (int f = threadIdx.x; f < BM * NCH; f += 256) {
        const int cl = f / NCH, ch = f % NCH;
        *(uint4 *)(X + (int64_t)(col0 + cl) * ldx + row0 + ch * 8) = *(const uint4 *)(st + sym_idx<BM>(cl, ch * 8));
    }
}
// off-diagonal tile (ti, tj) itself from the staged copy of its transpose:
// each thread reads an 8 x 8 block (eight 16-byte reads of copy rows),
// transposes it in registers and writes eight 16-byte row segments, so the
// 16 threads of a block row store 256 contiguous bytes of each tile row
// (the row ^ (row >> 3) term of sym_idx spreads the eight copy rows a
// block read touches, 8 apart, over all chunk positions)
template <int BM> __device__ __forceinline__ void sym_store_direct(uint16_t *X, int ldx, int row0, int col0) {
    constexpr int NB8 = BM / 8;
    const uint16_t *st = lp_lds<BM>();
    for (int b = threadIdx.x; b < NB8 * NB8; b += 256) {
        const int r0 = (b / NB8) * 8, c0 = (b % NB8) * 8;
        uint4 v[8];   // v[q] = T[r0 .. r0 + 7][c0 + q]
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = *(const uint4 *)(st + sym_idx<BM>(c0 + q, r0));
        auto dw = [](const uint4 &x, int d) { return d == 0 ? x.x : d == 1 ? x.y : d == 2 ? x.z : x.w; };
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            uint32_t o[4];
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const uint32_t a = dw(v[2 * d], p >> 1), c = dw(v[2 * d + 1], p >> 1);
                o[d] = (p & 1) ? ((a >> 16) | (c & 0xFFFF0000u)) : ((a & 0xFFFFu) | (c << 16));
            }
            *(uint4 *)(X + (int64_t)(row0 + r0 + p) * ldx + col0 + c0) = make_uint4(o[0], o[1], o[2], o[3]);
        }
    }
}
// A BM x BM tile of X_k into LDS as it stands (16-byte row loads), the
// 16-byte chunk c of row r at chunk position c ^ 4 ((r / 4) % (BM / 32)):
// the accumulator-layout reads (32 consecutive columns of one row, and of
// the row 4 below) then fall on distinct banks
template <int BM> __device__ __forceinline__ int dir_idx(int r, int c) {
    return r * BM + ((((c >> 3) ^ (((r >> 2) & (BM / 32 - 1)) << 2))) << 3) + (c & 7);
}
template <int BM> __device__ __forceinline__ void dir_load(const uint16_t *X, int ldx, int row0, int col0) {
    constexpr int NCH = BM / 8, NQ = BM * NCH / 256;
    uint16_t *st = lp_lds<BM>();
    uint4 v[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int f = threadIdx.x + q * 256, r = f / NCH, ch = f % NCH;
        v[q] = *(const uint4 *)(X + (int64_t)(row0 + r) * ldx + col0 + ch * 8);
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int f = threadIdx.x + q * 256, r = f / NCH, ch = f % NCH;
        *(uint4 *)(st + dir_idx<BM>(r, ch * 8)) = v[q];
    }
}
// diagonal tile: X R (and X X^T up to rounding) is symmetric only in exact
// arithmetic, and an iteration whose B operand is read as rows (X^T) doubles
// the skew part that anticommutes with the sign at every step. The tile is
// written exactly symmetric, from its upper triangle: (r, c) takes T[r][c]
// for r <= c and T[c][r] below (staged copy: T[r][c] at row c, column r).
template <int BM> __device__ __forceinline__ void sym_store_diag(uint16_t *X, int ldx, int row0) {
    constexpr int NCH = BM / 8;
    const uint16_t *st = lp_lds<BM>();
    for (int f = threadIdx.x; f < BM * NCH; f += 256) {
        const int r = f / NCH, c0 = (f % NCH) * 8;
        uint4 v;
        if (c0 + 7 < r) {
            v = *(const uint4 *)(st + sym_idx<BM>(r, c0));   // T[c][r], c < r: row r of the copy
        } else {
            uint16_t h[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int c = c0 + k;
                h[k] = (r <= c) ? st[sym_idx<BM>(c, r)] : st[sym_idx<BM>(r, c)];
            }
            v = make_uint4(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16), h[4] | ((uint32_t)h[5] << 16),
                           h[6] | ((uint32_t)h[7] << 16));
        }
        *(uint4 *)(X + (int64_t)(row0 + r) * ldx + row0 + c0) = v;
    }
}

// One BM x BM tile of a sign-iteration GEMM: mode 1 forms R = I - X_k^2 and
// the tile's share of ||R||_F^2, mode 2 decides stop / continue / restart and
// forms X_{k+1} = X_k + X_k R / 2. SYM: X_k and R are symmetric, only tiles
// ti <= tj are launched and each writes its mirror too.
// DIAG1: the diagonal tiles of X_k^2 take the one-operand product (kept out
// of the persistent kernel, whose loop would spill with both copies inlined)
template <typename T, int BM, bool SYM, bool DIAG1 = false>
__device__ __forceinline__ void ns_lp_tile(const ChunkDev &cd, uint32_t task, char *ws, const NsArgs &na, int it,
                                           int mode) {
    __shared__ double red[256];
    __shared__ int act_s;
    if (task == NOLSM_TASK_NONE) return;
    const int s = task_slot(task), ti = task_a(task), tj = task_b(task);
    const SubMeta M = cd.meta[s];
    SubCtl *ctl = cd.ctl + s;
    const int np = M.np, nt = (np + BM - 1) / BM, tile = ti * nt + tj;
    uint16_t *Xc = (uint16_t *)(ws + ((it & 1) ? M.offX1 : M.offX0));
    uint16_t *Xn = (uint16_t *)(ws + ((it & 1) ? M.offX0 : M.offX1));
    uint16_t *Bb = (uint16_t *)(ws + M.offB);
    // one thread reads the control state and decides for the whole workgroup
    if (threadIdx.x == 0) act_s = ctl->done ? ACT_STOP : (mode == 2 ? ns_decide(na, M, ctl, ws, it, tile) : ACT_UPDATE);
    __syncthreads();
    {
        const int act = act_s;
        if (act == ACT_STOP) return;
        if (act == ACT_RESTART) {
            restart_tile(M, ctl, ws, Xn, ti * BM, tj * BM, BM, BM, [](double v) { return Lp<T>::enc((float)v); },
                         SYM);
            if (SYM && ti != tj)
                restart_tile(M, ctl, ws, Xn, tj * BM, ti * BM, BM, BM, [](double v) { return Lp<T>::enc((float)v); },
                             SYM);
            return;
        }
    }
    constexpr int WT = BM / 2, NB = WT / 32;
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, wm = w >> 1, wn = w & 1;
    const int row0 = ti * BM, col0 = tj * BM, ldx = M.ldx;
    const int nrec = ldx * ldx * 2;
    v16f acc[NB][NB];
    // a diagonal tile of X_k^2 (symmetric route) loads its one operand tile once
    if (DIAG1 && SYM && mode == 1 && ti == tj) lp_tile_product<T, BM, SYM, DIAG1 && SYM>(Xc, Xc, ldx, np, row0, col0, acc);
    else lp_tile_product<T, BM, SYM>(Xc, (mode == 1) ? Xc : Bb, ldx, np, row0, col0, acc);
    // Epilogue over the whole tile, padding included: rows and columns in
    // [np, ldx) of R and X_{k+1} only ever feed outputs that are never used,
    // so the accesses need no bounds test and the X_k reads of the update
    // are issued together rather than one guarded load at a time.
    // element e of block (i, j) sits (i * 32 + (e / 4) * 8 + e % 4) rows and
    // j * 32 columns from the lane's base: a uniform offset per element
    const int er0 = row0 + wm * WT + (l >> 5) * 4, ec0 = col0 + wn * WT + (l & 31);
    const uint32_t eo = (uint32_t)((er0 * ldx + ec0) * 2);
#define NS_EOFF(i, j, e) ((((i) * 32 + ((e) >> 2) * 8 + ((e) & 3)) * ldx + (j) * 32) * 2)
    if constexpr (SYM) {
        // every value is formed first and staged in LDS behind one barrier,
        // and all global stores come after it: a barrier behind stores
        // would wait for them to complete
        uint16_t *Out;
        if (mode == 1) {
            double part = 0.0;
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j)
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        const int gr = er0 + i * 32 + (e >> 2) * 8 + (e & 3), gc = ec0 + j * 32;
                        acc[i][j][e] = (gr == gc ? 1.0f : 0.0f) - acc[i][j][e];   // R
                        if (gr < np && gc < np) part += (double)acc[i][j][e] * (double)acc[i][j][e];
                    }
            const double sum = block_sum(part, red);
            if (threadIdx.x == 0) {
                double *res = (double *)(ws + M.offRes) + (int64_t)it * M.ntile_ns;
                res[tile] = (ti != tj ? 2.0 : 1.0) * sum;   // the mirror tile is never launched
                if (ti != tj) res[tj * nt + ti] = 0.0;
            }
            Out = Bb;
        } else {
            // X_k of the tile through LDS (the operand buffers are free
            // again): 16-byte row loads, then each lane's elements
            dir_load<BM>(Xc, ldx, row0, col0);
            __syncthreads();
            const uint16_t *xs = lp_lds<BM>();
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j)
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        const int rl = wm * WT + i * 32 + (e >> 2) * 8 + (l >> 5) * 4 + (e & 3);
                        const int cl = wn * WT + j * 32 + (l & 31);
                        acc[i][j][e] = Lp<T>::dec(xs[dir_idx<BM>(rl, cl)]) + 0.5f * acc[i][j][e];
                    }
            __syncthreads();
            Out = Xn;
        }
        sym_stage<BM>([&](int i, int j, int e) { return Lp<T>::enc(acc[i][j][e]); });
        __syncthreads();
        if (ti != tj) {
            sym_store_direct<BM>(Out, ldx, row0, col0);
            sym_store_mirror<BM>(Out, ldx, row0, col0);
        } else {
            sym_store_diag<BM>(Out, ldx, row0);
        }
    } else if (mode == 1) {
        const __amdgpu_buffer_rsrc_t rsR = __builtin_amdgcn_make_buffer_rsrc((void *)Bb, (short)0, nrec, 0x00020000);
        double part = 0.0;
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j)
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int gr = er0 + i * 32 + (e >> 2) * 8 + (e & 3), gc = ec0 + j * 32;
                    // R = I - X^2 is small near convergence and keeps full
                    // relative precision in 16 bits (3I - X^2 would not: its
                    // diagonal ~2 is quantised at 2^-9 in FP16)
                    const float rr = (gr == gc ? 1.0f : 0.0f) - acc[i][j][e];
                    __builtin_amdgcn_raw_buffer_store_b16(Lp<T>::enc(rr), rsR, eo, NS_EOFF(i, j, e), 0);
                    if (gr < np && gc < np) part += (double)rr * (double)rr;
                }
        const double sum = block_sum(part, red);
        if (threadIdx.x == 0) ((double *)(ws + M.offRes))[(int64_t)it * M.ntile_ns + tile] = sum;
    } else {
        const __amdgpu_buffer_rsrc_t rsX = __builtin_amdgcn_make_buffer_rsrc((void *)Xc, (short)0, nrec, 0x00020000);
        const __amdgpu_buffer_rsrc_t rsN = __builtin_amdgcn_make_buffer_rsrc((void *)Xn, (short)0, nrec, 0x00020000);
        // X_{k+1} = X_k + X_k R / 2 = X_k (3I - X_k^2) / 2, one block at a time
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                uint16_t xo[16];
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    xo[e] = __builtin_amdgcn_raw_buffer_load_b16(rsX, eo, NS_EOFF(i, j, e), 0);
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    __builtin_amdgcn_raw_buffer_store_b16(Lp<T>::enc(Lp<T>::dec(xo[e]) + 0.5f * acc[i][j][e]), rsN,
                                                          eo, NS_EOFF(i, j, e), 0);
            }
    }
#undef NS_EOFF
}

template <typename T, int BM, bool SYM>
__global__ __launch_bounds__(256, 3) void k_ns_lp(ChunkDev cd, const uint32_t *tasks, char *ws, NsArgs na, int it,
                                               int mode) {
    ns_lp_tile<T, BM, SYM, true>(cd, xcd_task(tasks), ws, na, it, mode);
}

template <typename T, int BM, bool SYM>
__global__ __launch_bounds__(256, 3) void k_ns_lp_pq(ChunkDev cd, const uint32_t *tasks, int ntask, int *q, char *ws,
                                                  NsArgs na, int it, int mode) {
    __shared__ int idx_s;
    const int x = blockIdx.x & 7, seg = ntask >> 3;
    for (;;) {
        const int i = queue_pop(q + x, &idx_s);
        if (i >= seg) break;
        ns_lp_tile<T, BM, SYM>(cd, tasks[x * seg + i], ws, na, it, mode);
    }
}

// Late iterations, when most submatrices have converged: a small grid in
// which every workgroup scans its share of its XCD's task segment, 256
// tasks at a time (one per thread), keeps the tasks whose submatrix is still
// iterating and runs those tiles. A launch after convergence then costs one
// scan instead of one dispatched workgroup per tile. The order in which the
// kept tiles run does not matter: each writes only its own outputs.
template <typename T, int BM, bool SYM>
__global__ __launch_bounds__(256, 2) void k_ns_lp_tail(ChunkDev cd, const uint32_t *tasks, int ntask, char *ws,
                                                    NsArgs na, int it, int mode) {
    __shared__ uint32_t kept[256];
    __shared__ int nkept;
    const int x = blockIdx.x & 7, seg = ntask >> 3, g8 = gridDim.x >> 3, wb = blockIdx.x >> 3;
    const int span = (seg + g8 - 1) / g8, lo = wb * span, hi = min(seg, lo + span);
    for (int i0 = lo; i0 < hi; i0 += 256) {
        if (threadIdx.x == 0) nkept = 0;
        __syncthreads();
        const int i = i0 + (int)threadIdx.x;
        if (i < hi) {
            const uint32_t task = tasks[x * seg + i];
            if (task != NOLSM_TASK_NONE && !cd.ctl[task_slot(task)].done) kept[atomicAdd(&nkept, 1)] = task;
        }
        __syncthreads();
        const int nk = nkept;
        for (int k = 0; k < nk; ++k) ns_lp_tile<T, BM, SYM>(cd, kept[k], ws, na, it, mode);
        __syncthreads();
    }
}
// iterations from this one on take the scanning launch
#define NS_TAIL_IT 16

// queue counters of one launch: [iteration][half][tile class][XCD]
static int *launch_queue(const ChunkDev &cd, int it, int mode, int cls) {
    return cd.queues + (((size_t)it * 2 + (mode - 1)) * 2 + cls) * 8;
}
static int persistent_grid(const NsArgs &na, int ntask) {
    int g = na.pgrid < ntask ? na.pgrid : ntask;
    g = (g + 7) / 8 * 8;
    return g < 8 ? 8 : g;
}

template <typename T, bool SYM>
static void launch_lp(const ChunkDev &cd, char *ws, const NsArgs &na, int it, int mode, hipStream_t st) {
    if (na.persistent) {
        if (cd.n_ns > 0)
            hipLaunchKernelGGL((k_ns_lp_pq<T, 128, SYM>), dim3(persistent_grid(na, cd.n_ns)), dim3(256), 0, st, cd,
                               cd.t_ns, cd.n_ns, launch_queue(cd, it, mode, 0), ws, na, it, mode);
        if (cd.n_ns64 > 0)
            hipLaunchKernelGGL((k_ns_lp_pq<T, 64, SYM>), dim3(persistent_grid(na, cd.n_ns64)), dim3(256), 0, st, cd,
                               cd.t_ns64, cd.n_ns64, launch_queue(cd, it, mode, 1), ws, na, it, mode);
        return;
    }
    if (it >= NS_TAIL_IT) {
        // four scanning workgroups per CU (2 x pgrid), at most one per task
        auto grid = [&](int ntask) {
            const int g = (2 * na.pgrid < ntask ? 2 * na.pgrid : ntask) / 8 * 8;
            return g < 8 ? 8 : g;
        };
        if (cd.n_ns > 0)
            hipLaunchKernelGGL((k_ns_lp_tail<T, 128, SYM>), dim3(grid(cd.n_ns)), dim3(256), 0, st, cd, cd.t_ns,
                               cd.n_ns, ws, na, it, mode);
        if (cd.n_ns64 > 0)
            hipLaunchKernelGGL((k_ns_lp_tail<T, 64, SYM>), dim3(grid(cd.n_ns64)), dim3(256), 0, st, cd, cd.t_ns64,
                               cd.n_ns64, ws, na, it, mode);
        return;
    }
    if (cd.n_ns > 0)
        hipLaunchKernelGGL((k_ns_lp<T, 128, SYM>), dim3(cd.n_ns), dim3(256), 0, st, cd, cd.t_ns, ws, na, it, mode);
    if (cd.n_ns64 > 0)
        hipLaunchKernelGGL((k_ns_lp<T, 64, SYM>), dim3(cd.n_ns64), dim3(256), 0, st, cd, cd.t_ns64, ws, na, it, mode);
}

template <typename T>
static void launch_64(const ChunkDev &cd, char *ws, const NsArgs &na, int it, int mode, hipStream_t st) {
    if (cd.n_ns <= 0) return;
    if (na.persistent)
        hipLaunchKernelGGL(k_ns64_pq<T>, dim3(persistent_grid(na, cd.n_ns)), dim3(256), 0, st, cd, cd.n_ns,
                           launch_queue(cd, it, mode, 0), ws, na, it, mode);
    else
        hipLaunchKernelGGL(k_ns64<T>, dim3(cd.n_ns), dim3(256), 0, st, cd, ws, na, it, mode);
}

hipError_t launch_ns_iter(const ChunkDev &cd, char *ws, const NsArgs &na, int it, hipStream_t st) {
    for (int mode = 1; mode <= 2; ++mode) {
        switch (na.prec) {
            case NOLSM_FP64: launch_64<double>(cd, ws, na, it, mode, st); break;
            case NOLSM_FP32: launch_64<float>(cd, ws, na, it, mode, st); break;
            case NOLSM_FP16:
                if (na.sym) launch_lp<_Float16, true>(cd, ws, na, it, mode, st);
                else launch_lp<_Float16, false>(cd, ws, na, it, mode, st);
                break;
            default:
                if (na.sym) launch_lp<__bf16, true>(cd, ws, na, it, mode, st);
                else launch_lp<__bf16, false>(cd, ws, na, it, mode, st);
                break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
