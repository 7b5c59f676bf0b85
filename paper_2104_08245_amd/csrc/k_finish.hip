// Finishing iterations, extraction of the owned columns, traces, write-back.
//
// Only the owned columns of T_J(D) are needed (Sec. III-B.2, write-back step):
//   T_J(D)[:, cJ] = (Y_J - sign(A_J) Y_J) / 2,   Y_J = T_J(S)^-1 E_cJ.
// With the low-precision iterate P = X_K, f further Newton-Schulz steps
// (Eq. NS1) applied only to the n x bs block Y_J are exact rewrites of full
// FP32 iterations:
//   X_{K+1} v = (3 P v - P^3 v) / 2,   X_{K+2} Y = (3 w1 - w3) / 2 with
//   w1 = X_{K+1} Y, w3 = X_{K+1}^2 w1,
// i.e. 3^f products of P with n x bs blocks ("column-restricted" finishing,
// O(n^2) work instead of full GEMMs).
#include "dev_common.h"
#include "kernels.h"

struct SkinnyArgs {
    int32_t ina, inb;      // input vectors (index, -1 = Y_J, -2 = none)
    double alpha, beta;    // in = alpha * ina + beta * inb
    int32_t out;           // output vector index
    int32_t save;          // if >= 0: also store `in` (this workgroup's rows)
};

template <typename TP> struct Dec;
template <> struct Dec<double> { typedef double storage; static __device__ __forceinline__ double get(double x) { return x; } };
template <> struct Dec<float> { typedef float storage; static __device__ __forceinline__ float get(float x) { return x; } };
struct F16 {};
struct BF16 {};
template <> struct Dec<F16> {
    typedef uint16_t storage;
    static __device__ __forceinline__ float get(uint16_t x) { return (float)__builtin_bit_cast(_Float16, x); }
};
template <> struct Dec<BF16> {
    typedef uint16_t storage;
    static __device__ __forceinline__ float get(uint16_t x) { return (float)__builtin_bit_cast(__bf16, x); }
};

#define BSMAX 6

// Input block of the products for owned molecule o: Y_J (its bs columns of
// the K buffer) or a combination of its stored vectors.
template <typename TV>
__device__ __forceinline__ TV vec_in(const SkinnyArgs &a, const SubMeta &M, const char *ws, int o, int bs, int row,
                                     int j) {
    const int np = M.np;
    const int64_t vs = (int64_t)np * 6 * 8 / sizeof(TV);   // stride between vectors
    const TV *V = (const TV *)(ws + M.offVec) + (int64_t)o * NOLSM_NVEC * vs;
    auto get = [&](int idx) -> TV {
        if (idx == -1) return (TV)kbuf_get(M, ws, (int64_t)row * (np + 64) + np + o * bs + j);
        return V[(int64_t)idx * vs + (int64_t)row * 6 + j];
    };
    TV v = (TV)a.alpha * get(a.ina);
    if (a.inb >= -1) v += (TV)a.beta * get(a.inb);
    return v;
}

// out = P * in for 256 rows per workgroup, one row per lane, one workgroup
// per (row block, owned molecule). The input block (n x bs, formed from up to
// two stored vectors) is staged once per workgroup in LDS and read as a
// broadcast; each lane streams its row of P with 16-byte loads, so the kernel
// is a plain HBM stream of P. The owned molecules of one row block are
// adjacent in the task list and share P through the L2 of their XCD.
// Dynamic LDS: max_np x 6 values of TV.
template <typename TP, typename TV>
__global__ __launch_bounds__(256) void k_skinny(ChunkDev cd, char *ws, SkinnyArgs sa, int bs) {
    typedef typename Dec<TP>::storage ST;
    constexpr int EPL = 16 / (int)sizeof(ST);   // elements per 16-byte load
    extern __shared__ __attribute__((aligned(16))) char skm[];
    TV *vin = (TV *)skm;
    const uint32_t task = xcd_task(cd.t_rows);
    if (task == NOLSM_TASK_NONE) return;
    const int s = task_slot(task), rq = task_a(task), o = task_b(task);
    const SubMeta M = cd.meta[s];
    const SubCtl *ctl = cd.ctl + s;
    if (ctl->status == NOLSM_MOL_NOT_SPD) return;
    const int np = M.np, t = threadIdx.x;
    const int K = ctl->iters;
    const ST *P = (const ST *)(ws + ((K & 1) ? M.offX1 : M.offX0));
    const int64_t vs = (int64_t)np * 6 * 8 / sizeof(TV);
    TV *V = (TV *)(ws + M.offVec) + (int64_t)o * NOLSM_NVEC * vs;
    for (int f = t; f < np * 6; f += 256) {
        const int r = f / 6, j = f - r * 6;
        vin[f] = (j < bs) ? vec_in<TV>(sa, M, ws, o, bs, r, j) : (TV)0;
    }
    __syncthreads();
    const int row = rq * 256 + t;
    if (row >= np) return;   // np is a multiple of 64: whole waves leave
    if (sa.save >= 0)
        for (int j = 0; j < bs; ++j) V[(int64_t)sa.save * vs + (int64_t)row * 6 + j] = vin[row * 6 + j];
    const ST *prow = P + (int64_t)row * M.ldx;
    TV acc[BSMAX];
#pragma unroll
    for (int j = 0; j < BSMAX; ++j) acc[j] = 0;
#pragma unroll 4
    for (int c = 0; c < np; c += EPL) {
        const uint4 raw = *(const uint4 *)(prow + c);
        const ST *pe = (const ST *)&raw;
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
            const TV p = (TV)Dec<TP>::get(pe[e]);
            const TV *vi = vin + (c + e) * 6;
#pragma unroll
            for (int j = 0; j < BSMAX; ++j) acc[j] += p * vi[j];
        }
    }
#pragma unroll
    for (int j = 0; j < BSMAX; ++j)
        if (j < bs) V[(int64_t)sa.out * vs + (int64_t)row * 6 + j] = acc[j];
}

template <typename TP, typename TV>
static hipError_t run_finish(const ChunkDev &cd, char *ws, int nfinal, int bs, hipStream_t st) {
    auto L = [&](int ina, int inb, double al, double be, int out, int save) {
        SkinnyArgs a{ina, inb, al, be, out, save};
        hipLaunchKernelGGL((k_skinny<TP, TV>), dim3(cd.n_rows), dim3(256),
                           (size_t)cd.max_np * 6 * sizeof(TV), st, cd, ws, a, bs);
        return hipGetLastError();
    };
    hipError_t e;
    if ((e = L(-1, -2, 1.0, 0.0, 0, -1))) return e;              // u1 = P Y
    if (nfinal == 0) return hipSuccess;
    if ((e = L(0, -2, 1.0, 0.0, 1, -1))) return e;               // u2 = P u1
    if ((e = L(1, -2, 1.0, 0.0, 2, -1))) return e;               // u3 = P u2
    if (nfinal == 1) return hipSuccess;                          // w1 = (3u1 - u3)/2
    if ((e = L(0, 2, 1.5, -0.5, 4, 3))) return e;                // p1 = P w1, save w1
    if ((e = L(4, -2, 1.0, 0.0, 5, -1))) return e;               // p2
    if ((e = L(5, -2, 1.0, 0.0, 6, -1))) return e;               // p3
    if ((e = L(4, 6, 1.5, -0.5, 8, 7))) return e;                // q1 = P w2, save w2
    if ((e = L(8, -2, 1.0, 0.0, 9, -1))) return e;               // q2
    if ((e = L(9, -2, 1.0, 0.0, 10, -1))) return e;              // q3
    return hipSuccess;                                           // Z = 1.5 w1 - 0.75 q1 + 0.25 q3
}

// ---------------------------------------------------------------------------
// FP16 finishing fused on the matrix cores: one workgroup per (submatrix,
// owned molecule) runs all the products above in order. P is exact in FP16;
// each input block v (n x bs, FP32) is split into FP16 parts h = fp16(v) and
// l = fp16(v - h), which hold 22 of its 24 bits (the rest is below 2^-22
// relative, absolute below 2^-24 times the FP16 subnormal scale), and
// P [h | l | 0] is one n x 16 product on v_mfma_f32_16x16x32_f16 with FP32
// accumulation; P v = P h + P l. The B operand [h | l | 0] sits in LDS as 16
// rows of np + 8 values (the pad spreads the 16 rows a wave reads over all
// banks); A is read straight from P, a 16-byte row segment per lane. The
// workgroup (16 waves) holds at least 96 KB of LDS so that one runs per CU:
// the 256 submatrices in flight then keep their P (0.8 MB each at n ~ 640)
// in the 256 MB last-level cache across the nine products, where more
// workgroups per CU would re-read it from HBM.
// ---------------------------------------------------------------------------
#define FIN_THREADS 1024
#define FIN_LDS_MIN (96 * 1024)
typedef float v4f_fin __attribute__((ext_vector_type(4)));

struct FinStep { int8_t ina, inb, out, save; float alpha, beta; };
// u1 = P y, u2 = P u1, u3 = P u2, w1 = 1.5 u1 - 0.5 u3 (saved), p1 = P w1,
// p2, p3, w2 = 1.5 p1 - 0.5 p3 (saved), q1 = P w2, q2, q3: the sequence of
// run_finish, same vector slots
__constant__ FinStep fin_steps[9] = {{-1, -2, 0, -1, 1.0f, 0.0f}, {0, -2, 1, -1, 1.0f, 0.0f},
                                     {1, -2, 2, -1, 1.0f, 0.0f},  {0, 2, 4, 3, 1.5f, -0.5f},
                                     {4, -2, 5, -1, 1.0f, 0.0f},  {5, -2, 6, -1, 1.0f, 0.0f},
                                     {4, 6, 8, 7, 1.5f, -0.5f},   {8, -2, 9, -1, 1.0f, 0.0f},
                                     {9, -2, 10, -1, 1.0f, 0.0f}};

__global__ __launch_bounds__(FIN_THREADS, 1) void k_finish_f16(ChunkDev cd, char *ws, int nsteps, int bs) {
    extern __shared__ __attribute__((aligned(16))) uint16_t vb[];   // [16][np + 8]
    const int s = blockIdx.x, o = blockIdx.y;
    if (s >= cd.nsub) return;
    const SubMeta M = cd.meta[s];
    const SubCtl *ctl = cd.ctl + s;
    if (o >= M.nown || ctl->status == NOLSM_MOL_NOT_SPD) return;
    const int np = M.np, ldb = np + 8, ldx = M.ldx, t = threadIdx.x, w = t >> 6, l = t & 63;
    const uint16_t *P = (const uint16_t *)(ws + ((ctl->iters & 1) ? M.offX1 : M.offX0));
    const int64_t vs = (int64_t)np * 12;   // floats per vector slot (np x 6 doubles reserved)
    float *V = (float *)(ws + M.offVec) + (int64_t)o * NOLSM_NVEC * vs;
    for (int f = t; f < 4 * ldb; f += FIN_THREADS) vb[12 * ldb + f] = 0;   // columns 12..15 of B
    for (int step = 0; step < nsteps; ++step) {
        const FinStep S = fin_steps[step];
        // input block, split into its FP16 high and low parts
        for (int f = t; f < np * 6; f += FIN_THREADS) {
            const int r = f / 6, j = f - r * 6;
            float v = 0.0f;
            if (j < bs) {
                auto get = [&](int idx) -> float {
                    if (idx == -1) return (float)kbuf_get(M, ws, (int64_t)r * (np + 64) + np + o * bs + j);
                    return V[(int64_t)idx * vs + (int64_t)r * 6 + j];
                };
                v = S.alpha * get(S.ina);
                if (S.inb >= -1) v += S.beta * get(S.inb);
                if (S.save >= 0) V[(int64_t)S.save * vs + (int64_t)r * 6 + j] = v;
            }
            const _Float16 h = (_Float16)v;
            const _Float16 lo = (_Float16)(v - (float)h);
            vb[j * ldb + r] = __builtin_bit_cast(uint16_t, h);
            vb[(6 + j) * ldb + r] = __builtin_bit_cast(uint16_t, lo);
        }
        __syncthreads();
        // out = P [h | l | 0], 16 rows per block: lane l holds A row l % 16,
        // k = 8 (l / 16) .. + 7 of each 32-deep step, B column l % 16 of the
        // same k, and the results of rows 4 (l / 16) + e, column l % 16
        const int nb = np >> 4;
        const uint16_t *brow = vb + (l & 15) * ldb + (l >> 4) * 8;
        // two row blocks per wave at a time (the second may be past the
        // end: its rows are clamped to the first block and not stored), two
        // accumulators each over k (np is a multiple of 64): eight 16-byte
        // row segments of P in flight per lane
        for (int rb = w; rb < nb; rb += 2 * (FIN_THREADS / 64)) {
            const int rb2 = rb + FIN_THREADS / 64;
            const bool two = rb2 < nb;
            v4f_fin c00 = {0.0f, 0.0f, 0.0f, 0.0f}, c01 = c00, c10 = c00, c11 = c00;
            const uint16_t *a0row = P + (int64_t)(rb * 16 + (l & 15)) * ldx + (l >> 4) * 8;
            const uint16_t *a1row = P + (int64_t)((two ? rb2 : rb) * 16 + (l & 15)) * ldx + (l >> 4) * 8;
            for (int k0 = 0; k0 < np; k0 += 64) {
                const v8h a00 = *(const v8h *)(a0row + k0);
                const v8h a01 = *(const v8h *)(a0row + k0 + 32);
                const v8h a10 = *(const v8h *)(a1row + k0);
                const v8h a11 = *(const v8h *)(a1row + k0 + 32);
                const v8h b0 = *(const v8h *)(brow + k0);
                const v8h b1 = *(const v8h *)(brow + k0 + 32);
                c00 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a00, b0, c00, 0, 0, 0);
                c01 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a01, b1, c01, 0, 0, 0);
                c10 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a10, b0, c10, 0, 0, 0);
                c11 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a11, b1, c11, 0, 0, 0);
            }
            c00 += c01;
            c10 += c11;
            // column j + 6 holds P l of column j: lanes of columns 0..5 add it
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float p0 = __shfl(c00[e], l + 6), p1 = __shfl(c10[e], l + 6);
                const int r = (l >> 4) * 4 + e, j = l & 15;
                if (j < bs) {
                    V[(int64_t)S.out * vs + (int64_t)(rb * 16 + r) * 6 + j] = c00[e] + p0;
                    if (two) V[(int64_t)S.out * vs + (int64_t)(rb2 * 16 + r) * 6 + j] = c10[e] + p1;
                }
            }
        }
        __syncthreads();
    }
}

int finish_launches(const FinishArgs &fa) {
    const int products = fa.nfinal == 0 ? 1 : (fa.nfinal == 1 ? 3 : 9);
    return (fa.prec == NOLSM_FP16 && !fa.rows) ? 1 : products;
}

hipError_t launch_finish(const ChunkDev &cd, char *ws, const FinishArgs &fa, hipStream_t st) {
    const int bs = 6;
    switch (fa.prec) {
        case NOLSM_FP64: return run_finish<double, double>(cd, ws, 0, bs, st);
        case NOLSM_FP32: return run_finish<float, float>(cd, ws, 0, bs, st);
        case NOLSM_FP16:
            if (!fa.rows) {
                size_t lds = (size_t)16 * (cd.max_np + 8) * 2;
                if (lds < FIN_LDS_MIN) lds = FIN_LDS_MIN;
                const int nsteps = fa.nfinal == 0 ? 1 : (fa.nfinal == 1 ? 3 : 9);
                hipLaunchKernelGGL(k_finish_f16, dim3(cd.nsub, cd.max_own), dim3(FIN_THREADS), lds, st, cd, ws,
                                   nsteps, bs);
                return hipGetLastError();
            }
            return run_finish<F16, float>(cd, ws, fa.nfinal, bs, st);
        default: return run_finish<BF16, float>(cd, ws, fa.nfinal, bs, st);
    }
}

// ---------------------------------------------------------------------------
// Extraction, traces and write-back, one workgroup per submatrix.
//   Dcols_J = (Y_J - Z_J) / 2 (FP64), Z_J = X Y_J from the products above;
//   N_J = sum_c (S_J Dcols_J)[bs p + c, c], E_J = sum_c (K_J Dcols_J)[bs p + c, c]
// (Eq. e_elec: the energy only needs D where K is stored; row J of K / S
// holds every block of those rows inside N(J)). FP64 accumulation.
// ---------------------------------------------------------------------------
struct MolStatsDev {
    int32_t iters, iters_fp32, fallback, status;
    double scale, resid, trace_SD, energy_KD;
    int32_t iters_inv, reserved_;
};
static_assert(sizeof(MolStatsDev) == sizeof(nolsm_mol_stats), "stats layout");

// Symmetric sign iteration: Df (np x bs in LDS) holds (y - sign(A~) y) / 2
// with y = L^-1 E; the column block of D is L^-T of it. Backward
// substitution over 64-row blocks with the factor and its diagonal-tile
// inverses (FP64 arithmetic). Per block i, the rows below the block are
// taken off with the FP64 matrix cores: wave w forms the 16 columns
// i 64 + 16 w .. + 15 of L^T times the solved rows of Df, four rows per
// v_mfma_f64_16x16x4 (A from L, one value per lane; B from Df in LDS, its
// bs columns padded to 16), four accumulators in turn; each wave owns its
// columns, so no reduction across waves is needed. tmp: 64 x BSMAX doubles
// of LDS (of 4 x 64 x BSMAX).
template <typename TL>
__device__ void back_solve_lt(const TL *L, const TL *Dinv, const SubMeta &M, double *Df, double *tmp, int bs) {
    const int t = threadIdx.x, np = M.np, l = t & 63, w = t >> 6, mi = l & 15, kq = l >> 4;
    for (int i = M.P - 1; i >= 0; --i) {
        v4d acc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] = v4d{0.0, 0.0, 0.0, 0.0};
        const TL *lc = L + i * 64 + 16 * w + mi;   // column i 64 + 16 w + mi of L
        // 32 rows per step (np - (i + 1) 64 is a multiple of 64): the eight
        // loads of a step are issued before its products
        for (int row0 = (i + 1) * 64; row0 < np; row0 += 32) {
            double a[8], b[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] = (double)lc[(int64_t)(row0 + 4 * u + kq) * np];
#pragma unroll
            for (int u = 0; u < 8; ++u) b[u] = (mi < bs) ? Df[(row0 + 4 * u + kq) * bs + mi] : 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[u & 3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc[u & 3], 0, 0, 0);
        }
        // element e of lane l: column 16 w + kq + 4 e of the block, RHS column mi
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (mi < bs) tmp[(16 * w + kq + 4 * e) * BSMAX + mi] = (acc[0][e] + acc[1][e]) + (acc[2][e] + acc[3][e]);
        __syncthreads();
        if (t < 64) {
#pragma unroll
            for (int c = 0; c < BSMAX; ++c)
                if (c < bs) tmp[t * BSMAX + c] = Df[(i * 64 + t) * bs + c] - tmp[t * BSMAX + c];
        }
        __syncthreads();
        for (int p = t; p < 64 * bs; p += 256) {
            const int rr = p & 63, c = p >> 6;
            const TL *dc = Dinv + (int64_t)i * 4096 + rr;   // column rr of Dinv_i
            double x = 0.0;
            for (int q = 0; q < 64; ++q) x += (double)dc[q * 64] * tmp[q * BSMAX + c];
            Df[(i * 64 + rr) * bs + c] = x;
        }
        __syncthreads();
    }
}

template <typename TV>
__global__ __launch_bounds__(256) void k_extract(ChunkDev cd, char *ws, ExtractArgs ea) {
    extern __shared__ double smem[];
    __shared__ double red[256];
    __shared__ double tmp[4 * 64 * BSMAX];
    const int s = blockIdx.x;
    if (s >= cd.nsub) return;
    const SubMeta M = cd.meta[s];
    const SubCtl *ctl = cd.ctl + s;
    const int bs = ea.bs, n = M.n, np = M.np, t = threadIdx.x;
    double *Df = smem;                                    // np x bs: whole-submatrix column block
    int *rows = (int *)(smem + (size_t)cd.max_np * bs);   // row blocks of the submatrix
    for (int i = t; i < M.m; i += 256) rows[i] = ea.grp_blk[M.sub_off + i];
    const bool ok = ctl->status != NOLSM_MOL_NOT_SPD;
    const int64_t vs = (int64_t)np * 6 * 8 / sizeof(TV);
    for (int o = 0; o < M.nown; ++o) {
        const int J = ea.own_J[M.own_off + o];
        const int so = ea.sub_ptr[J], mJ = ea.sub_ptr[J + 1] - so;
        const TV *V = (const TV *)(ws + M.offVec) + (int64_t)o * NOLSM_NVEC * vs;
        __syncthreads();   // Df of the previous molecule is no longer read
        for (int f = t; f < np * bs; f += 256) {
            const int r = f / bs, c = f % bs;
            double v = 0.0;
            if (ok && r < n) {
                const double y = kbuf_get(M, ws, (int64_t)r * (np + 64) + np + o * bs + c);
                const int64_t q = (int64_t)r * 6 + c;
                double z;
                if (ea.nfinal == 0)
                    z = (double)V[q];
                else if (ea.nfinal == 1)
                    z = 1.5 * (double)V[q] - 0.5 * (double)V[2 * vs + q];
                else
                    z = 1.5 * (double)V[3 * vs + q] - 0.75 * (double)V[8 * vs + q] + 0.25 * (double)V[10 * vs + q];
                v = 0.5 * (y - z);
            }
            Df[f] = v;
        }
        __syncthreads();
        if (ea.sym && ok) {
            // the FP32 factor, or the FP32 copy of the FP64 factor where the
            // route applies it in FP32, else the FP64 factor
            if (ea.L_fp32) back_solve_lt((const float *)(ws + M.offL), (const float *)(ws + M.offDinv), M, Df, tmp, bs);
            else if (M.offL32)
                back_solve_lt((const float *)(ws + M.offL32), (const float *)(ws + M.offDinv32), M, Df, tmp, bs);
            else back_solve_lt((const double *)(ws + M.offL), (const double *)(ws + M.offDinv), M, Df, tmp, bs);
        }
        // the owned columns on the rows N(J) (the pattern of D), through
        // the row positions of N(J) in this submatrix
        double *Dout = ea.Dcols + (int64_t)bs * bs * so;
        for (int f = t; f < mJ * bs * bs; f += 256) {
            const int a = f / (bs * bs), rc = f % (bs * bs);
            const double v = Df[(ea.rowpos[so + a] * bs) * bs + rc];
            Dout[f] = v;
            if (ea.Dval) ea.Dval[(int64_t)ea.scatter_pos[so + a] * bs * bs + rc] = v;
        }
        // the whole column block is kept for the W columns
        if (ea.Wcols) {
            double *Wk = (double *)(ws + M.offVec) + (int64_t)(o * NOLSM_NVEC + NOLSM_NVEC - 1) * np * 6;
            for (int f = t; f < np * bs; f += 256) Wk[(f / bs) * 6 + f % bs] = Df[f];
        }
        // traces over row J of S and of K: every stored column block C of
        // row J lies in N(J), hence in the submatrix rows
        double tr[2];
        for (int which = 0; which < 2; ++which) {
            const int *rp = which ? ea.Krp : ea.Srp;
            const int *ci = which ? ea.Kci : ea.Sci;
            const double *val = which ? ea.Kval : ea.Sval;
            const int lo = rp[J], hi = rp[J + 1];
            const int nel = (hi - lo) * bs * bs;
            double part = 0.0;
            for (int f = t; f < nel; f += 256) {
                const int e = lo + f / (bs * bs), rc = f % (bs * bs);
                const int c = rc / bs, d = rc % bs;
                const int C = ci[e];
                int l = 0, h = M.m - 1, b = -1;
                while (l <= h) {
                    const int mid = (l + h) >> 1;
                    const int v = rows[mid];
                    if (v == C) { b = mid; break; }
                    if (v < C) l = mid + 1; else h = mid - 1;
                }
                if (b >= 0) part += val[(int64_t)e * bs * bs + rc] * Df[(b * bs + d) * bs + c];
            }
            tr[which] = block_sum(part, red);
        }
        if (t == 0) {
            MolStatsDev *st = (MolStatsDev *)ea.stats + J;
            st->iters = ctl->iters;
            st->iters_fp32 = (ok && (ea.prec == NOLSM_FP16 || ea.prec == NOLSM_BF16)) ? ea.nfinal : 0;
            st->fallback = ctl->fallback;
            st->status = ctl->status;
            st->scale = ctl->scale;
            st->resid = ctl->resid;
            st->trace_SD = ok ? tr[0] : 0.0;
            st->energy_KD = ok ? tr[1] : 0.0;
            st->iters_inv = cd.ictl ? cd.ictl[s].iters : 0;
            st->reserved_ = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// Owned columns of the energy-weighted density matrix (Sec. III-B.2):
//   T_J(W)[:, cJ] = T_J(D) T_J(K) T_J(D)[:, cJ].
// With T_J(D) = P T_J(S)^-1, P = (I - sign A_J)/2 a projector that commutes
// with A_J = T_J(S)^-1 T_J(K) - mu I, this is P (A_J + mu I) P Y_J =
// (A_J + mu I) Dcols_J: one n x n by n x bs product with the FP64 A_J still in
// the workspace, on the whole submatrix column block of the molecule (kept by
// the extraction) and written back on the rows N(J). One row per lane, 256
// rows per workgroup, one workgroup per (row block, owned molecule); the
// column block is staged in LDS (max_np x bs doubles). NOT_SPD molecules get
// zeros.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_wcols(ChunkDev cd, char *ws, ExtractArgs ea) {
    extern __shared__ __attribute__((aligned(16))) double dcs[];
    const uint32_t task = xcd_task(cd.t_rows);
    if (task == NOLSM_TASK_NONE) return;
    const int s = task_slot(task), rq = task_a(task), o = task_b(task);
    const SubMeta M = cd.meta[s];
    const int n = M.n, np = M.np, bs = ea.bs, t = threadIdx.x;
    const int J = ea.own_J[M.own_off + o];
    const int so = ea.sub_ptr[J], mJ = ea.sub_ptr[J + 1] - so;
    const double mu = ((const WsHeader *)ws)->mu;
    const bool ok = cd.ctl[s].status != NOLSM_MOL_NOT_SPD;
    // whole-submatrix column block of molecule J, kept by the extraction
    const double *Df = (const double *)(ws + M.offVec) + (int64_t)(o * NOLSM_NVEC + NOLSM_NVEC - 1) * np * 6;
    double *Wc = ea.Wcols + (int64_t)bs * bs * so;
    for (int f = t; f < n * bs; f += 256) dcs[f] = Df[(f / bs) * 6 + f % bs];
    __syncthreads();
    const int row = rq * 256 + t;   // row of W_J on N(J)
    if (row >= mJ * bs) return;
    const int gr = ea.rowpos[so + row / bs] * bs + row % bs;   // its submatrix row
    double acc[BSMAX];
#pragma unroll
    for (int j = 0; j < BSMAX; ++j) acc[j] = 0.0;
    if (ok) {
        auto row_times = [&](auto arow) {
#pragma unroll 4
            for (int k = 0; k < n; k += 2) {   // n = bs m is even for bs = 6
                const double ax = arow[k], ay = arow[k + 1];
#pragma unroll
                for (int j = 0; j < BSMAX; ++j)
                    if (j < bs) acc[j] += ax * dcs[k * bs + j] + ay * dcs[(k + 1) * bs + j];
            }
        };
        // A_J row gr of the K buffer, FP32 or FP64 storage
        if (M.kf32) row_times((const float *)(ws + M.offK) + (int64_t)gr * (np + 64));
        else row_times((const double *)(ws + M.offK) + (int64_t)gr * (np + 64));
#pragma unroll
        for (int j = 0; j < BSMAX; ++j)
            if (j < bs) acc[j] += mu * dcs[gr * bs + j];
    }
#pragma unroll
    for (int j = 0; j < BSMAX; ++j)
        if (j < bs) Wc[(int64_t)row * bs + j] = acc[j];
}

hipError_t launch_wcols(const ChunkDev &cd, char *ws, const ExtractArgs &ea, hipStream_t st) {
    if (ea.bs & 1) return hipErrorInvalidValue;   // the row loop takes k in pairs
    hipLaunchKernelGGL(k_wcols, dim3(cd.n_rows), dim3(256), (size_t)cd.max_np * ea.bs * 8, st, cd, ws,
                       ea);
    return hipGetLastError();
}

hipError_t launch_extract(const ChunkDev &cd, char *ws, const ExtractArgs &ea, hipStream_t st) {
    const size_t lds = (size_t)cd.max_np * ea.bs * 8 + (size_t)cd.max_m * 4 + 16;
    if (ea.prec == NOLSM_FP64)
        hipLaunchKernelGGL(k_extract<double>, dim3(cd.nsub), dim3(256), lds, st, cd, ws, ea);
    else
        hipLaunchKernelGGL(k_extract<float>, dim3(cd.nsub), dim3(256), lds, st, cd, ws, ea);
    return hipGetLastError();
}

__global__ void k_set_header(char *ws, double mu) {
    if (threadIdx.x == 0) {
        WsHeader *h = (WsHeader *)ws;
        h->mu = mu;
        h->sumN = 0.0;
        h->sumE = 0.0;
        h->n_bad = 0;
    }
}

hipError_t launch_set_header(char *ws, double mu, hipStream_t st) {
    hipLaunchKernelGGL(k_set_header, dim3(1), dim3(64), 0, st, ws, mu);
    return hipGetLastError();
}

// sum_J N_J and sum_J E_J in FP64, one workgroup, fixed summation order
// (each thread a strided range, then a tree): the trace sums of the
// chemical-potential bisection.
__global__ __launch_bounds__(256) void k_trace_sums(const MolStatsDev *st, int nb, char *ws) {
    __shared__ double red[256];
    double n = 0.0, e = 0.0, bad = 0.0;
    for (int J = threadIdx.x; J < nb; J += 256) {
        n += st[J].trace_SD;
        e += st[J].energy_KD;
        bad += st[J].status != NOLSM_MOL_OK ? 1.0 : 0.0;
    }
    n = block_sum(n, red);
    e = block_sum(e, red);
    bad = block_sum(bad, red);
    if (threadIdx.x == 0) {
        WsHeader *h = (WsHeader *)ws;
        h->sumN = n;
        h->sumE = e;
        h->n_bad = (int32_t)bad;
    }
}

hipError_t launch_trace_sums(const void *stats, int32_t nb, char *ws, hipStream_t st) {
    hipLaunchKernelGGL(k_trace_sums, dim3(1), dim3(256), 0, st, (const MolStatsDev *)stats, nb, ws);
    return hipGetLastError();
}

__global__ void k_assemble(const double *Dcols, double *Dval, const int32_t *scatter_pos, int64_t sum_m, int bs) {
    const int64_t total = sum_m * bs * bs;
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < total; f += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = f / (bs * bs), rc = f % (bs * bs);
        Dval[(int64_t)scatter_pos[k] * bs * bs + rc] = Dcols[f];
    }
}

hipError_t launch_assemble(const double *Dcols, double *Dval, const int32_t *scatter_pos, int64_t sum_m,
                           int32_t bs, hipStream_t st) {
    const int64_t total = sum_m * bs * bs;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_assemble, dim3((unsigned)blocks), dim3(256), 0, st, Dcols, Dval, scatter_pos, sum_m, bs);
    return hipGetLastError();
}

hipError_t nolsm_finish_init() {
    const void *fns[] = {(const void *)k_extract<double>,          (const void *)k_extract<float>,
                         (const void *)k_skinny<double, double>,   (const void *)k_skinny<float, float>,
                         (const void *)k_skinny<F16, float>,       (const void *)k_skinny<BF16, float>,
                         (const void *)k_wcols,                (const void *)k_finish_f16};
    for (const void *f : fns)
        if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) != hipSuccess)
            return hipErrorInvalidValue;
    return hipSuccess;
}
