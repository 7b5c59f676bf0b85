// Inverse of T_J(S) by the coupled Newton-Schulz iteration (Sec. III-C.3,
// Eq. inv1-inv3) on the matrix cores, FP16 / BF16 operands with FP32
// accumulation, and the formation of A_J = T_J(S)^-1 T_J(K) - mu I and
// Y_J = T_J(S)^-1 E_cJ from it (Eq. purification_submatrix).
//
//   Y_0 = c S_J, Z_0 = I,  c = 1 / max row sum of |S_J| (spectrum of c S_J
//   inside (0, 1]); per iteration k:
//     R_k = I - Z_k Y_k                       (one GEMM; ||R_k||_F^2 partials)
//     Y_{k+1} = Y_k + Y_k R_k / 2,  Z_{k+1} = Z_k + R_k Z_k / 2
//   which equal Y_k (3I - V_k) / 2 and (3I - V_k) Z_k / 2 with V_k = Z_k Y_k;
//   R_k is small near convergence and keeps its relative precision in 16
//   bits. Z_k tends to (c S_J)^(-1/2), so S_J^-1 = c Z_K^2.
// The iteration stops like the 16-bit sign iteration (stagnation of
// ||R_k||_F below 0.5); a diverging one marks the molecule NOT_SPD. The
// outputs are exactly those of the Cholesky route: [A | Y] in the FP64 K
// buffer, |A| row / column sums and Frobenius partials per 64-column tile.
#include "dev_common.h"
#include "kernels.h"
#include "lp_gemm.h"

enum { IM_R = 1, IM_UPD = 2, IM_SQ = 3, IM_A = 4 };
enum { IACT_STOP = 0, IACT_UPDATE = 1 };

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// c = 1 / max row sum of |S_J| over the padded np x np matrix (padding rows
// are identity), Y_0 = c S_J and Z_0 = I in 16 bits; one workgroup per slot.
template <typename T>
__global__ __launch_bounds__(256) void k_inv_init(ChunkDev cd, char *ws) {
    __shared__ double red[256];
    const int s = blockIdx.x;
    if (s >= cd.nsub) return;
    const SubMeta M = cd.meta[s];
    InvCtl *ic = cd.ictl + s;
    const int np = M.np, ldx = M.ldx, t = threadIdx.x, w = t >> 6, l = t & 63;
    const double *S = (const double *)(ws + M.offL);
    double mx = 0.0;
    for (int r = w; r < np; r += 4) {
        double rs = 0.0;
        for (int c = l; c < np; c += 64) rs += fabs(S[(int64_t)r * np + c]);
        mx = fmax(mx, wave_sum(rs));
    }
    mx = block_max(mx, red);
    const double c = 1.0 / mx;
    uint16_t *Y0 = (uint16_t *)(ws + M.offY0);
    uint16_t *Z0 = (uint16_t *)(ws + M.offZ0);
    for (int r = w; r < np; r += 4)
        for (int q = l; q < np; q += 64) {
            Y0[(int64_t)r * ldx + q] = Lp<T>::enc((float)(c * S[(int64_t)r * np + q]));
            Z0[(int64_t)r * ldx + q] = Lp<T>::enc(r == q ? 1.0f : 0.0f);
        }
    if (t == 0) {
        ic->done = 0;
        ic->iters = 0;
        ic->scale = c;
    }
    for (int i = t; i < NOLSM_MAX_ITER_CAP; i += 256) ic->rhist[i] = 0.0;
}

// Decision at the update of iteration `it`, taken by thread 0 of every
// workgroup of the slot from the finished residual partials; the tile-0
// workgroup records it.
__device__ int inv_decide(const InvArgs &ia, const SubMeta &M, InvCtl *ic, SubCtl *ctl, const char *ws, int it,
                          int tile) {
    const double *res = (const double *)(ws + M.offRes) + (int64_t)it * M.ntile_ns;
    double ssum = 0.0;
    for (int i = 0; i < M.ntile_ns; ++i) ssum += res[i];
    const double r = sqrt(ssum);
    const double rprev = it > 0 ? ic->rhist[it - 1] : INFINITY;
    const bool stop = it >= 1 && r < ia.rmax && r > ia.theta * rprev;
    const bool diverge = !isfinite(r) || (it >= 1 && r > 2.0 * rprev && r > 1.0);
    const bool last = it + 1 >= ia.max_iter;
    if (tile == 0) {
        ic->rhist[it] = r;
        if (stop || diverge || last) {
            ic->done = 1;
            ic->iters = it;
            // no usable inverse (a diverging iteration, or none within the
            // slots): the molecule is reported NOT_SPD and the sign iteration,
            // finishing and extraction skip it, leaving its columns at zero
            if (diverge || !stop) {
                ctl->status = NOLSM_MOL_NOT_SPD;
                ctl->done = 1;
            }
        }
    }
    return (stop || diverge || last) ? IACT_STOP : IACT_UPDATE;
}

// One BM x BM tile of an inverse-route GEMM. `which` selects the product of
// the update (0: Y, 1: Z).
template <typename T, int BM>
__device__ __forceinline__ void inv_tile(const ChunkDev &cd, uint32_t task, char *ws, const InvArgs &ia, int it,
                                         int mode, int which) {
    __shared__ double red[256];
    __shared__ int act_s;
    if (task == NOLSM_TASK_NONE) return;
    const int s = task_slot(task), ti = task_a(task), tj = task_b(task);
    const SubMeta M = cd.meta[s];
    SubCtl *ctl = cd.ctl + s;
    InvCtl *ic = cd.ictl + s;
    const int np = M.np, nt = (np + BM - 1) / BM, tile = ti * nt + tj, ldx = M.ldx;
    if (threadIdx.x == 0) {
        int act;
        if (ctl->status != NOLSM_MOL_OK) act = IACT_STOP;
        else if (mode == IM_R) act = ic->done ? IACT_STOP : IACT_UPDATE;
        else if (mode == IM_UPD) act = ic->done ? IACT_STOP : inv_decide(ia, M, ic, ctl, ws, it, tile);
        else act = IACT_UPDATE;   // after the loop: every OK slot
        act_s = act;
    }
    __syncthreads();
    if (act_s == IACT_STOP) return;
    // buffers of iteration k: Y_k, Z_k in ping-pong slot k % 2
    const int K = (mode == IM_SQ || mode == IM_A) ? ic->iters : it;
    uint16_t *Yc = (uint16_t *)(ws + ((K & 1) ? M.offY1 : M.offY0));
    uint16_t *Yn = (uint16_t *)(ws + ((K & 1) ? M.offY0 : M.offY1));
    uint16_t *Zc = (uint16_t *)(ws + ((K & 1) ? M.offZ1 : M.offZ0));
    uint16_t *Zn = (uint16_t *)(ws + ((K & 1) ? M.offZ0 : M.offZ1));
    uint16_t *Rb = (uint16_t *)(ws + M.offB);
    // after the loop the Y buffers are free: S^-1 goes to Y0, K to Y1
    uint16_t *Sinv = (uint16_t *)(ws + M.offY0);
    uint16_t *K16 = (uint16_t *)(ws + M.offY1);
    const uint16_t *Ag, *Bg;
    switch (mode) {
        case IM_R: Ag = Zc; Bg = Yc; break;
        case IM_UPD: Ag = which ? Rb : Yc; Bg = which ? Zc : Rb; break;
        case IM_SQ: Ag = Zc; Bg = Zc; break;
        default: Ag = Sinv; Bg = K16; break;
    }
    constexpr int WT = BM / 2, NB = WT / 32;
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, wm = w >> 1, wn = w & 1;
    const int row0 = ti * BM, col0 = tj * BM;
    const int nrec = ldx * ldx * 2;
    v16f acc[NB][NB];
    lp_tile_product<T, BM>(Ag, Bg, ldx, np, row0, col0, acc);
    // element e of block (i, j): row er0 + i 32 + (e / 4) 8 + e % 4, column ec0 + j 32
    const int er0 = row0 + wm * WT + (l >> 5) * 4, ec0 = col0 + wn * WT + (l & 31);
    const uint32_t eo = (uint32_t)((er0 * ldx + ec0) * 2);
#define INV_EOFF(i, j, e) ((((i) * 32 + ((e) >> 2) * 8 + ((e) & 3)) * ldx + (j) * 32) * 2)
#define INV_ROW(i, e) (er0 + (i) * 32 + ((e) >> 2) * 8 + ((e) & 3))
    if (mode == IM_R) {
        const __amdgpu_buffer_rsrc_t rsR = __builtin_amdgcn_make_buffer_rsrc((void *)Rb, (short)0, nrec, 0x00020000);
        double part = 0.0;
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j)
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int gr = INV_ROW(i, e), gc = ec0 + j * 32;
                    const float rr = (gr == gc ? 1.0f : 0.0f) - acc[i][j][e];
                    __builtin_amdgcn_raw_buffer_store_b16(Lp<T>::enc(rr), rsR, eo, INV_EOFF(i, j, e), 0);
                    if (gr < np && gc < np) part += (double)rr * (double)rr;
                }
        const double sum = block_sum(part, red);
        if (threadIdx.x == 0) ((double *)(ws + M.offRes))[(int64_t)it * M.ntile_ns + tile] = sum;
    } else if (mode == IM_UPD) {
        // Y_{k+1} = Y_k + Y_k R_k / 2 or Z_{k+1} = Z_k + R_k Z_k / 2
        const uint16_t *E = which ? Zc : Yc;
        uint16_t *O = which ? Zn : Yn;
        const __amdgpu_buffer_rsrc_t rsE = __builtin_amdgcn_make_buffer_rsrc((void *)E, (short)0, nrec, 0x00020000);
        const __amdgpu_buffer_rsrc_t rsO = __builtin_amdgcn_make_buffer_rsrc((void *)O, (short)0, nrec, 0x00020000);
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                uint16_t eo16[16];
#pragma unroll
                for (int e = 0; e < 16; ++e) eo16[e] = __builtin_amdgcn_raw_buffer_load_b16(rsE, eo, INV_EOFF(i, j, e), 0);
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    __builtin_amdgcn_raw_buffer_store_b16(Lp<T>::enc(Lp<T>::dec(eo16[e]) + 0.5f * acc[i][j][e]), rsO,
                                                          eo, INV_EOFF(i, j, e), 0);
            }
    } else if (mode == IM_SQ) {
        // S^-1 = c Z_K^2 in 16 bits for the A GEMM; the columns of every
        // owned molecule o (block position q_o) also go, from the FP32
        // accumulators, to its FP64 Y columns np + o bs .. of the K buffer
        const double c = ic->scale;
        const __amdgpu_buffer_rsrc_t rsS = __builtin_amdgcn_make_buffer_rsrc((void *)Sinv, (short)0, nrec, 0x00020000);
        double *Kb = (double *)(ws + M.offK);
        const int ldk = np + 64, bs = ia.bs;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            // the output column of this lane in block column j, and its owner
            const int gc = ec0 + j * 32, qb = gc / bs;
            int yc = -1;
            for (int o = 0; o < M.nown; ++o)
                if (ia.own_pos[M.own_off + o] == qb) yc = np + o * bs + (gc - qb * bs);
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const float v = (float)c * acc[i][j][e];
                    __builtin_amdgcn_raw_buffer_store_b16(Lp<T>::enc(v), rsS, eo, INV_EOFF(i, j, e), 0);
                    const int gr = INV_ROW(i, e);
                    if (gr < np && gc < np && yc >= 0) Kb[(int64_t)gr * ldk + yc] = c * (double)acc[i][j][e];
                }
        }
    } else {
        // A_J = S^-1 K_J - mu I, FP64, rows and columns < np only (columns
        // np.. of the K buffer hold Y_J)
        const double mu = ((const WsHeader *)ws)->mu;
        double *Kb = (double *)(ws + M.offK);
        const int ldk = np + 64;
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j)
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int gr = INV_ROW(i, e), gc = ec0 + j * 32;
                    if (gr < np && gc < np) Kb[(int64_t)gr * ldk + gc] = (double)acc[i][j][e] - (gr == gc ? mu : 0.0);
                }
    }
#undef INV_EOFF
#undef INV_ROW
}

template <typename T, int BM>
__global__ __launch_bounds__(256, 3) void k_inv_lp(ChunkDev cd, const uint32_t *tasks, char *ws, InvArgs ia, int it,
                                                int mode) {
    inv_tile<T, BM>(cd, xcd_task(tasks), ws, ia, it, mode, blockIdx.y);
}

// K_J (FP64, columns < np of the K buffer) to 16 bits in the Y1 buffer for
// the A GEMM; one workgroup per slot.
template <typename T>
__global__ __launch_bounds__(256) void k_inv_k16(ChunkDev cd, char *ws) {
    const int s = blockIdx.x;
    if (s >= cd.nsub) return;
    const SubMeta M = cd.meta[s];
    if (cd.ctl[s].status != NOLSM_MOL_OK) return;
    const int np = M.np, ldx = M.ldx, w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const double *Kb = (const double *)(ws + M.offK);
    uint16_t *K16 = (uint16_t *)(ws + M.offY1);
    for (int r = w; r < np; r += 4)
        for (int q = l; q < np; q += 64) K16[(int64_t)r * ldx + q] = Lp<T>::enc((float)Kb[(int64_t)r * (np + 64) + q]);
}

// The bounds inputs the substitution would have written, from the FP64 A_J:
// for 64-column tile cc, partial |A| row sums (columns < n) per row, the
// complete |A| column sums (rows < n) and the tile's Frobenius share. Tasks
// (slot, cc) with cc <= P; cc = P (the Y tile) has nothing to add.
__global__ __launch_bounds__(256) void k_inv_sums(ChunkDev cd, char *ws) {
    __shared__ double red[256];
    const uint32_t task = xcd_task(cd.t_subst);
    if (task == NOLSM_TASK_NONE) return;
    const int s = task_slot(task), cc = task_a(task);
    const SubMeta M = cd.meta[s];
    if (cd.ctl[s].status != NOLSM_MOL_OK || cc >= M.P) return;
    const int n = M.n, np = M.np, t = threadIdx.x;
    const int64_t ldk = np + 64;
    const double *A = (const double *)(ws + M.offK);
    double *rowp = (double *)(ws + M.offRow);
    double *colp = (double *)(ws + M.offCol);
    double fs = 0.0;
    for (int r = t; r < np; r += 256) {
        double rs = 0.0;
        if (r < n)
            for (int c = 0; c < 64; ++c) {
                const int gc = cc * 64 + c;
                if (gc < n) {
                    const double v = A[(int64_t)r * ldk + gc];
                    rs += fabs(v);
                    fs += v * v;
                }
            }
        rowp[(int64_t)cc * np + r] = rs;
    }
    if (t < 64) {
        const int gc = cc * 64 + t;
        double cs = 0.0;
        if (gc < n)
            for (int r = 0; r < n; ++r) cs += fabs(A[(int64_t)r * ldk + gc]);
        colp[gc] = cs;
    }
    const double fsum = block_sum(fs, red);
    if (t == 0) colp[np + cc] = fsum;
}

template <typename T>
static void launch_inv_gemm(const ChunkDev &cd, char *ws, const InvArgs &ia, int it, int mode, int nprod,
                            hipStream_t st) {
    if (cd.n_ns > 0)
        hipLaunchKernelGGL((k_inv_lp<T, 128>), dim3(cd.n_ns, nprod), dim3(256), 0, st, cd, cd.t_ns, ws, ia, it, mode);
    if (cd.n_ns64 > 0)
        hipLaunchKernelGGL((k_inv_lp<T, 64>), dim3(cd.n_ns64, nprod), dim3(256), 0, st, cd, cd.t_ns64, ws, ia, it,
                           mode);
}

template <typename T>
static hipError_t run_inverse(const ChunkDev &cd, char *ws, const InvArgs &ia, hipStream_t st) {
    hipLaunchKernelGGL(k_inv_init<T>, dim3(cd.nsub), dim3(256), 0, st, cd, ws);
    for (int it = 0; it < ia.max_iter; ++it) {
        launch_inv_gemm<T>(cd, ws, ia, it, IM_R, 1, st);
        launch_inv_gemm<T>(cd, ws, ia, it, IM_UPD, 2, st);
    }
    hipLaunchKernelGGL(k_inv_k16<T>, dim3(cd.nsub), dim3(256), 0, st, cd, ws);
    launch_inv_gemm<T>(cd, ws, ia, 0, IM_SQ, 1, st);
    launch_inv_gemm<T>(cd, ws, ia, 0, IM_A, 1, st);
    hipLaunchKernelGGL(k_inv_sums, dim3(cd.n_subst), dim3(256), 0, st, cd, ws);
    return hipGetLastError();
}

hipError_t launch_inverse(const ChunkDev &cd, char *ws, const InvArgs &ia, hipStream_t st) {
    if (!cd.ictl) return hipErrorInvalidValue;
    return ia.prec == NOLSM_FP16 ? run_inverse<_Float16>(cd, ws, ia, st) : run_inverse<__bf16>(cd, ws, ia, st);
}
