// FP16 / BF16 tile products on v_mfma_f32_32x32x16_{f16,bf16} with FP32
// accumulation, shared by the Newton-Schulz sign iteration and the coupled
// Newton-Schulz inverse. Operands are row-major ldx x ldx 16-bit matrices in
// the workspace with ldx >= every tile extent (so loads need no masking) and
// the contraction runs over k < np (np a multiple of 64).
#pragma once
#include "dev_common.h"

template <typename T> struct Lp;
template <> struct Lp<_Float16> {
    typedef v8h vec;
    static __device__ __forceinline__ v16f mma(vec a, vec b, v16f c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ uint16_t enc(float x) {
        _Float16 h = (_Float16)x;
        return __builtin_bit_cast(uint16_t, h);
    }
    static __device__ __forceinline__ float dec(uint16_t x) { return (float)__builtin_bit_cast(_Float16, x); }
};
template <> struct Lp<__bf16> {
    typedef v8bf vec;
    static __device__ __forceinline__ v16f mma(vec a, vec b, v16f c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ uint16_t enc(float x) {
        __bf16 h = (__bf16)x;
        return __builtin_bit_cast(uint16_t, h);
    }
    static __device__ __forceinline__ float dec(uint16_t x) { return (float)__builtin_bit_cast(__bf16, x); }
};

#define LBK 64

// LDS tiles hold 64 k per row (128 bytes, no padding). The 16-byte chunk c
// (8 consecutive k) of row n sits at chunk position c ^ ((n ^ n >> 3) & 7):
// an MFMA operand read (32 rows, one chunk) then touches 8 distinct chunk
// positions in every 8 consecutive rows, and the transposing B stores (one
// row per 8 columns) spread over all positions as well.
__device__ __forceinline__ int lds_swz(int n, int c) { return n * LBK + ((c ^ ((n ^ (n >> 3)) & 7)) << 3); }

// The two operand tiles of lp_tile_product (BM x LBK 16-bit values each),
// one allocation per kernel; free again when lp_tile_product returns, so an
// epilogue may stage through them.
template <int BM> __device__ __forceinline__ uint16_t *lp_lds() {
    __shared__ __attribute__((aligned(16))) uint16_t buf[2 * BM * LBK];
    return buf;
}

// acc = A[row0 .. row0 + BM, 0 .. np) * B[0 .. np, col0 .. col0 + BM): one
// BM x BM tile (BM = 128: each of the 4 waves 64x64 as 2x2 32x32 MFMA blocks;
// BM = 64: one 32x32 block per wave), K in slices of 64. A is staged in LDS
// as [m][k]; B is read row-major from HBM and transposed on its way into LDS
// ([n][k]) so that both MFMA operands are 16-byte LDS reads of 8 consecutive
// k. On return, element e of block (i, j) of the calling lane holds output
// row wm WT + i 32 + (e / 4) 8 + (l / 32) 4 + e % 4 and column
// wn WT + j 32 + l % 32 of the tile (w = wave = 2 wm + wn, l = lane,
// WT = BM / 2). All 256 threads must call it.
// BSYM: B is symmetric, so B[k][n] = B[n][k] and its tile is loaded by rows
// exactly like A (no transposition on the way into LDS).
// SAME (with BSYM): B is A and col0 = row0 (a diagonal tile of X X with X
// symmetric), so the B tile would equal the A tile: only A is loaded, and the
// products read both operands from it.
template <typename T, int BM, bool BSYM = false, bool SAME = false>
__device__ __forceinline__ void lp_tile_product(const uint16_t *Ag, const uint16_t *Bg, int ldx, int np, int row0,
                                                int col0, v16f (&acc)[BM / 64][BM / 64]) {
    typedef typename Lp<T>::vec vec;
    static_assert(!SAME || BSYM, "a shared operand tile needs B loaded by rows like A");
    constexpr int WT = BM / 2;          // wave tile
    constexpr int NB = WT / 32;         // 32x32 MFMA blocks per wave dimension
    constexpr int AQ = BM / 32;         // 16-byte A loads per thread
    constexpr int BT = 2 * BM;          // threads that load a 4(k) x 8(n) B block
    uint16_t(*sA)[BM * LBK] = (uint16_t(*)[BM * LBK])lp_lds<BM>();
    uint16_t(*sB)[BM * LBK] = (uint16_t(*)[BM * LBK])(lp_lds<BM>() + BM * LBK);
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const int wm = w >> 1, wn = w & 1;
    const int ac = (t & 7) * 8;
    const bool bload = BSYM || (BT >= 256) || t < BT;   // BM = 128: every thread
    // B block of thread t: k rows 4 kq .. 4 kq + 3, columns 8 nci .. 8 nci + 7.
    // Each group of 16 lanes covers 8 column blocks and two k quads, so its
    // 8-byte LDS stores land on 16 distinct 8-byte bank slots.
    const int nci = (BM == 128) ? ((t & 7) | (((t >> 4) & 1) << 3)) : (t & 7);
    const int kq = (BM == 128) ? (((t >> 3) & 1) | ((t >> 5) << 1)) : (t >> 3);
    const int nc = nci * 8;
    // The buffers have ldx >= the tile extent rows and columns, so loads need
    // no masking: rows of A / columns of B past np only feed outputs that are
    // never stored (an output (r, c) reads only row r of A and column c of B),
    // and the k range stops at np. Staging is straight-line code on named
    // registers (no arrays or lambdas, which the compiler spilled to scratch).
    // Slices are fetched with raw buffer loads over the ldx x ldx buffers:
    // a 32-bit lane offset plus a uniform row-block offset. A slice past the
    // end (and B for threads that stage none) gets a lane offset beyond the
    // buffer size, which the hardware answers with zeros and no memory
    // access, so every load is unconditional and the compiler's wait counts
    // stay exact across the prefetch ring.
    const int nrec = ldx * ldx * 2;
    const __amdgpu_buffer_rsrc_t rsA = __builtin_amdgcn_make_buffer_rsrc((void *)Ag, (short)0, nrec, 0x00020000);
    const __amdgpu_buffer_rsrc_t rsB = __builtin_amdgcn_make_buffer_rsrc((void *)Bg, (short)0, nrec, 0x00020000);
    const uint32_t va = (uint32_t)(((row0 + (t >> 3)) * ldx + ac) * 2);
    const uint32_t vb = BSYM ? (uint32_t)(((col0 + (t >> 3)) * ldx + ac) * 2)
                             : (uint32_t)((kq * 4 * ldx + col0 + nc) * 2);
    const int sa32 = 64 * ldx, srow = 2 * ldx;   // bytes of 32 rows / one row
    const int nk = np / LBK;
    // One LDS buffer and one register set per workgroup (32 KB of LDS and
    // about 140 VGPRs for BM = 128), so three workgroups share a CU: slice
    // kt + 1 is fetched into registers while slice kt is multiplied from LDS,
    // and latency is hidden across workgroups rather than by a deeper ring.
    const uint4 z4 = {0, 0, 0, 0};
    uint4 pa0 = z4, pa1 = z4, pa2 = z4, pa3 = z4, pb0 = z4, pb1 = z4, pb2 = z4, pb3 = z4;
#define NS_BUF(rs, vo, so) __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, vo, so, 0))
#define NS_GLOAD(S, ks)                                                          \
    do {                                                                         \
        const bool in_ = (ks) < nk;                                              \
        const uint32_t oa_ = in_ ? va + (uint32_t)((ks) * LBK * 2) : 0x80000000u; \
        const uint32_t ob_ = !(in_ && bload) ? 0x80000000u                      \
                             : BSYM ? vb + (uint32_t)((ks) * LBK * 2)            \
                                    : vb + (uint32_t)((ks) * LBK * srow);        \
        S##a0 = NS_BUF(rsA, oa_, 0);                                             \
        S##a1 = NS_BUF(rsA, oa_, sa32);                                          \
        if constexpr (AQ > 2) {                                                  \
            S##a2 = NS_BUF(rsA, oa_, 2 * sa32);                                  \
            S##a3 = NS_BUF(rsA, oa_, 3 * sa32);                                  \
        }                                                                        \
        if constexpr (SAME) {                                                    \
        } else if constexpr (BSYM) {                                             \
            S##b0 = NS_BUF(rsB, ob_, 0);                                         \
            S##b1 = NS_BUF(rsB, ob_, sa32);                                      \
            if constexpr (AQ > 2) {                                              \
                S##b2 = NS_BUF(rsB, ob_, 2 * sa32);                              \
                S##b3 = NS_BUF(rsB, ob_, 3 * sa32);                              \
            }                                                                    \
        } else {                                                                 \
            S##b0 = NS_BUF(rsB, ob_, 0);                                         \
            S##b1 = NS_BUF(rsB, ob_, srow);                                      \
            S##b2 = NS_BUF(rsB, ob_, 2 * srow);                                  \
            S##b3 = NS_BUF(rsB, ob_, 3 * srow);                                  \
        }                                                                        \
    } while (0)
// B is a 4(k) x 8(n) block in S##b0..S##b3 (one k row each); column j of it
// becomes 4 consecutive k for LDS row n = nc + j
#define NS_BCOL(S, j, W)                                                         \
    do {                                                                         \
        uint32_t lo_, hi_;                                                       \
        if (((j) & 1) == 0) {                                                    \
            lo_ = (S##b0.W & 0xFFFFu) | (S##b1.W << 16);                         \
            hi_ = (S##b2.W & 0xFFFFu) | (S##b3.W << 16);                         \
        } else {                                                                 \
            lo_ = (S##b0.W >> 16) | (S##b1.W & 0xFFFF0000u);                     \
            hi_ = (S##b2.W >> 16) | (S##b3.W & 0xFFFF0000u);                     \
        }                                                                        \
        *(uint2 *)&sB[buf_][lds_swz(nc + (j), kq >> 1) + (kq & 1) * 4] =         \
            make_uint2(lo_, hi_);                                                \
    } while (0)
#define NS_SSTORE(S, bufi)                                                       \
    do {                                                                         \
        const int buf_ = (bufi);                                                 \
        *(uint4 *)&sA[buf_][lds_swz(t >> 3, t & 7)] = S##a0;                     \
        *(uint4 *)&sA[buf_][lds_swz((t >> 3) + 32, t & 7)] = S##a1;              \
        if constexpr (AQ > 2) {                                                  \
            *(uint4 *)&sA[buf_][lds_swz((t >> 3) + 64, t & 7)] = S##a2;          \
            *(uint4 *)&sA[buf_][lds_swz((t >> 3) + 96, t & 7)] = S##a3;          \
        }                                                                        \
        if constexpr (SAME) {                                                    \
        } else if constexpr (BSYM) {                                             \
            *(uint4 *)&sB[buf_][lds_swz(t >> 3, t & 7)] = S##b0;                 \
            *(uint4 *)&sB[buf_][lds_swz((t >> 3) + 32, t & 7)] = S##b1;          \
            if constexpr (AQ > 2) {                                              \
                *(uint4 *)&sB[buf_][lds_swz((t >> 3) + 64, t & 7)] = S##b2;      \
                *(uint4 *)&sB[buf_][lds_swz((t >> 3) + 96, t & 7)] = S##b3;      \
            }                                                                    \
        } else if (bload) {                                                      \
            NS_BCOL(S, 0, x); NS_BCOL(S, 1, x); NS_BCOL(S, 2, y);                \
            NS_BCOL(S, 3, y); NS_BCOL(S, 4, z); NS_BCOL(S, 5, z);                \
            NS_BCOL(S, 6, w); NS_BCOL(S, 7, w);                                  \
        }                                                                        \
    } while (0)
// one k slice of MFMA work from LDS buffer bufi
#define NS_COMPUTE(bufi)                                                         \
    do {                                                                         \
        _Pragma("unroll") for (int kk = 0; kk < LBK; kk += 16) {                 \
            vec a[NB], b[NB];                                                    \
            _Pragma("unroll") for (int i = 0; i < NB; ++i) a[i] =                \
                *(const vec *)&sA[bufi][lds_swz(wm * WT + i * 32 + (l & 31),     \
                                                (kk >> 3) + (l >> 5))];          \
            _Pragma("unroll") for (int j = 0; j < NB; ++j) b[j] =                \
                *(const vec *)&(SAME ? sA : sB)[bufi][lds_swz(wn * WT + j * 32 + (l & 31), \
                                                (kk >> 3) + (l >> 5))];          \
            _Pragma("unroll") for (int i = 0; i < NB; ++i)                       \
                _Pragma("unroll") for (int j = 0; j < NB; ++j)                   \
                    acc[i][j] = Lp<T>::mma(a[i], b[j], acc[i][j]);               \
        }                                                                        \
    } while (0)
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;
    NS_GLOAD(p, 0);
    NS_SSTORE(p, 0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        NS_GLOAD(p, kt + 1);   // past the last slice: zeros, no memory access
        // the loads stay ahead of the products: without this fence (and with
        // a conditional store) the compiler sinks them behind the MFMAs,
        // next to their use, and every slice waits out the full load latency
        __builtin_amdgcn_sched_barrier(0);
        NS_COMPUTE(0);
        __syncthreads();
        NS_SSTORE(p, 0);       // the last one stores zeros nothing reads
        __syncthreads();
    }
#undef NS_BUF
#undef NS_GLOAD
#undef NS_BCOL
#undef NS_SSTORE
#undef NS_COMPUTE
}
