// Device helpers shared by the HIP kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nolsm_internal.h"

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// Task lists are padded to a multiple of 8 entries. Workgroup b takes entry
// (b % 8) * (G / 8) + b / 8: the dispatcher hands workgroups to the 8 XCDs
// round-robin, so consecutive list entries (the tiles of one submatrix) land
// on one XCD and share its L2.
__device__ __forceinline__ uint32_t xcd_task(const uint32_t *list) {
    const uint32_t G = gridDim.x, b = blockIdx.x;
    return list[(b & 7u) * (G >> 3) + (b >> 3)];
}
__device__ __forceinline__ int task_slot(uint32_t t) { return (int)(t >> 16); }
__device__ __forceinline__ int task_a(uint32_t t) { return (int)((t >> 8) & 0xFF); }
__device__ __forceinline__ int task_b(uint32_t t) { return (int)(t & 0xFF); }

// ---------------------------------------------------------------------------
// 64x64 tiles on the matrix cores, 256 threads, in FP64
// (v_mfma_f64_16x16x4_f64) or FP32 (v_mfma_f32_16x16x4_f32); the global
// operands are FP64 either way and are rounded when staged. Wave w owns the
// 32x32 quadrant (w>>1, w&1) as 2x2 blocks of 16x16. In a block, A[i][k]
// comes from lane i + 16k and B[k][j] from lane j + 16k for both types;
// element e of lane l is D[l/16 + 4e][l%16] in FP64 and D[4(l/16) + e][l%16]
// in FP32 (both measured on gfx950). LDS tiles are [64][LDP] values,
// LDP = 65 (one pad value per row).
// ---------------------------------------------------------------------------
#define LDP 65

template <typename T> struct Mfma16;
template <> struct Mfma16<double> {
    typedef v4d acc_t;
    static __device__ __forceinline__ v4d mma(double a, double b, v4d c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma16<float> {
    typedef v4f acc_t;
    static __device__ __forceinline__ v4f mma(float a, float b, v4f c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <typename T> struct Same { typedef T type; };

template <typename T> struct AccT {
    typename Mfma16<T>::acc_t c[2][2];
};
typedef AccT<double> Acc64;

template <typename T> __device__ __forceinline__ void acc_zero(AccT<T> &a) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) a.c[i][j][e] = (T)0;
}

// row/col of element e of block (i, j) for this lane
template <typename T> __device__ __forceinline__ int acc_row(int i, int e) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    return (w >> 1) * 32 + i * 16 + (sizeof(T) == 8 ? (l >> 4) + 4 * e : 4 * (l >> 4) + e);
}
__device__ __forceinline__ int acc_col(int j) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    return (w & 1) * 32 + j * 16 + (l & 15);
}

// acc += op(A) * op(B) with A, B 64x64 tiles in LDS.
// TA = false: A[m][k] = sA[m][k];  TA = true: A[m][k] = sA[k][m].
// TB = false: B[k][n] = sB[k][n];  TB = true: B[k][n] = sB[n][k].
template <bool TA, bool TB, typename T>
__device__ __forceinline__ void mma64(AccT<T> &acc, const T (*sA)[LDP], const T (*sB)[LDP],
                                      typename Same<T>::type sign = (T)1) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32;
    const int li = l & 15, lk = l >> 4;
#pragma unroll 4
    for (int k0 = 0; k0 < 64; k0 += 4) {
        const int k = k0 + lk;
        T a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int m = r0 + i * 16 + li;
            a[i] = (TA ? sA[k][m] : sA[m][k]) * sign;
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = c0 + j * 16 + li;
            b[j] = TB ? sB[n][k] : sB[k][n];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc.c[i][j] = Mfma16<T>::mma(a[i], b[j], acc.c[i][j]);
    }
}

// global (ld values per row, FP64 or FP32) <-> LDS tile copies, 256 threads
template <typename T, typename G> __device__ __forceinline__ void g2s_tile(T (*s)[LDP], const G *g, int64_t ld) {
    const int t = threadIdx.x;
    const int c4 = (t & 15) * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = i * 16 + (t >> 4);
        if constexpr (sizeof(G) == 8) {
            const double2 *p = (const double2 *)(g + (int64_t)r * ld + c4);
            const double2 x = p[0], y = p[1];
            s[r][c4] = (T)x.x; s[r][c4 + 1] = (T)x.y; s[r][c4 + 2] = (T)y.x; s[r][c4 + 3] = (T)y.y;
        } else {
            const float4 x = *(const float4 *)(g + (int64_t)r * ld + c4);
            s[r][c4] = (T)x.x; s[r][c4 + 1] = (T)x.y; s[r][c4 + 2] = (T)x.z; s[r][c4 + 3] = (T)x.w;
        }
    }
}
// the same copy, transposed: s[c][r] = g[r][c]
template <typename T, typename G> __device__ __forceinline__ void g2s_tile_t(T (*s)[LDP], const G *g, int64_t ld) {
    const int t = threadIdx.x;
    const int c4 = (t & 15) * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = i * 16 + (t >> 4);
        if constexpr (sizeof(G) == 8) {
            const double2 *p = (const double2 *)(g + (int64_t)r * ld + c4);
            const double2 x = p[0], y = p[1];
            s[c4][r] = (T)x.x; s[c4 + 1][r] = (T)x.y; s[c4 + 2][r] = (T)y.x; s[c4 + 3][r] = (T)y.y;
        } else {
            const float4 x = *(const float4 *)(g + (int64_t)r * ld + c4);
            s[c4][r] = (T)x.x; s[c4 + 1][r] = (T)x.y; s[c4 + 2][r] = (T)x.z; s[c4 + 3][r] = (T)x.w;
        }
    }
}
template <typename T, typename G> __device__ __forceinline__ void s2g_tile(G *g, int64_t ld, const T (*s)[LDP]) {
    const int t = threadIdx.x;
    const int c4 = (t & 15) * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = i * 16 + (t >> 4);
        if constexpr (sizeof(G) == 8) {
            double2 *p = (double2 *)(g + (int64_t)r * ld + c4);
            p[0] = make_double2((double)s[r][c4], (double)s[r][c4 + 1]);
            p[1] = make_double2((double)s[r][c4 + 2], (double)s[r][c4 + 3]);
        } else {
            *(float4 *)(g + (int64_t)r * ld + c4) =
                make_float4((float)s[r][c4], (float)s[r][c4 + 1], (float)s[r][c4 + 2], (float)s[r][c4 + 3]);
        }
    }
}
// The same 64x64 tile copy split in two halves, so that the global loads of
// the next tile can be in flight while the current one is multiplied from
// LDS: g2r_tile issues the loads into registers (same thread mapping as
// g2s_tile), r2s_tile writes them to LDS.
template <typename G> struct RegTile { G v[16]; };
template <typename G> __device__ __forceinline__ void g2r_tile(RegTile<G> &x, const G *g, int64_t ld) {
    const int t = threadIdx.x;
    const int c4 = (t & 15) * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = i * 16 + (t >> 4);
        if constexpr (sizeof(G) == 8) {
            const double2 *p = (const double2 *)(g + (int64_t)r * ld + c4);
            const double2 a = p[0], b = p[1];
            x.v[4 * i] = a.x; x.v[4 * i + 1] = a.y; x.v[4 * i + 2] = b.x; x.v[4 * i + 3] = b.y;
        } else {
            const float4 a = *(const float4 *)(g + (int64_t)r * ld + c4);
            x.v[4 * i] = a.x; x.v[4 * i + 1] = a.y; x.v[4 * i + 2] = a.z; x.v[4 * i + 3] = a.w;
        }
    }
}
template <typename T, typename G> __device__ __forceinline__ void r2s_tile(T (*s)[LDP], const RegTile<G> &x) {
    const int t = threadIdx.x;
    const int c4 = (t & 15) * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = i * 16 + (t >> 4);
#pragma unroll
        for (int q = 0; q < 4; ++q) s[r][c4 + q] = (T)x.v[4 * i + q];
    }
}
template <typename T> __device__ __forceinline__ void acc2s(T (*s)[LDP], const AccT<T> &a) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) s[acc_row<T>(i, e)][acc_col(j)] = a.c[i][j][e];
}
template <typename T> __device__ __forceinline__ void s2acc(AccT<T> &a, const T (*s)[LDP]) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) a.c[i][j][e] = s[acc_row<T>(i, e)][acc_col(j)];
}
// global tile (ld values per row) straight into the accumulator layout
template <typename T, typename G> __device__ __forceinline__ void g2acc(AccT<T> &a, const G *g, int64_t ld) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) a.c[i][j][e] = (T)g[(int64_t)acc_row<T>(i, e) * ld + acc_col(j)];
}

// element idx of a slot's K buffer, stored in FP32 when the substitution
// runs in FP32 arithmetic (SubMeta::kf32), else in FP64
__device__ __forceinline__ double kbuf_get(const SubMeta &M, const char *ws, int64_t idx) {
    return M.kf32 ? (double)((const float *)(ws + M.offK))[idx] : ((const double *)(ws + M.offK))[idx];
}

// deterministic block reductions (256 threads); `red` is LDS scratch of 256
__device__ __forceinline__ double block_sum(double v, double *red) {
    const int t = threadIdx.x;
    __syncthreads();
    red[t] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}
__device__ __forceinline__ double block_max(double v, double *red) {
    const int t = threadIdx.x;
    __syncthreads();
    red[t] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) red[t] = fmax(red[t], red[t + s]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}
__device__ __forceinline__ double block_min(double v, double *red) {
    return -block_max(-v, red);
}
