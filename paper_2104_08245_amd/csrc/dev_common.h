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
// 64x64 FP64 tiles on the FP64 MFMA (v_mfma_f64_16x16x4_f64), 256 threads.
// Wave w owns the 32x32 quadrant (w>>1, w&1) as 2x2 blocks of 16x16. In a
// block, A[i][k] comes from lane i + 16k, B[k][j] from lane j + 16k, and
// element e of lane l is D[l/16 + 4e][l%16] (measured on gfx950; the FP32
// 16x16x4 instruction instead returns D[4(l/16) + e][l%16]).
// LDS tiles are [64][LDP] doubles, LDP = 65 (one pad double per row).
// ---------------------------------------------------------------------------
#define LDP 65

struct Acc64 {
    v4d c[2][2];
};

__device__ __forceinline__ void acc_zero(Acc64 &a) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) a.c[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};
}

// row/col of element e of block (i, j) for this lane
__device__ __forceinline__ int acc_row(int i, int e) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    return (w >> 1) * 32 + i * 16 + (l >> 4) + 4 * e;
}
__device__ __forceinline__ int acc_col(int j) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    return (w & 1) * 32 + j * 16 + (l & 15);
}

// acc += op(A) * op(B) with A, B 64x64 tiles in LDS.
// TA = false: A[m][k] = sA[m][k];  TA = true: A[m][k] = sA[k][m].
// TB = false: B[k][n] = sB[k][n];  TB = true: B[k][n] = sB[n][k].
template <bool TA, bool TB>
__device__ __forceinline__ void mma64(Acc64 &acc, const double (*sA)[LDP], const double (*sB)[LDP],
                                      double sign = 1.0) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32;
    const int li = l & 15, lk = l >> 4;
#pragma unroll 4
    for (int k0 = 0; k0 < 64; k0 += 4) {
        const int k = k0 + lk;
        double a[2], b[2];
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
            for (int j = 0; j < 2; ++j)
                acc.c[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc.c[i][j], 0, 0, 0);
    }
}

// global (ld doubles per row) <-> LDS tile copies, 256 threads
__device__ __forceinline__ void g2s_tile(double (*s)[LDP], const double *g, int64_t ld) {
    const int t = threadIdx.x;
    const int c4 = (t & 15) * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = i * 16 + (t >> 4);
        const double2 *p = (const double2 *)(g + (int64_t)r * ld + c4);
        const double2 x = p[0], y = p[1];
        s[r][c4] = x.x; s[r][c4 + 1] = x.y; s[r][c4 + 2] = y.x; s[r][c4 + 3] = y.y;
    }
}
__device__ __forceinline__ void s2g_tile(double *g, int64_t ld, const double (*s)[LDP]) {
    const int t = threadIdx.x;
    const int c4 = (t & 15) * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = i * 16 + (t >> 4);
        double2 *p = (double2 *)(g + (int64_t)r * ld + c4);
        p[0] = make_double2(s[r][c4], s[r][c4 + 1]);
        p[1] = make_double2(s[r][c4 + 2], s[r][c4 + 3]);
    }
}
__device__ __forceinline__ void acc2s(double (*s)[LDP], const Acc64 &a) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) s[acc_row(i, e)][acc_col(j)] = a.c[i][j][e];
}
__device__ __forceinline__ void s2acc(Acc64 &a, const double (*s)[LDP]) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) a.c[i][j][e] = s[acc_row(i, e)][acc_col(j)];
}

// global tile (ld doubles per row) straight into the accumulator layout
__device__ __forceinline__ void g2acc(Acc64 &a, const double *g, int64_t ld) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) a.c[i][j][e] = g[(int64_t)acc_row(i, e) * ld + acc_col(j)];
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
