// FP32 tile products on the FP16 matrix cores, for the substitutions of the
// symmetric route (L^-1 K and its right solve by L^-T, whose result is
// rounded to FP16 for the sign iteration anyway).
//
// Each FP32 operand value x is held as the unevaluated sum of two FP16
// values, hi = fp16(x) and lo = fp16(x - hi), and a product of two such
// values as hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_f16 with FP32
// accumulation (the lo*lo term, below 2^-22 relative, is dropped). That keeps
// about 22 significant bits per operand, against 24 in FP32, for three
// products at the FP16 rate (16x that of v_mfma_f32_16x16x4_f32). FP16 has
// a narrow exponent range, so the caller scales an operand by a power of two
// that brings its largest magnitude into [1, 2) (the pair then holds every
// entry x to within max(2^-22 |x|, 2^-25)) and divides the result by it.
//
// Tiles are 64 x 64 in LDS, row n holding 64 contraction values k, in hi
// and lo planes: an MFMA operand (16 rows, 8 consecutive k per lane) is one
// 16-byte read per plane. The 16-byte chunk c of row n sits at chunk
// position c ^ ((n ^ n >> 3) & 7), so the 16 rows that a read touches cover
// all bank groups.
#pragma once
#include "dev_common.h"

typedef _Float16 v4h __attribute__((ext_vector_type(4)));

struct HLTile {
    _Float16 h[64 * 64];
    _Float16 l[64 * 64];
};

__device__ __forceinline__ int hl_pos(int n, int k) {
    return n * 64 + ((((k >> 3) ^ ((n ^ (n >> 3)) & 7))) << 3) + (k & 7);
}

// four consecutive k of row n (k0 a multiple of 4), each value times sc
__device__ __forceinline__ void hl_put4(HLTile &s, int n, int k0, float a, float b, float c, float d, float sc) {
    const float x[4] = {a * sc, b * sc, c * sc, d * sc};
    v4h h, l;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        h[q] = (_Float16)x[q];
        l[q] = (_Float16)(x[q] - (float)h[q]);
    }
    const int p = hl_pos(n, k0);
    *(v4h *)&s.h[p] = h;
    *(v4h *)&s.l[p] = l;
}
__device__ __forceinline__ void hl_put1(HLTile &s, int n, int k, float x) {
    const _Float16 h = (_Float16)x;
    const int p = hl_pos(n, k);
    s.h[p] = h;
    s.l[p] = (_Float16)(x - (float)h);
}

// s(n, k) = sc * g[n][k]: a global FP32 tile as it stands (256 threads)
__device__ __forceinline__ void g2hl(HLTile &s, const float *g, int64_t ld, float sc) {
    const int t = threadIdx.x, c4 = (t & 15) * 4;
    float4 v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = *(const float4 *)(g + (int64_t)(i * 16 + (t >> 4)) * ld + c4);
#pragma unroll
    for (int i = 0; i < 4; ++i) hl_put4(s, i * 16 + (t >> 4), c4, v[i].x, v[i].y, v[i].z, v[i].w, sc);
}
// s(n, k) = sc * g[k][n]: the transposed tile; thread t reads the 4 x 4
// block at rows 4 (t / 16), columns 4 (t % 16)
__device__ __forceinline__ void g2hl_t(HLTile &s, const float *g, int64_t ld, float sc) {
    const int t = threadIdx.x, r4 = (t >> 4) * 4, c4 = (t & 15) * 4;
    float4 v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = *(const float4 *)(g + (int64_t)(r4 + i) * ld + c4);
    hl_put4(s, c4 + 0, r4, v[0].x, v[1].x, v[2].x, v[3].x, sc);
    hl_put4(s, c4 + 1, r4, v[0].y, v[1].y, v[2].y, v[3].y, sc);
    hl_put4(s, c4 + 2, r4, v[0].z, v[1].z, v[2].z, v[3].z, sc);
    hl_put4(s, c4 + 3, r4, v[0].w, v[1].w, v[2].w, v[3].w, sc);
}
// the second half of g2hl for a tile already loaded by g2r_tile
__device__ __forceinline__ void r2hl(HLTile &s, const RegTile<float> &x, float sc) {
    const int t = threadIdx.x, c4 = (t & 15) * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        hl_put4(s, i * 16 + (t >> 4), c4, x.v[4 * i], x.v[4 * i + 1], x.v[4 * i + 2], x.v[4 * i + 3], sc);
}
// accumulator tile (FP32 16x16 block layout) into s, as it stands:
// s(row, col) = sc * D[row][col]
__device__ __forceinline__ void acc2hl(HLTile &s, const AccT<float> &a, float sc) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) hl_put1(s, acc_row<float>(i, e), acc_col(j), a.c[i][j][e] * sc);
}
// and transposed: s(col, row) = sc * D[row][col] (a lane's four elements of
// a block are consecutive rows of one column)
__device__ __forceinline__ void acc2hl_t(HLTile &s, const AccT<float> &a, float sc) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            hl_put4(s, acc_col(j), acc_row<float>(i, 0), a.c[i][j][0], a.c[i][j][1], a.c[i][j][2], a.c[i][j][3], sc);
}

// acc += A B for the 64 x 64 tiles A[m][k] = sA(m, k), B[k][n] = sB(n, k);
// wave w owns the 32 x 32 quadrant (w / 2, w % 2) of the output as 2 x 2
// blocks of 16 x 16 in the layout of AccT<float>.
__device__ __forceinline__ void mma64_hl(AccT<float> &acc, const HLTile &sA, const HLTile &sB) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32;
    const int li = l & 15, kg = (l >> 4) * 8;
#pragma unroll
    for (int k0 = 0; k0 < 64; k0 += 32) {
        v8h ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int p = hl_pos(r0 + i * 16 + li, k0 + kg);
            ah[i] = *(const v8h *)&sA.h[p];
            al[i] = *(const v8h *)&sA.l[p];
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int p = hl_pos(c0 + j * 16 + li, k0 + kg);
            bh[j] = *(const v8h *)&sB.h[p];
            bl[j] = *(const v8h *)&sB.l[p];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                v4f c = acc.c[i][j];
                c = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[i], bh[j], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], bl[j], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], bh[j], c, 0, 0, 0);
                acc.c[i][j] = c;
            }
    }
}

// Power of two that brings a largest magnitude amax into [1, 2) (1 for 0 or
// a non-finite amax), and its inverse.
__device__ __forceinline__ void hl_scale(float amax, float &sc, float &inv) {
    if (!(amax > 0.0f) || !__builtin_isfinite(amax)) {
        sc = inv = 1.0f;
        return;
    }
    int e;
    (void)frexpf(amax, &e);   // amax in [2^(e-1), 2^e)
    sc = ldexpf(1.0f, 1 - e);
    inv = ldexpf(1.0f, e - 1);
}
