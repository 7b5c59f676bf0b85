// Learned spectral bounds: forward, loss + hand-written backward, Adam.
//
// The paper only requires that A is rescaled before the sign iteration so that
// it converges (Sec. III-B.2, after Eq. NS2). The 12 -> 64 -> 64 -> 2 SiLU
// perceptron predicts the normalised extreme eigenvalues of A_J from O(n^2)
// features; the scale it implies is clamped at the Gershgorin scale.
// Parameter packing: W1[64][12], b1[64], W2[64][64], b2[64], W3[2][64], b3[2].
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/nolsm.h"

#define NF 12
#define NH 64
#define NO 2
#define OFF_B1 (NH * NF)
#define OFF_W2 (OFF_B1 + NH)
#define OFF_B2 (OFF_W2 + NH * NH)
#define OFF_W3 (OFF_B2 + NH)
#define OFF_B3 (OFF_W3 + NO * NH)
#define NPAR (OFF_B3 + NO)
static_assert(NPAR == NOLSM_MLP_NPARAM, "parameter packing");

__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
    const float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// one thread per sample; parameters staged in LDS
__global__ __launch_bounds__(256) void k_mlp_forward(const float *__restrict__ prm, const float *__restrict__ norm,
                                                     const float *__restrict__ x, int B, float *__restrict__ out) {
    __shared__ float P[NPAR];
    __shared__ float nm[2 * NF];
    for (int i = threadIdx.x; i < NPAR; i += blockDim.x) P[i] = prm[i];
    for (int i = threadIdx.x; i < 2 * NF; i += blockDim.x) nm[i] = norm[i];
    __syncthreads();
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float xs[NF];
    for (int i = 0; i < NF; ++i) xs[i] = (x[(int64_t)b * NF + i] - nm[i]) / nm[NF + i];
    float h1[NH];
    for (int j = 0; j < NH; ++j) {
        float z = P[OFF_B1 + j];
        for (int i = 0; i < NF; ++i) z += P[j * NF + i] * xs[i];
        h1[j] = silu(z);
    }
    float o0 = P[OFF_B3], o1 = P[OFF_B3 + 1];
    for (int j = 0; j < NH; ++j) {
        float z = P[OFF_B2 + j];
        for (int i = 0; i < NH; ++i) z += P[OFF_W2 + j * NH + i] * h1[i];
        const float h = silu(z);
        o0 += P[OFF_W3 + j] * h;
        o1 += P[OFF_W3 + NH + j] * h;
    }
    out[(int64_t)b * 2] = o0;
    out[(int64_t)b * 2 + 1] = o1;
}

// Loss and gradient over a batch, one workgroup of 16 waves. Wave w takes
// samples w, w+16, ...; lane j owns hidden unit j and keeps its share of the
// gradient in registers (gW2[:, j], gW1[j, :], gW3[:, j], gb1[j], gb2[j]);
// the 16 per-wave gradients are then summed in wave order (deterministic).
#define NWAVE 16
__global__ __launch_bounds__(1024) void k_mlp_loss_grad(const float *__restrict__ prm, const float *__restrict__ norm,
                                                        const float *__restrict__ x, const float *__restrict__ y,
                                                        int B, float *__restrict__ grad, float *__restrict__ loss_out) {
    __shared__ float P[NPAR];
    __shared__ float W2T[NH * NH];
    __shared__ float nm[2 * NF];
    __shared__ float xs[NWAVE][NF];
    __shared__ float h1s[NWAVE][NH];
    __shared__ float gz2s[NWAVE][NH];
    __shared__ float G[NPAR];
    __shared__ float lw[NWAVE];
    const int t = threadIdx.x, w = t >> 6, j = t & 63;
    for (int i = t; i < NPAR; i += 1024) P[i] = prm[i];
    for (int i = t; i < NH * NH; i += 1024) {
        const int r = i / NH, c = i % NH;
        W2T[c * NH + r] = prm[OFF_W2 + i];
    }
    for (int i = t; i < 2 * NF; i += 1024) nm[i] = norm[i];
    __syncthreads();
    float gW2[NH], gW1[NF], gW3[NO], gb1 = 0, gb2 = 0, gb3[NO] = {0, 0}, lsum = 0;
    for (int k = 0; k < NH; ++k) gW2[k] = 0;
    for (int i = 0; i < NF; ++i) gW1[i] = 0;
    gW3[0] = gW3[1] = 0;
    const float scale = 2.0f / (float)(B * NO);
    const int rounds = (B + NWAVE - 1) / NWAVE;
    for (int rd = 0; rd < rounds; ++rd) {
        const int b = rd * NWAVE + w;
        const bool valid = b < B;
        if (valid && j < NF) xs[w][j] = (x[(int64_t)b * NF + j] - nm[j]) / nm[NF + j];
        __syncthreads();
        float z1 = 0, h1 = 0;
        if (valid) {
            z1 = P[OFF_B1 + j];
            for (int i = 0; i < NF; ++i) z1 += P[j * NF + i] * xs[w][i];
            h1 = silu(z1);
            h1s[w][j] = h1;
        }
        __syncthreads();
        float z2 = 0, h2 = 0, go0 = 0, go1 = 0;
        if (valid) {
            z2 = P[OFF_B2 + j];
            for (int i = 0; i < NH; ++i) z2 += W2T[i * NH + j] * h1s[w][i];
            h2 = silu(z2);
            float o0 = P[OFF_W3 + j] * h2, o1 = P[OFF_W3 + NH + j] * h2;
            for (int off = 32; off > 0; off >>= 1) {
                o0 += __shfl_xor(o0, off, 64);
                o1 += __shfl_xor(o1, off, 64);
            }
            o0 += P[OFF_B3];
            o1 += P[OFF_B3 + 1];
            const float d0 = o0 - y[(int64_t)b * 2], d1 = o1 - y[(int64_t)b * 2 + 1];
            const float w0 = d0 < 0 ? 4.0f : 1.0f, w1 = d1 < 0 ? 4.0f : 1.0f;
            lsum += w0 * d0 * d0 + w1 * d1 * d1;
            go0 = scale * w0 * d0;
            go1 = scale * w1 * d1;
            gW3[0] += go0 * h2;
            gW3[1] += go1 * h2;
            gb3[0] += go0;
            gb3[1] += go1;
            const float gh2 = go0 * P[OFF_W3 + j] + go1 * P[OFF_W3 + NH + j];
            gz2s[w][j] = gh2 * dsilu(z2);
        }
        __syncthreads();
        if (valid) {
            float gh1 = 0;
            for (int k = 0; k < NH; ++k) {
                const float g = gz2s[w][k];
                gh1 += g * P[OFF_W2 + k * NH + j];
                gW2[k] += g * h1;
            }
            gb2 += gz2s[w][j];
            const float gz1 = gh1 * dsilu(z1);
            for (int i = 0; i < NF; ++i) gW1[i] += gz1 * xs[w][i];
            gb1 += gz1;
        }
        __syncthreads();
    }
    // deterministic reduction in wave order
    for (int ww = 0; ww < NWAVE; ++ww) {
        if (w == ww) {
            const bool first = ww == 0;
            for (int i = 0; i < NF; ++i) G[j * NF + i] = (first ? 0.0f : G[j * NF + i]) + gW1[i];
            G[OFF_B1 + j] = (first ? 0.0f : G[OFF_B1 + j]) + gb1;
            for (int k = 0; k < NH; ++k) G[OFF_W2 + k * NH + j] = (first ? 0.0f : G[OFF_W2 + k * NH + j]) + gW2[k];
            G[OFF_B2 + j] = (first ? 0.0f : G[OFF_B2 + j]) + gb2;
            G[OFF_W3 + j] = (first ? 0.0f : G[OFF_W3 + j]) + gW3[0];
            G[OFF_W3 + NH + j] = (first ? 0.0f : G[OFF_W3 + NH + j]) + gW3[1];
            if (j == 0) {
                G[OFF_B3] = (first ? 0.0f : G[OFF_B3]) + gb3[0];
                G[OFF_B3 + 1] = (first ? 0.0f : G[OFF_B3 + 1]) + gb3[1];
            }
        }
        __syncthreads();
    }
    // per-wave loss: lane sums are lane-uniform; lane 0 holds the wave total
    if (j == 0) lw[w] = lsum;
    __syncthreads();
    for (int i = t; i < NPAR; i += 1024) grad[i] = G[i];
    if (t == 0) {
        float L = 0;
        for (int ww = 0; ww < NWAVE; ++ww) L += lw[ww];
        *loss_out = L / (float)(B * NO);
    }
}

// omb1 = 1 - beta1 and omb2 = 1 - beta2 are formed on the host from the
// double-precision hyper-parameters and rounded once to FP32.
__global__ void k_mlp_adam(float *p, const float *g, float *m, float *v, float lr, float b1, float b2, float omb1,
                           float omb2, float eps, float bc1, float bc2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPAR) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + omb1 * gi;
    const float vi = b2 * v[i] + omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

extern "C" int nolsm_mlp_forward(const float *d_params, const float *d_norm, const float *d_x, int32_t B,
                                 float *d_out, void *stream) {
    if (!d_params || !d_norm || !d_x || !d_out || B < 0) return NOLSM_E_ARG;
    if (B == 0) return NOLSM_OK;
    hipLaunchKernelGGL(k_mlp_forward, dim3((B + 255) / 256), dim3(256), 0, (hipStream_t)stream, d_params, d_norm,
                       d_x, B, d_out);
    return hipGetLastError() == hipSuccess ? NOLSM_OK : NOLSM_E_HIP;
}

extern "C" int nolsm_mlp_loss_grad(const float *d_params, const float *d_norm, const float *d_x, const float *d_y,
                                   int32_t B, float *d_grad, float *d_loss, void *stream) {
    if (!d_params || !d_norm || !d_x || !d_y || !d_grad || !d_loss || B < 1) return NOLSM_E_ARG;
    hipLaunchKernelGGL(k_mlp_loss_grad, dim3(1), dim3(1024), 0, (hipStream_t)stream, d_params, d_norm, d_x, d_y, B,
                       d_grad, d_loss);
    return hipGetLastError() == hipSuccess ? NOLSM_OK : NOLSM_E_HIP;
}

extern "C" int nolsm_mlp_adam(float *d_params, const float *d_grad, float *d_m, float *d_v, int32_t t, double lr,
                              double beta1, double beta2, double eps, void *stream) {
    if (!d_params || !d_grad || !d_m || !d_v || t < 1) return NOLSM_E_ARG;
    const float bc1 = (float)(1.0 - pow(beta1, (double)t));
    const float bc2 = (float)(1.0 - pow(beta2, (double)t));
    const float omb1 = (float)(1.0 - beta1), omb2 = (float)(1.0 - beta2);
    hipLaunchKernelGGL(k_mlp_adam, dim3((NPAR + 255) / 256), dim3(256), 0, (hipStream_t)stream, d_params, d_grad,
                       d_m, d_v, (float)lr, (float)beta1, (float)beta2, omb1, omb2, (float)eps, bc1, bc2);
    return hipGetLastError() == hipSuccess ? NOLSM_OK : NOLSM_E_HIP;
}
