// llr_mlp.hip -- warm-start network a(u, 1/L) for the Robbins-Monro iteration
// (the paper's initial values a_i-bar, Sec. 2.4, learned from converged a_k):
//   uh = (u - 0.6)/0.1, lh = (1/L - 0.0875)/0.0375
//   h1 = tanh(W1 x + b1)        64, FP32 vector units
//   h2 = tanh(W2 h1 + b2)       64x64: bfloat16 MFMA (FP32 accumulate) or FP32
//   a  = 1 + 0.1 (W3 h2 + b3)   FP32
// Parameter vector (4417 FP32): W1[64][2], b1, W2[64][64], b2, W3[64], b3.
// Training: mean squared error on a, full-batch Adam; gradients in FP32.
#include <hip/hip_runtime.h>

#include "llr_internal.hpp"

namespace llr {

constexpr int H = kMlpH;
constexpr int OW1 = 0, OB1 = OW1 + 2 * H, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H, OB3 = OW3 + H;
constexpr int kRows = 64;     // samples per chunk
constexpr int kMB = 256;      // threads per block

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even
    return (short)(u >> 16);
}

struct Chunk {
    float x[kRows][2];
    float h1[kRows][H];
    float h2[kRows][H];
    float y[kRows];
};

// Forward of rows [0, nr) of a chunk whose inputs are already in c.x.
__device__ void fwd_chunk(const float* __restrict__ w, Chunk& c, int nr, int bf16) {
    const int t = threadIdx.x;
    for (int e = t; e < kRows * H; e += kMB) {
        const int i = e / H, j = e - i * H;
        float v = 0.f;
        if (i < nr) v = tanhf(w[OW1 + 2 * j] * c.x[i][0] + w[OW1 + 2 * j + 1] * c.x[i][1] + w[OB1 + j]);
        c.h1[i][j] = v;
    }
    __syncthreads();
    if (bf16) {
        // wave wv computes rows 16 wv .. 16 wv + 15, all 64 columns, with
        // v_mfma_f32_16x16x16_bf16: A[i][k] = h1, B[k][j] = W2[j][k].
        const int lane = t & 63, wv = t >> 6;
        const int li = lane & 15, kq = lane >> 4;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                bf16x4 av, bv;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int k = 16 * ks + 4 * kq + r;
                    av[r] = to_bf16(c.h1[16 * wv + li][k]);
                    bv[r] = to_bf16(w[OW2 + H * (16 * nt + li) + k]);
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 16 * wv + 4 * kq + r, j = 16 * nt + li;
                c.h2[i][j] = tanhf(acc[r] + w[OB2 + j]);
            }
        }
    } else {
        for (int e = t; e < kRows * H; e += kMB) {
            const int i = e / H, j = e - i * H;
            float z = w[OB2 + j];
            for (int k = 0; k < H; ++k) z += w[OW2 + H * j + k] * c.h1[i][k];
            c.h2[i][j] = tanhf(z);
        }
    }
    __syncthreads();
    if (t < kRows) {
        float y = w[OB3];
        for (int k = 0; k < H; ++k) y += w[OW3 + k] * c.h2[t][k];
        c.y[t] = y;
    }
    __syncthreads();
}

__device__ __forceinline__ void load_inputs(Chunk& c, const float* u, const float* invL, int row0, int nr) {
    if ((int)threadIdx.x < kRows) {
        const int i = threadIdx.x;
        c.x[i][0] = i < nr ? (u[row0 + i] - 0.6f) / 0.1f : 0.f;
        c.x[i][1] = i < nr ? (invL[row0 + i] - 0.0875f) / 0.0375f : 0.f;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kMB) void k_mlp_forward(const float* __restrict__ w, const float* __restrict__ u,
                                                      const float* __restrict__ invL, int n, int bf16,
                                                      double* __restrict__ a_out) {
    __shared__ Chunk c;
    const int row0 = blockIdx.x * kRows;
    const int nr = min(kRows, n - row0);
    load_inputs(c, u, invL, row0, nr);
    fwd_chunk(w, c, nr, bf16);
    if ((int)threadIdx.x < nr) a_out[row0 + threadIdx.x] = 1.0 + 0.1 * (double)c.y[threadIdx.x];
}

// One block: loss and gradient over all n samples, chunk by chunk (fixed order).
__global__ __launch_bounds__(kMB) void k_mlp_loss_grad(const float* __restrict__ w, const float* __restrict__ u,
                                                        const float* __restrict__ invL, const double* __restrict__ a,
                                                        int n, int bf16, float* __restrict__ grad,
                                                        double* __restrict__ loss_out) {
    __shared__ Chunk c;
    __shared__ float d2[kRows][H];
    __shared__ float g[kMlpNP];
    __shared__ float dy[kRows];
    __shared__ double lpart[kRows];
    const int t = threadIdx.x;
    for (int e = t; e < kMlpNP; e += kMB) g[e] = 0.f;
    double loss = 0.0;
    for (int row0 = 0; row0 < n; row0 += kRows) {
        const int nr = min(kRows, n - row0);
        load_inputs(c, u, invL, row0, nr);
        fwd_chunk(w, c, nr, bf16);
        if (t < kRows) {
            float r = 0.f;
            double rr = 0.0;
            if (t < nr) {
                rr = (1.0 + 0.1 * (double)c.y[t]) - a[row0 + t];
                r = (float)rr;
            }
            lpart[t] = rr * rr;
            dy[t] = 2.f * r / (float)n * 0.1f;
        }
        __syncthreads();
        if (t == 0) {
            double sacc = 0.0;
            for (int i = 0; i < nr; ++i) sacc += lpart[i];
            loss += sacc / (double)n;
        }
        // output layer
        if (t < H) {
            float s = 0.f;
            for (int i = 0; i < nr; ++i) s += dy[i] * c.h2[i][t];
            g[OW3 + t] += s;
        }
        if (t == H) {
            float s = 0.f;
            for (int i = 0; i < nr; ++i) s += dy[i];
            g[OB3] += s;
        }
        for (int e = t; e < kRows * H; e += kMB) {
            const int i = e / H, k = e - i * H;
            d2[i][k] = i < nr ? dy[i] * w[OW3 + k] * (1.f - c.h2[i][k] * c.h2[i][k]) : 0.f;
        }
        __syncthreads();
        // hidden layer 2: dW2[j][k] = sum_i d2[i][j] h1[i][k]; db2[j] = sum_i d2[i][j]
        for (int e = t; e < H * H; e += kMB) {
            const int j = e / H, k = e - j * H;
            float s = 0.f;
            for (int i = 0; i < nr; ++i) s += d2[i][j] * c.h1[i][k];
            g[OW2 + e] += s;
        }
        if (t < H) {
            float s = 0.f;
            for (int i = 0; i < nr; ++i) s += d2[i][t];
            g[OB2 + t] += s;
        }
        __syncthreads();
        // back to layer 1: d1[i][k] = (sum_j W2[j][k] d2[i][j]) (1 - h1^2); reuse c.h2 as d1
        for (int e = t; e < kRows * H; e += kMB) {
            const int i = e / H, k = e - i * H;
            float s = 0.f;
            for (int j = 0; j < H; ++j) s += w[OW2 + H * j + k] * d2[i][j];
            c.h2[i][k] = i < nr ? s * (1.f - c.h1[i][k] * c.h1[i][k]) : 0.f;
        }
        __syncthreads();
        if (t < H) {
            float sb = 0.f, s0 = 0.f, s1 = 0.f;
            for (int i = 0; i < nr; ++i) {
                const float d = c.h2[i][t];
                sb += d;
                s0 += d * c.x[i][0];
                s1 += d * c.x[i][1];
            }
            g[OB1 + t] += sb;
            g[OW1 + 2 * t] += s0;
            g[OW1 + 2 * t + 1] += s1;
        }
        __syncthreads();
    }
    for (int e = t; e < kMlpNP; e += kMB) grad[e] = g[e];
    if (t == 0) *loss_out = loss;
}

// Adam (Kingma & Ba), step t >= 1
__global__ void k_mlp_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                           const float* __restrict__ g, int t, float lr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kMlpNP) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    const float mi = b1 * m[i] + (1.f - b1) * g[i];
    const float vi = b2 * v[i] + (1.f - b2) * g[i] * g[i];
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Xavier-uniform weights from Philox (kind 4, w0 = parameter index), zero biases.
__global__ void k_mlp_init(uint32_t k0, uint32_t k1, float* __restrict__ w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kMlpNP) return;
    double lim = 0.0;
    if (i < OB1) lim = sqrt(6.0 / (2 + H));
    else if (i >= OW2 && i < OB2) lim = sqrt(6.0 / (H + H));
    else if (i >= OW3 && i < OB3) lim = sqrt(6.0 / (H + 1));
    if (lim == 0.0) { w[i] = 0.f; return; }
    const uint4 r = philox10(make_uint4((uint32_t)i, ctr1_word(0, 0, kMlp, 0), 0u, 0u), k0, k1);
    const double uu = ((double)r.x + 0.5) * 0x1p-32;
    w[i] = (float)__fma_rn(2.0 * lim, uu, -lim);
}

void launch_mlp_init(uint64_t seed, float* w, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_init, dim3((kMlpNP + 255) / 256), dim3(256), 0, st, (uint32_t)seed,
                       (uint32_t)(seed >> 32), w);
}
void launch_mlp_forward(const float* w, const float* u, const float* invL, int n, int bf16, double* a_out,
                        hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mlp_forward, dim3((n + kRows - 1) / kRows), dim3(kMB), 0, st, w, u, invL, n, bf16, a_out);
}
void launch_mlp_loss_grad(const float* w, const float* u, const float* invL, const double* a, int n, int bf16,
                          float* grad, double* loss, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_loss_grad, dim3(1), dim3(kMB), 0, st, w, u, invL, a, n, bf16, grad, loss);
}
void launch_mlp_adam(float* w, float* m, float* v, const float* g, int t, float lr, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpNP + 255) / 256), dim3(256), 0, st, w, m, v, g, t, lr);
}

}  // namespace llr
