// The learned flip proposal: features of every bit of a batch of states, the
// 3 -> 256 -> 1 perceptron that maps them to flip logits (BF16 matrix
// weights, FP32 biases, activations and sums), its minibatch training
// (forward, binary cross-entropy backward with deterministic reductions,
// Adam in FP32), and the tile attempt masks the annealer reads.
//
// The network is small (1281 parameters) and its inputs have three features,
// so it runs on the vector ALUs: a thread owns samples in the forward pass and
// hidden units in the gradient pass, and the weights sit in LDS.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "device_common.h"

namespace hobo {

constexpr int kHid = 256;
constexpr int kOffB1 = 3 * kHid, kOffW2 = 4 * kHid, kOffB2 = 5 * kHid;
constexpr int kNParam = kOffB2 + 1;  // 1281
constexpr int kPartRow = 1284;       // per-block gradient row: 1281 gradients, loss sum, padding
constexpr int kSPB = 256;            // samples per gradient block

// round to the nearest BF16 value (ties to even), kept as FP32 (finite inputs)
__device__ inline float bf16r(float f) {
  unsigned u = __float_as_uint(f);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(u);
}

struct MlpLds {
  float4 w[kHid];  // W1[0][u], W1[1][u], W1[2][u] (BF16-rounded), b1[u]
  float w2[kHid];  // W2[u] (BF16-rounded)
  float b2;
};

__device__ inline void mlp_stage(MlpLds* L, const float* params) {
  for (int u = threadIdx.x; u < kHid; u += blockDim.x) {
    L->w[u] = make_float4(bf16r(gld(params + u)), bf16r(gld(params + kHid + u)), bf16r(gld(params + 2 * kHid + u)),
                          gld(params + kOffB1 + u));
    L->w2[u] = bf16r(gld(params + kOffW2 + u));
  }
  if (threadIdx.x == 0) L->b2 = gld(params + kOffB2);
}

// logit of one feature vector (hidden units in order, FP32)
__device__ inline float mlp_logit(const MlpLds* L, float f0, float f1, float f2) {
  float acc = 0.0f;
  for (int u = 0; u < kHid; ++u) {
    const float4 w = L->w[u];
    const float pre = fmaf(f2, w.z, fmaf(f1, w.y, fmaf(f0, w.x, w.w)));
    acc = fmaf(L->w2[u], fmaxf(pre, 0.0f), acc);
  }
  return acc + L->b2;
}

// ------------------------------------------------------------ forward
__global__ __launch_bounds__(256) void mlp_forward_kernel(const float* params, const float* feats, long long M,
                                                          float* logits) {
  __shared__ MlpLds L;
  mlp_stage(&L, params);
  __syncthreads();
  // four samples per thread share every LDS read of the weights
  const long long base = (long long)blockIdx.x * 1024 + threadIdx.x;
  float f[4][3];
  float acc[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const long long m = base + 256 * k;
    const bool ok = m < M;
#pragma unroll
    for (int q = 0; q < 3; ++q) f[k][q] = ok ? gld(feats + 3 * m + q) : 0.0f;
    acc[k] = 0.0f;
  }
  for (int u = 0; u < kHid; ++u) {
    const float4 w = L.w[u];
    const float w2 = L.w2[u];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float pre = fmaf(f[k][2], w.z, fmaf(f[k][1], w.y, fmaf(f[k][0], w.x, w.w)));
      acc[k] = fmaf(w2, fmaxf(pre, 0.0f), acc[k]);
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const long long m = base + 256 * k;
    if (m < M) logits[m] = acc[k] + L.b2;
  }
}

// ------------------------------------------------------------ training
// Gradient of the mean BCE loss of minibatch [m0, m0 + mb) over the samples
// of one block of kSPB, written to part[blockIdx.x][...] (gradients in the
// parameter layout, loss sum at 1281).
__global__ __launch_bounds__(256) void mlp_grad_kernel(const float* params, const float* feats, const float* labels,
                                                       long long m0, int mb, float* part) {
  __shared__ MlpLds L;
  __shared__ float sf[kSPB][3];
  __shared__ float sdl[kSPB];
  __shared__ float sloss[kSPB];
  mlp_stage(&L, params);
  const int t = threadIdx.x;
  const int s0 = blockIdx.x * kSPB;
  const int ns = mb - s0 < kSPB ? mb - s0 : kSPB;
  if (t < ns) {
    const long long m = m0 + s0 + t;
    sf[t][0] = gld(feats + 3 * m);
    sf[t][1] = gld(feats + 3 * m + 1);
    sf[t][2] = gld(feats + 3 * m + 2);
  }
  __syncthreads();
  // samples: logit, dloss/dlogit = (sigmoid(l) - y) / mb, loss term
  if (t < ns) {
    const float l = mlp_logit(&L, sf[t][0], sf[t][1], sf[t][2]);
    const float y = gld(labels + m0 + s0 + t);
    const float e = expf(-fabsf(l));
    const float sg = l >= 0.0f ? 1.0f / (1.0f + e) : e / (1.0f + e);
    sdl[t] = (sg - y) / (float)mb;
    sloss[t] = fmaxf(l, 0.0f) + log1pf(e) - y * l;
  }
  __syncthreads();
  // hidden units: sums over the block's samples in sample order
  const int u = t;
  const float4 w = L.w[u];
  const float w2 = L.w2[u];
  float gw1a = 0.0f, gw1b = 0.0f, gw1c = 0.0f, gb1 = 0.0f, gw2 = 0.0f;
  for (int q = 0; q < ns; ++q) {
    const float f0 = sf[q][0], f1 = sf[q][1], f2 = sf[q][2];
    const float pre = fmaf(f2, w.z, fmaf(f1, w.y, fmaf(f0, w.x, w.w)));
    const float dl = sdl[q];
    gw2 = fmaf(dl, fmaxf(pre, 0.0f), gw2);
    const float dp = pre > 0.0f ? dl * w2 : 0.0f;
    gw1a = fmaf(dp, f0, gw1a);
    gw1b = fmaf(dp, f1, gw1b);
    gw1c = fmaf(dp, f2, gw1c);
    gb1 += dp;
  }
  float* row = part + (size_t)blockIdx.x * kPartRow;
  row[u] = gw1a;
  row[kHid + u] = gw1b;
  row[2 * kHid + u] = gw1c;
  row[kOffB1 + u] = gb1;
  row[kOffW2 + u] = gw2;
  if (t == 0) {
    float gb2 = 0.0f, ls = 0.0f;
    for (int q = 0; q < ns; ++q) {
      gb2 += sdl[q];
      ls += sloss[q];
    }
    row[kOffB2] = gb2;
    row[kNParam] = ls;
  }
}

// Sum the block gradients (block order), one Adam step on the FP32 state
// [params | m | v] (rows of kPartRow), and the minibatch's mean loss.
__global__ __launch_bounds__(256) void mlp_adam_kernel(float* state, const float* part, int nblk, int mb, float lr,
                                                       float beta1, float beta2, float eps, float bc1, float bc2,
                                                       float* loss_out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < kNParam) {
    float g = 0.0f;
    for (int b = 0; b < nblk; ++b) g += part[(size_t)b * kPartRow + k];
    float* p = state;
    float* m = state + kPartRow;
    float* v = state + 2 * kPartRow;
    const float mk = beta1 * m[k] + (1.0f - beta1) * g;
    const float vk = beta2 * v[k] + (1.0f - beta2) * g * g;
    m[k] = mk;
    v[k] = vk;
    const float mh = mk / bc1, vh = vk / bc2;
    p[k] -= lr * mh / (sqrtf(vh) + eps);
  }
  if (k == 0 && loss_out) {
    float ls = 0.0f;
    for (int b = 0; b < nblk; ++b) ls += part[(size_t)b * kPartRow + kNParam];
    *loss_out = ls / (float)mb;
  }
}

// Sum the block gradients (block order) into grad [1281] and the mean loss.
__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float* part, int nblk, int mb, float* grad,
                                                         float* loss_out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < kNParam) {
    float g = 0.0f;
    for (int b = 0; b < nblk; ++b) g += part[(size_t)b * kPartRow + k];
    grad[k] = g;
  }
  if (k == 0 && loss_out) {
    float ls = 0.0f;
    for (int b = 0; b < nblk; ++b) ls += part[(size_t)b * kPartRow + kNParam];
    *loss_out = ls / (float)mb;
  }
}

// ------------------------------------------------------------ features
// feats[b][i] = (x_i, beta dE_i, beta ||H_i||); labels[b][i] = x_i != x_after_i
__global__ __launch_bounds__(256) void proposal_features_kernel(const unsigned long long* x, const unsigned long long* xa,
                                                                long long B, int N, const void* de, int de_int,
                                                                double beta, const double* rnorm, float* feats,
                                                                float* labels) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= B * N) return;
  const long long b = e / N;
  const int i = (int)(e - b * N);
  const unsigned long long wv = gld(x + (long long)(i >> 6) * B + b);
  const unsigned xi = (unsigned)(wv >> (i & 63)) & 1u;
  const double d = de_int ? (double)gld(reinterpret_cast<const long long*>(de) + e)
                          : (double)gld(reinterpret_cast<const float*>(de) + e);
  feats[3 * e] = (float)xi;
  feats[3 * e + 1] = (float)(beta * d);
  feats[3 * e + 2] = (float)(beta * gld(rnorm + i));
  if (labels) {
    const unsigned long long wa = gld(xa + (long long)(i >> 6) * B + b);
    labels[e] = (float)(((wv ^ wa) >> (i & 63)) & 1ull);
  }
}

// ------------------------------------------------------------ attempt masks
// One block: 16 replicas (one group) x 16 bits.  The logit of every (replica,
// bit) from its features at the segment start, the group maximum against
// logit(tau), then the masks of the segment's sweeps with the floor draws.
__global__ __launch_bounds__(256) void proposal_mask_kernel(const float* params, const unsigned long long* x,
                                                            long long B, int N, const void* de, int de_int, double beta,
                                                            const double* rnorm, float lthr, double p_floor,
                                                            unsigned long long seed, unsigned long long inst,
                                                            int s0, int nsw, unsigned char* mask) {
  __shared__ MlpLds L;
  __shared__ float slog[16][17];
  mlp_stage(&L, params);
  __syncthreads();
  const int r = threadIdx.x >> 4, c = threadIdx.x & 15;
  const int i = blockIdx.x * 16 + c;
  const int tile = blockIdx.y;
  const long long b = (long long)tile * 16 + r;
  float lg = -INFINITY;
  if (i < N && b < B) {
    const long long e = b * N + i;
    const unsigned long long wv = gld(x + (long long)(i >> 6) * B + b);
    const float f0 = (float)((wv >> (i & 63)) & 1ull);
    const double d = de_int ? (double)gld(reinterpret_cast<const long long*>(de) + e)
                            : (double)gld(reinterpret_cast<const float*>(de) + e);
    lg = mlp_logit(&L, f0, (float)(beta * d), (float)(beta * gld(rnorm + i)));
  }
  slog[r][c] = lg;
  __syncthreads();
  if (r == 0 && i < N) {
    float mx = -INFINITY;
    for (int q = 0; q < 16; ++q) mx = fmaxf(mx, slog[q][c]);
    const bool hot = mx >= lthr;
    for (int k = 0; k < nsw; ++k) {
      bool on = hot;
      if (!on && p_floor > 0.0) {
        const U64x4 o = philox((unsigned long long)tile, (unsigned long long)(s0 + k), (unsigned long long)(i >> 2),
                               2ull, seed, inst);
        const double u = (double)(o.w[i & 3] >> 11) * 0x1.0p-53;
        on = u < p_floor;
      }
      mask[((size_t)tile * nsw + k) * N + i] = on ? 1 : 0;
    }
  }
}

// ------------------------------------------------------------ launchers
int mlp_forward(const float* params, const float* feats, long long M, float* logits, hipStream_t st,
                std::string* err) {
  if (M > 0)
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)((M + 1023) / 1024)), dim3(256), 0, st, params, feats, M,
                       logits);
  return hip_fail(hipGetLastError(), err, "mlp forward");
}

size_t mlp_train_workspace(int batch) { return (size_t)((batch + kSPB - 1) / kSPB) * kPartRow * sizeof(float); }

int mlp_train_step(float* state, const float* feats, const float* labels, long long m0, int mb, float lr,
                   float beta1, float beta2, float eps, float bc1, float bc2, float* part, float* loss_out,
                   hipStream_t st, std::string* err) {
  const int nblk = (mb + kSPB - 1) / kSPB;
  hipLaunchKernelGGL(mlp_grad_kernel, dim3((unsigned)nblk), dim3(256), 0, st, state, feats, labels, m0, mb, part);
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((unsigned)((kNParam + 255) / 256)), dim3(256), 0, st, state, part, nblk,
                     mb, lr, beta1, beta2, eps, bc1, bc2, loss_out);
  return hip_fail(hipGetLastError(), err, "mlp train step");
}

int mlp_grad(const float* params, const float* feats, const float* labels, int mb, float* part, float* grad,
             float* loss_out, hipStream_t st, std::string* err) {
  const int nblk = (mb + kSPB - 1) / kSPB;
  hipLaunchKernelGGL(mlp_grad_kernel, dim3((unsigned)nblk), dim3(256), 0, st, params, feats, labels, 0ll, mb, part);
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((unsigned)((kNParam + 255) / 256)), dim3(256), 0, st, part, nblk, mb,
                     grad, loss_out);
  return hip_fail(hipGetLastError(), err, "mlp grad");
}

int proposal_features(const unsigned long long* x, const unsigned long long* xa, long long B, int N, const void* de,
                      int de_int, double beta, const double* rnorm, float* feats, float* labels, hipStream_t st,
                      std::string* err) {
  const long long tot = B * N;
  hipLaunchKernelGGL(proposal_features_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, x, xa, B, N, de,
                     de_int, beta, rnorm, feats, labels);
  return hip_fail(hipGetLastError(), err, "proposal features");
}

int proposal_masks(const float* params, const unsigned long long* x, long long B, int N, const void* de, int de_int,
                   double beta, const double* rnorm, float lthr, double p_floor, unsigned long long seed,
                   unsigned long long inst, int s0, int nsw, unsigned char* mask, hipStream_t st, std::string* err) {
  const unsigned tiles = (unsigned)((B + 15) / 16);
  hipLaunchKernelGGL(proposal_mask_kernel, dim3((unsigned)((N + 15) / 16), tiles), dim3(256), 0, st, params, x, B, N,
                     de, de_int, beta, rnorm, lthr, p_floor, seed, inst, s0, nsw, mask);
  return hip_fail(hipGetLastError(), err, "proposal masks");
}

}  // namespace hobo
