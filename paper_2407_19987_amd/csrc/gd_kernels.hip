// Gradient-descent search (Sec. II.D.2) on the multilinear extension of the
// HOBO energy, E(p) = sum_S w_S prod_{i in S} p_i over p in [0, 1]^N:
//   g_i(p) = sum_{S containing i} w_S prod_{j in S, j != i} p_j,
//   one step: p_i <- min(1, max(0, p_i - eta g_i(p))) for every i at once.
// Layout: p is [N][B] (variable-major), so a wave's 64 lanes -- 64 replicas --
// read and write consecutive doubles.  A work-group takes 64 replicas and a
// slice of the variables: it stages the replicas' whole p in LDS ([N][64]
// doubles), then each wave walks the record lists of its variables; every
// lane reads the same record (scalar loads) and its own p entries
// (consecutive LDS doubles).  FP64 with separately rounded products and sums,
// the order of the records being the monomial order: this file is built with
// -ffp-contract=off (HIP's __dmul_rn and __dadd_rn are plain operators, and
// the default contraction would fuse them into multiply-adds).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "device_common.h"

namespace hobo {

constexpr int kGDWaves = 16;     // waves per work-group (one variable each)
constexpr int kGDSliceVars = 16; // variables per work-group (grid.y covers N)

// MAXO: largest monomial order of the tensor (records carry up to MAXO - 1
// other variables), so the product loop has a fixed trip count with
// wave-uniform guards
template <int MAXO>
__global__ __launch_bounds__(64 * kGDWaves) void gd_step_kernel(GDArgs a) {
  extern __shared__ double sp[];  // [N][64], then a row of 64 ones
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const long long b0 = (long long)blockIdx.x * 64;
  const long long b = b0 + lane;
  const bool live = b < a.B;
  const int N = a.n_vars;
  for (int e = threadIdx.x; e < N * 64; e += blockDim.x) {
    const int i = e >> 6, l = e & 63;
    const long long bb = b0 + l;
    sp[e] = bb < a.B ? gld(a.p_in + (long long)i * a.B + bb) : 0.0;
  }
  for (int e = threadIdx.x; e < 64; e += blockDim.x) sp[N * 64 + e] = 1.0;
  __syncthreads();
  const int i0 = blockIdx.y * kGDSliceVars;
  const int i1 = i0 + kGDSliceVars < N ? i0 + kGDSliceVars : N;
  for (int i = i0 + w; i < i1; i += kGDWaves) {
    const int r0 = __builtin_amdgcn_readfirstlane(gld(a.ptr + i));
    const int r1 = __builtin_amdgcn_readfirstlane(gld(a.ptr + i + 1));
    double g = 0.0;
    // the records come through scalar loads, eight at a time, the next eight
    // issued before the current ones are used; the lanes read their own p
    // entries (consecutive LDS doubles)
    typedef const __attribute__((address_space(4))) u4* ConstU4;
    const ConstU4 srec = (ConstU4)a.rec;
    // product of a record: its weight times the other variables' p.  Every
    // slot is read, an unused one from the row of ones (the choice is made on
    // the wave-uniform index), and multiplying by 1.0 is exact, so the reads
    // need no branch and overlap
    auto term = [&](const u4& rc) {
      double prod = __hiloint2double((int)rc[1], (int)rc[0]);
      const int nn = (int)(rc[2] & 0xFFu);
#pragma unroll
      for (int q = 0; q < MAXO - 1; ++q) {
        const unsigned o = q < 3 ? (rc[2] >> (8 * (q + 1))) & 0xFFu : (rc[3] >> (8 * (q - 3))) & 0xFFu;
        const unsigned oe = q < nn ? o : (unsigned)N;
        prod = __dmul_rn(prod, sp[oe * 64 + lane]);
      }
      return prod;
    };
    int r = r0;
    if (r + 8 <= r1) {
      u4 nx[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) nx[q] = srec[r + q];
      for (; r + 8 <= r1; r += 8) {
        u4 cu[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) cu[q] = nx[q];
#pragma unroll
        for (int q = 0; q < 8; ++q) asm volatile("" : "+s"(cu[q]));
        if (r + 16 <= r1)
#pragma unroll
          for (int q = 0; q < 8; ++q) nx[q] = srec[r + 8 + q];
        // the eight products' LDS reads overlap; the sum keeps the record order
        double t[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) t[q] = term(cu[q]);
#pragma unroll
        for (int q = 0; q < 8; ++q) g = __dadd_rn(g, t[q]);
      }
    }
    for (; r < r1; ++r) {
      const u4 rc = srec[r];
      g = __dadd_rn(g, term(rc));
    }
    if (live) {
      if (a.mode == 1) {
        a.p_out[(long long)i * a.B + b] = g;
      } else {
        const double v = __dadd_rn(sp[i * 64 + lane], -__dmul_rn(a.eta, g));
        a.p_out[(long long)i * a.B + b] = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
      }
    }
  }
}

// p[i][b] = (r >> 11) 2^-53 from Philox4x64-10 word i % 4 at counter
// (b, 0, i / 4, 3), key (seed, 0)
__global__ void gd_init_kernel(int N, long long B, unsigned long long seed, double* p) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int nq = (N + 3) / 4;
  if (idx >= (long long)nq * B) return;
  const int q = (int)(idx / B);
  const long long b = idx - (long long)q * B;
  const U64x4 o = philox((unsigned long long)b, 0ull, (unsigned long long)q, 3ull, seed, 0ull);
  for (int e = 0; e < 4; ++e) {
    const int i = 4 * q + e;
    if (i < N) p[(long long)i * B + b] = (double)(o.w[e] >> 11) * 0x1.0p-53;
  }
}

// x = [p > 1/2], [W][B] words
__global__ void gd_round_kernel(int N, long long B, const double* p, unsigned long long* x) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int W = (N + 63) / 64;
  if (idx >= (long long)W * B) return;
  const int w = (int)(idx / B);
  const long long b = idx - (long long)w * B;
  unsigned long long v = 0;
  for (int i = 64 * w; i < N && i < 64 * (w + 1); ++i)
    if (gld(p + (long long)i * B + b) > 0.5) v |= 1ull << (i & 63);
  x[idx] = v;
}

int launch_gd_step(const GDArgs& a, std::string* err) {
  const dim3 grid((unsigned)((a.B + 63) / 64), (unsigned)((a.n_vars + kGDSliceVars - 1) / kGDSliceVars));
  const size_t lds = (size_t)(a.n_vars + 1) * 64 * sizeof(double);  // up to 128.5 KB at N = 256
  static std::once_flag once;
  static hipError_t attr = hipSuccess;
  std::call_once(once, [] {
    const int bytes = (int)((kMaxVars + 1) * 64 * sizeof(double));
    const void* fns[4] = {reinterpret_cast<const void*>(&gd_step_kernel<2>),
                          reinterpret_cast<const void*>(&gd_step_kernel<3>),
                          reinterpret_cast<const void*>(&gd_step_kernel<4>),
                          reinterpret_cast<const void*>(&gd_step_kernel<kMaxOrder>)};
    for (const void* f : fns)
      if (attr == hipSuccess) attr = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  });
  if (int s = hip_fail(attr, err, "hipFuncSetAttribute(gradient step LDS)")) return s;
  const dim3 blk(64 * kGDWaves);
  const hipStream_t st = (hipStream_t)a.stream;
  if (a.max_order <= 2)
    hipLaunchKernelGGL(gd_step_kernel<2>, grid, blk, lds, st, a);
  else if (a.max_order == 3)
    hipLaunchKernelGGL(gd_step_kernel<3>, grid, blk, lds, st, a);
  else if (a.max_order == 4)
    hipLaunchKernelGGL(gd_step_kernel<4>, grid, blk, lds, st, a);
  else
    hipLaunchKernelGGL(gd_step_kernel<kMaxOrder>, grid, blk, lds, st, a);
  return hip_fail(hipGetLastError(), err, "gradient step launch");
}

int launch_gd_init(int n_vars, int64_t B, uint64_t seed, double* p, void* stream, std::string* err) {
  const long long n = (long long)((n_vars + 3) / 4) * B;
  hipLaunchKernelGGL(gd_init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, n_vars,
                     (long long)B, (unsigned long long)seed, p);
  return hip_fail(hipGetLastError(), err, "gradient start launch");
}

int launch_gd_round(int n_vars, int64_t B, const double* p, uint64_t* x, void* stream, std::string* err) {
  const long long n = (long long)((n_vars + 63) / 64) * B;
  hipLaunchKernelGGL(gd_round_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, n_vars,
                     (long long)B, p, reinterpret_cast<unsigned long long*>(x));
  return hip_fail(hipGetLastError(), err, "rounding launch");
}

}  // namespace hobo
