// Batched contraction of the tensor-train form of the HOBO tensor
// (Sec. VI.E-F): for each replica x,
//   E(x) = prod_k M_k(x),  M_k(x) = sum_i x_i G_k[:, i, :]   (r_{k-1} x r_k),
// evaluated left to right as a row vector v <- v M_k(x), O(d n r^2) per
// replica instead of the dense tensor's O(n^d).  One thread per replica;
// every lane of a wave walks the same core entries in the same order (the
// bit only selects a zero or the vector entry).  The work-group copies each
// core to LDS a slice of variables at a time and its four waves read the
// rows from there (one address per wave: broadcast reads), instead of each
// wave fetching them through the scalar cache.  FP64 throughout, one fused
// multiply-add per (variable, row, column) in that order.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "device_common.h"

namespace hobo {

struct TTParams {
  const double* cores;
  const unsigned long long* bits;
  double* e_out;
  long long B;
  int n, order, W;
  int ranks[kMaxOrder + 1];
  long long off[kMaxOrder];
};

constexpr int kTTStage = 4096;  // doubles of a core slice staged in LDS (32 KB)

template <int RMAX>
__global__ __launch_bounds__(256) void tt_energy_kernel(TTParams p) {
  // G_k[a][i0 .. i0 + ni)[c], rows (a, i) of r doubles, then RMAX zeros: a
  // row is read whole (RMAX columns, no branch per column); the columns at or
  // past r accumulate values that are never used
  __shared__ double sg[kTTStage + RMAX];
  for (int e = threadIdx.x; e < RMAX; e += blockDim.x) sg[kTTStage + e] = 0.0;
  const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = b < p.B;
  unsigned long long xw[4] = {0, 0, 0, 0};
  for (int w = 0; w < p.W && w < 4; ++w) xw[w] = live ? gld(p.bits + (long long)w * p.B + b) : 0ull;
  double v[RMAX];
#pragma unroll
  for (int a = 0; a < RMAX; ++a) v[a] = a == 0 ? 1.0 : 0.0;
  int rp = 1;
  for (int k = 0; k < p.order; ++k) {
    const int r = p.ranks[k + 1];
    const double* g = p.cores + p.off[k];
    const int ni = kTTStage / (rp * r);  // variables per slice (ranks <= 32: at least 4)
    double w[RMAX];
#pragma unroll
    for (int c = 0; c < RMAX; ++c) w[c] = 0.0;
    for (int i0 = 0; i0 < p.n; i0 += ni) {
      const int nn = p.n - i0 < ni ? p.n - i0 : ni;
      __syncthreads();  // the previous slice has been read
      for (int e = threadIdx.x; e < rp * nn * r; e += blockDim.x) {
        const int a = e / (nn * r);
        sg[e] = g[((long long)a * p.n + i0) * r + (e - a * nn * r)];
      }
      __syncthreads();
      for (int ii = 0; ii < nn; ++ii) {
        const int i = i0 + ii;
        const int wi = i >> 6;
        const unsigned long long word = wi == 0 ? xw[0] : wi == 1 ? xw[1] : wi == 2 ? xw[2] : xw[3];
        const bool on = (word >> (i & 63)) & 1ull;
        // rows in groups of G, each group's reads in flight together; a row
        // of the group at or past rp reads the zeros after the slice (v[a] is
        // +0 there and fma(+0, 0, w) is w, w being never -0)
        constexpr int G = RMAX >= 32 ? 2 : (RMAX >= 4 ? 4 : RMAX);
#pragma unroll
        for (int a0 = 0; a0 < RMAX; a0 += G) {
          if (a0 < rp) {
            double rw[G][RMAX];
#pragma unroll
            for (int q = 0; q < G; ++q) {
              const double* row = a0 + q < rp ? sg + ((a0 + q) * nn + ii) * r : sg + kTTStage;
#pragma unroll
              for (int c = 0; c < RMAX; ++c) rw[q][c] = row[c];
            }
#pragma unroll
            for (int q = 0; q < G; ++q) {
              const double va = on ? v[a0 + q] : 0.0;
#pragma unroll
              for (int c = 0; c < RMAX; ++c) w[c] = fma(va, rw[q][c], w[c]);
            }
          }
        }
      }
    }
#pragma unroll
    for (int c = 0; c < RMAX; ++c) v[c] = c < r ? w[c] : 0.0;
    rp = r;
  }
  if (live) p.e_out[b] = v[0];
}

int launch_tt_energy(const TTDev* tt, const uint64_t* bits, int64_t B, double* e_out, void* stream,
                     std::string* err) {
  TTParams p{};
  p.cores = tt->d_cores;
  p.bits = reinterpret_cast<const unsigned long long*>(bits);
  p.e_out = e_out;
  p.B = B;
  p.n = tt->n;
  p.order = tt->order;
  p.W = (tt->n + 63) / 64;
  int rmax = 1;
  for (int k = 0; k <= tt->order; ++k) {
    p.ranks[k] = tt->ranks[(size_t)k];
    rmax = rmax > tt->ranks[(size_t)k] ? rmax : tt->ranks[(size_t)k];
  }
  for (int k = 0; k < tt->order; ++k) p.off[k] = tt->core_off[(size_t)k];
  hipStream_t st = (hipStream_t)stream;
  const dim3 grid((unsigned)((B + 255) / 256)), block(256);
  if (rmax <= 4)
    hipLaunchKernelGGL(tt_energy_kernel<4>, grid, block, 0, st, p);
  else if (rmax <= 8)
    hipLaunchKernelGGL(tt_energy_kernel<8>, grid, block, 0, st, p);
  else if (rmax <= 16)
    hipLaunchKernelGGL(tt_energy_kernel<16>, grid, block, 0, st, p);
  else
    hipLaunchKernelGGL(tt_energy_kernel<32>, grid, block, 0, st, p);
  return hip_fail(hipGetLastError(), err, "TT energy launch");
}

}  // namespace hobo
