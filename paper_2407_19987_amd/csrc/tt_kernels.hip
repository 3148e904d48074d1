// Batched contraction of the tensor-train form of the HOBO tensor
// (Sec. VI.E-F): for each replica x,
//   E(x) = prod_k M_k(x),  M_k(x) = sum_i x_i G_k[:, i, :]   (r_{k-1} x r_k),
// evaluated left to right as a row vector v <- v M_k(x), O(d n r^2) per
// replica instead of the dense tensor's O(n^d).  One thread per replica;
// every lane of a wave walks the same core entries in the same order (the
// bit only selects a zero or the vector entry), so the rows are wave-uniform
// and come through scalar registers: no per-lane data return.  Each row is
// read whole (RMAX columns; those past the rank add products that are never
// used, so no branch per column), a few rows at a time; a row past the rank
// reads the zeros the upload appends after the cores.  FP64 throughout, one
// fused multiply-add per (variable, row, column) in that order.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "device_common.h"

namespace hobo {

struct TTParams {
  const double* cores;  // the cores, then kTTMaxRank zeros
  const unsigned long long* bits;
  double* e_out;
  long long B;
  int n, order, W;
  int ranks[kMaxOrder + 1];
  long long off[kMaxOrder];
  long long zero_off;  // offset of the zeros
};

template <int RMAX>
__global__ __launch_bounds__(256) void tt_energy_kernel(TTParams p) {
  typedef const __attribute__((address_space(4))) double* CD;
  const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = b < p.B;
  unsigned long long xw[4] = {0, 0, 0, 0};
  for (int w = 0; w < p.W && w < 4; ++w) xw[w] = live ? gld(p.bits + (long long)w * p.B + b) : 0ull;
  double v[RMAX];
#pragma unroll
  for (int a = 0; a < RMAX; ++a) v[a] = a == 0 ? 1.0 : 0.0;
  const CD zero = (CD)p.cores + p.zero_off;
  int rp = 1;
  for (int k = 0; k < p.order; ++k) {
    const int r = p.ranks[k + 1];
    const CD g = (CD)p.cores + p.off[k];
    double w[RMAX];
#pragma unroll
    for (int c = 0; c < RMAX; ++c) w[c] = 0.0;
    for (int i = 0; i < p.n; ++i) {
      const int wi = i >> 6;
      const unsigned long long word = wi == 0 ? xw[0] : wi == 1 ? xw[1] : wi == 2 ? xw[2] : xw[3];
      const bool on = (word >> (i & 63)) & 1ull;
      // rows in groups of G (G x RMAX doubles in scalar registers); a row of
      // the group past rp reads zeros (v[a] is +0 there and fma(+0, 0, w) is
      // w, w being never -0)
      constexpr int G = RMAX >= 32 ? 1 : (RMAX >= 16 ? 2 : 4);
#pragma unroll
      for (int a0 = 0; a0 < RMAX; a0 += G) {
        if (a0 < rp) {
          double rw[G][RMAX];
#pragma unroll
          for (int q = 0; q < G; ++q) {
            const CD row = a0 + q < rp ? g + ((long long)(a0 + q) * p.n + i) * r : zero;
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
  p.zero_off = (long long)tt->h_cores.size();
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
