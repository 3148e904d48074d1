// Launch of the batched energy and local-field kernels (hobo_energy,
// hobo_local_fields; the kernel is in eval_kernel.h) and the FP64 / int64
// term-by-term energy kernel.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <string>
#include <type_traits>

#include "eval_kernel.h"

namespace hobo {

__global__ void reduce_partials(const void* work, void* e_out, int ncg, long long B, int integer, int scale) {
  long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  if (integer) {
    long long s = 0;
    for (int c = 0; c < ncg; ++c) s += reinterpret_cast<const long long*>(work)[(long long)c * B + b];
    reinterpret_cast<long long*>(e_out)[b] = s / scale;
  } else {
    double s = 0.0;
    for (int c = 0; c < ncg; ++c) s += reinterpret_cast<const double*>(work)[(long long)c * B + b];
    reinterpret_cast<double*>(e_out)[b] = s / (double)scale;
  }
}

// ============================================================ term-loop energy
// FP64 (real) or int64 (integer) energies summed monomial by monomial.  A
// block of 256 threads (one replica each) walks one group of kTermGroup
// monomials, staged through LDS so that every record is read once per block
// and broadcast to all lanes; the group sums are then added in group order.
// The grouping depends only on the monomial count, so the result of a row
// does not depend on the batch it is evaluated in.
__global__ __launch_bounds__(256) void term_masks_one(TermJob J) {
  if ((long long)blockIdx.x * 256 >= J.B) return;
  term_masks(J, blockIdx.x);
}

__global__ __launch_bounds__(256) void term_partial_one(TermJob J) {
  if ((long long)blockIdx.x * 256 >= J.B || (int)blockIdx.y * kTermGroup >= J.n_mono) return;
  term_partial(J, blockIdx.x, blockIdx.y);
}

// e_out[b] = sum over groups of the partial sums, in group order
__global__ void term_reduce_one(TermJob J, void* out) {
  const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= J.B) return;
  const int G = term_groups(J.n_mono);
  if (J.integer) {
    long long s = 0;
    for (int q = 0; q < G; ++q) s += reinterpret_cast<const long long*>(J.part)[(long long)q * J.B + b];
    reinterpret_cast<long long*>(out)[b] = s;
  } else {
    double s = 0.0;
    for (int q = 0; q < G; ++q) s += reinterpret_cast<const double*>(J.part)[(long long)q * J.B + b];
    reinterpret_cast<double*>(out)[b] = s;
  }
}

size_t eval_workspace_bytes(const Tensor* t, int mode, int64_t B, int ct) {
  (void)mode;
  int T = (t->n_vars + 15) / 16;
  int ncg = (T + ct - 1) / ct;
  return ncg > 1 ? (size_t)(T > ncg ? T : ncg) * (size_t)B * 8 : 0;
}

int launch_eval(const EvalArgs& a, std::string* err) {
  const Packed* pk = a.pk;
  const Tensor* t = a.t;
  hipStream_t st = (hipStream_t)a.stream;
  const int T = (t->n_vars + 15) / 16;
  int ct = a.ct, rt = a.rt;
  if (pk->prec == P_INT8X4 && ct > 4) ct = 4;
  const int ncg = (T + ct - 1) / ct;
  EvalParams ep{};
  ep.tiles = reinterpret_cast<const unsigned char*>(pk->d_tiles);
  ep.chunks = pk->d_chunks;
  ep.runs = reinterpret_cast<const unsigned long long*>(pk->d_runs);
  ep.nchunks = pk->nchunks;
  ep.n_vars = t->n_vars;
  ep.W = (t->n_vars + 63) / 64;
  ep.ncg = ncg;
  ep.n_tiles = T;
  ep.n_tile_buf = (unsigned)pk->ntiles;
  ep.B = a.B;
  ep.bits = reinterpret_cast<const unsigned long long*>(a.bits);
  ep.de_out = a.de_out;
  ep.e_out = a.e_out;
  ep.work = a.work;
  ep.integer = t->integer ? 1 : 0;
  ep.want_e = a.e_out != nullptr;
  ep.inv_scale = std::ldexp(1.0, -pk->scale_exp);
  int r = -1;
  switch (pk->prec) {
    case P_FP32: r = dispatch_eval_prec<P_FP32>(ep, pk->mode, rt, ct, a.B, st); break;
    case P_BF16X2: r = dispatch_eval_prec<P_BF16X2>(ep, pk->mode, rt, ct, a.B, st); break;
    case P_BF16X3: r = dispatch_eval_prec<P_BF16X3>(ep, pk->mode, rt, ct, a.B, st); break;
    case P_FP16X2: r = dispatch_eval_prec<P_FP16X2>(ep, pk->mode, rt, ct, a.B, st); break;
    case P_INT8X4: r = dispatch_eval_prec<P_INT8X4>(ep, pk->mode, rt, ct, a.B, st); break;
    default: break;
  }
  if (r != 0) {
    *err = "no kernel for this precision / tile shape";
    return HOBO_ERR_UNSUPPORTED;
  }
  int s = hip_fail(hipGetLastError(), err, "eval kernel launch");
  if (s) return s;
  if (ncg > 1 && a.e_out) {
    // fields: one partial per column group (scaled by kLcm); energy: one per tile
    int scale = pk->mode == M_FIELDS ? kLcm : 1;
    int nparts = pk->mode == M_FIELDS ? ncg : T;
    hipLaunchKernelGGL(reduce_partials, dim3((unsigned)((a.B + 255) / 256)), dim3(256), 0, st, a.work, a.e_out,
                       nparts, (long long)a.B, ep.integer, scale);
    s = hip_fail(hipGetLastError(), err, "reduce kernel launch");
  }
  return s;
}

// ============================================================ no-allocation scratch
// Workspace of hobo_energy_noalloc: one array per GPU, held until the
// process ends, shared by every call on that GPU (calls that overlap on one
// GPU race on it).  In host code the symbol's name is not a device address;
// noalloc_scratch resolves the address once per device with
// hipGetSymbolAddress and every launch takes that pointer.
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

int noalloc_scratch(void** out, std::string* err) {
  constexpr int kMaxDev = 64;
  static std::mutex mu;
  static void* addr[kMaxDev] = {};
  int dev = 0;
  if (int s = hip_fail(hipGetDevice(&dev), err, "hipGetDevice")) return s;
  if (dev < 0 || dev >= kMaxDev) {
    *err = "device index beyond the no-allocation scratch table";
    return HOBO_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    if (int s = hip_fail(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), err, "hipGetSymbolAddress(scratch)")) return s;
    addr[dev] = p;
  }
  *out = addr[dev];
  return HOBO_OK;
}

__global__ void fill_zero_u64(unsigned long long* p, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

int launch_zero_u64(void* p, long long n, void* stream, std::string* err) {
  if (n <= 0) return HOBO_OK;
  hipLaunchKernelGGL(fill_zero_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     static_cast<unsigned long long*>(p), n);
  return hip_fail(hipGetLastError(), err, "zero fill launch");
}

size_t term_workspace_bytes(const Tensor* t, int64_t B) {
  return term_mask_offset(t->n_mono(), B) + term_mask_bytes(t->n_vars, B);
}

int launch_term_energy(const TermArgs& a, std::string* err) {
  hipStream_t st = (hipStream_t)a.stream;
  TermJob J{};
  J.rec = a.td->d_rec;
  J.n_mono = a.td->n_mono;
  J.W = (a.t->n_vars + 63) / 64;
  J.integer = a.t->integer ? 1 : 0;
  J.B = a.B;
  J.bits = reinterpret_cast<const unsigned long long*>(a.bits);
  J.part = a.work;
  const int G = term_groups(J.n_mono);
  hipLaunchKernelGGL(term_masks_one, dim3((unsigned)((a.B + 255) / 256)), dim3(256), 0, st, J);
  hipLaunchKernelGGL(term_partial_one, dim3((unsigned)((a.B + 255) / 256), (unsigned)G), dim3(256), 0, st, J);
  hipLaunchKernelGGL(term_reduce_one, dim3((unsigned)((a.B + 255) / 256)), dim3(256), 0, st, J, a.e_out);
  return hip_fail(hipGetLastError(), err, "term energy launch");
}

}  // namespace hobo

