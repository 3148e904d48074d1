#pragma once
// Device building blocks shared by the gfx950 (CDNA4) kernels of the HOBO engine.
//
// All contractions share one wave-level scheme (see pack.cpp for the layouts):
//   acc[16 replicas x 16 columns] += Y[replicas x 32 (or 64) monomials] * M[monomials x columns]
// on the matrix cores, where Y is generated on the fly from the replicas' bits
// (a run of eight monomials is one byte of the bit vector times the product
// of the run's prefix bits; a 256-entry LDS table turns that byte into eight
// BF16 / INT8 ones and zeros), and M streams from HBM/L2 in pre-swizzled
// per-lane order, prefetched one chunk ahead into registers.
//
// MFMA lane layouts (16x16 output tiles; checked on gfx950):
//   A: lane l holds row l%16, K group l/16;   B: lane l holds column l%16,
//   same K group;   C: lane l holds rows 4*(l/16)+r, r=0..3, column l%16.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "hobo_internal.h"
#include "../../include/hobo.h"

namespace hobo {

typedef __bf16 bf16x8 __attribute__((__vector_size__(8 * sizeof(__bf16))));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef int i4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

// Global-memory loads through the global address space: generic (flat)
// loads would also count against the LDS wait counter, so every LDS access
// would wait for the whole in-flight coefficient stream.
#define HOBO_GLOBAL __attribute__((address_space(1)))
template <class T> __device__ inline T gld(const T* p) { return *(const HOBO_GLOBAL T*)(p); }
template <class T> __device__ inline void gst(T* p, T v) { *(HOBO_GLOBAL T*)(p) = v; }

constexpr int kLcm = 420;  // lcm(1..7): scales the per-order energy sums to integers

// ------------------------------------------------------------ precision traits
template <int P> struct PT;
template <> struct PT<P_FP32> { static constexpr int RPC = 4, NP = 1, NLD = 2; };
template <> struct PT<P_BF16X2> { static constexpr int RPC = 4, NP = 2, NLD = 2; };
template <> struct PT<P_BF16X3> { static constexpr int RPC = 4, NP = 3, NLD = 3; };
template <> struct PT<P_INT8X4> { static constexpr int RPC = 8, NP = 4, NLD = 4; };
template <> struct PT<P_FP16X2> { static constexpr int RPC = 4, NP = 2, NLD = 2; };

// per-tile B registers: NLD x 16 bytes per lane
template <int P> struct BTile { u4 v[PT<P>::NLD]; };

// accumulator of one 16x16 output tile
template <int P> struct AccT { f4 v; };
template <> struct AccT<P_INT8X4> { i4 v[4]; };

// A operand of one 16-row tile for one chunk
template <int P> struct AOp { u4 v; };  // bf16x8 / 16 int8 / (FP32: low byte = run mask)

// ------------------------------------------------------------ LDS tables
struct Luts {
  u4 bf16[256];         // byte -> eight 16-bit values 0 / 1.0 (BF16, or FP16 for FP16X2)
  unsigned long long i8[256];  // byte -> eight INT8 values 0 / 1
};

// the 16-bit pattern of 1.0 in the operand type of precision P
template <int P> constexpr unsigned one16() { return P == P_FP16X2 ? 0x3C00u : 0x3F80u; }

template <int P = P_BF16X2>
__device__ inline void build_luts(Luts* L) {
  constexpr unsigned one = one16<P>();
  for (int m = threadIdx.x; m < 256; m += blockDim.x) {
    u4 v;
    for (int d = 0; d < 4; ++d) {
      unsigned lo = (m >> (2 * d)) & 1u, hi = (m >> (2 * d + 1)) & 1u;
      v[d] = (lo ? one : 0u) | (hi ? one << 16 : 0u);
    }
    L->bf16[m] = v;
    unsigned long long b = 0;
    for (int e = 0; e < 8; ++e) b |= (unsigned long long)((m >> e) & 1) << (8 * e);
    L->i8[m] = b;
  }
}

// Eight-monomial mask of run `d` for the replica whose bits start at `rb`
// (32 bytes in LDS): byte beta of the bits if every prefix bit is set.
__device__ inline unsigned run_mask(unsigned long long d, const unsigned char* rb) {
  unsigned np = (unsigned)(d >> 8) & 0xFFu;
  if (np == kRunNull) return 0u;
  if (np == kRunConst) return 1u;
  unsigned m = rb[d & 0xFFu];
  for (unsigned p = 0; p < np; ++p) {
    unsigned v = (unsigned)(d >> (16 + 8 * p)) & 0xFFu;
    if (!((rb[v >> 3] >> (v & 7u)) & 1u)) m = 0u;
  }
  return m;
}

template <int P>
__device__ inline AOp<P> gen_a(const unsigned long long* runs, int run_base, int g,
                               const unsigned char* rb, const Luts* L) {
  AOp<P> a;
  if constexpr (P == P_FP32) {
    a.v = u4{run_mask(runs[run_base + g], rb), 0u, 0u, 0u};
  } else if constexpr (P == P_INT8X4) {
    unsigned m0 = run_mask(runs[run_base + 2 * g], rb);
    unsigned m1 = run_mask(runs[run_base + 2 * g + 1], rb);
    unsigned long long lo = L->i8[m0], hi = L->i8[m1];
    a.v = u4{(unsigned)lo, (unsigned)(lo >> 32), (unsigned)hi, (unsigned)(hi >> 32)};
  } else {
    a.v = L->bf16[run_mask(runs[run_base + g], rb)];
  }
  return a;
}

template <int P>
__device__ inline void load_tile(BTile<P>& b, const unsigned char* tile, int lane) {
  if constexpr (P == P_FP32) {
    const u4* p = reinterpret_cast<const u4*>(tile + lane * 32);
    b.v[0] = gld(p);
    b.v[1] = gld(p + 1);
  } else {
#pragma unroll
    for (int q = 0; q < PT<P>::NLD; ++q) b.v[q] = gld(reinterpret_cast<const u4*>(tile + q * 1024 + lane * 16));
  }
}

template <int P>
__device__ inline void mma(AccT<P>& c, const AOp<P>& a, const BTile<P>& b) {
  if constexpr (P == P_FP32) {
    const unsigned m = a.v[0];
    for (int s = 0; s < 8; ++s) {
      float av = ((m >> s) & 1u) ? 1.0f : 0.0f;
      float bv = __uint_as_float(b.v[s >> 2][s & 3]);
      c.v = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, c.v, 0, 0, 0);
    }
  } else if constexpr (P == P_INT8X4) {
    i4 av = __builtin_bit_cast(i4, a.v);
    for (int q = 0; q < 4; ++q)
      c.v[q] = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, __builtin_bit_cast(i4, b.v[q]), c.v[q], 0, 0, 0);
  } else if constexpr (P == P_FP16X2) {
    f16x8 av = __builtin_bit_cast(f16x8, a.v);
    for (int q = 0; q < 2; ++q)
      c.v = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, __builtin_bit_cast(f16x8, b.v[q]), c.v, 0, 0, 0);
  } else {
    bf16x8 av = __builtin_bit_cast(bf16x8, a.v);
    for (int q = 0; q < PT<P>::NP; ++q)
      c.v = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, __builtin_bit_cast(bf16x8, b.v[q]), c.v, 0, 0, 0);
  }
}

template <int P> __device__ inline void acc_zero(AccT<P>& c) {
  if constexpr (P == P_INT8X4) {
    for (int q = 0; q < 4; ++q) c.v[q] = i4{0, 0, 0, 0};
  } else {
    c.v = f4{0.f, 0.f, 0.f, 0.f};
  }
}

// value r (0..3) of an accumulator as double (exact for INT8 limbs up to 2^53);
// FP16X2 sums are of coefficients times 2^scale_exp and are multiplied by
// scl = 2^-scale_exp (exact), the other precisions ignore scl
template <int P> __device__ inline double acc_f(const AccT<P>& c, int r, double scl = 1.0) {
  if constexpr (P == P_INT8X4) {
    long long v = (long long)c.v[0][r] + ((long long)c.v[1][r] << 8) + ((long long)c.v[2][r] << 16) +
                  ((long long)c.v[3][r] << 24);
    return (double)v;
  } else if constexpr (P == P_FP16X2) {
    return (double)c.v[r] * scl;
  } else {
    return (double)c.v[r];
  }
}
template <int P> __device__ inline long long acc_i(const AccT<P>& c, int r, double scl = 1.0) {
  if constexpr (P == P_INT8X4) {
    return (long long)c.v[0][r] + ((long long)c.v[1][r] << 8) + ((long long)c.v[2][r] << 16) +
           ((long long)c.v[3][r] << 24);
  } else if constexpr (P == P_FP16X2) {
    return (long long)__builtin_rint((double)c.v[r] * scl);
  } else {
    return (long long)__builtin_rintf(c.v[r]);
  }
}

__device__ inline int bit_at(const unsigned char* rb, int v) { return (rb[v >> 3] >> (v & 7)) & 1; }

// sum over the 16 lanes of a lane group
__device__ inline double group_sum(double v) {
  for (int o = 8; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline long long group_sum_i(long long v) {
  for (int o = 8; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// load the bits of `nrep` replicas starting at r0 into LDS (32 bytes each)
__device__ inline void load_bits(unsigned long long* dst, const unsigned long long* bits, int W,
                                 long long B, long long r0, int nrep, int lane) {
  for (int e = lane; e < nrep * 4; e += 64) {
    int rho = e >> 2, w = e & 3;
    long long r = r0 + rho;
    dst[e] = (w < W && r < B) ? gld(bits + (long long)w * B + r) : 0ull;
  }
}

// ============================================================ Philox4x64-10
// Salmon et al., SC'11: ten rounds of two 64x64->128-bit products with
// multipliers M0, M1, a word permutation and a key XOR; the key is bumped by
// two Weyl constants between rounds.
struct U64x4 { unsigned long long w[4]; };
__device__ inline U64x4 philox(unsigned long long c0, unsigned long long c1, unsigned long long c2,
                               unsigned long long c3, unsigned long long k0, unsigned long long k1) {
  const unsigned long long M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const unsigned long long W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    unsigned long long hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    unsigned long long hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    unsigned long long n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  return U64x4{{c0, c1, c2, c3}};
}

// ------------------------------------------------------------ wave primitives
// DPP controls (gfx9 encoding): rotate a 16-lane row by 8, mirror each half
// row, exchange lanes 2 apart / 1 apart inside each quad
constexpr int kDppRowRor8 = 0x128, kDppHalfMirror = 0x141, kDppQuadXor2 = 0x4E, kDppQuadXor1 = 0xB1;
constexpr int kDppRowRor4 = 0x124, kDppRowRor8b = 0x128, kDppRowRor12 = 0x12C;

template <int CTRL> __device__ inline double dpp_d(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL> __device__ inline unsigned dpp_u(unsigned v) {
  return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}

// Sums over the 16 lanes of each lane group of four per-lane values (the
// four output rows a lane holds): on return lane j of the group holds the
// sum of row j >> 2.  Five DPP exchanges (a reduce-scatter) instead of four
// separate all-reductions.
__device__ inline double rowsum4(double v0, double v1, double v2, double v3, int j) {
  const bool h8 = (j & 8) != 0;
  double k0 = h8 ? v2 : v0, k1 = h8 ? v3 : v1;
  const double s0 = h8 ? v0 : v2, s1 = h8 ? v1 : v3;
  k0 += dpp_d<kDppRowRor8>(s0);
  k1 += dpp_d<kDppRowRor8>(s1);
  const bool h4 = (j & 4) != 0;
  double k = h4 ? k1 : k0;
  const double s = h4 ? k0 : k1;
  k += dpp_d<kDppHalfMirror>(s);
  k += dpp_d<kDppQuadXor2>(k);
  k += dpp_d<kDppQuadXor1>(k);
  return k;
}

// Wave-uniform value loaded through the vector memory path (so that its
// wait does not serialise with LDS traffic): the lane offset is opaque zero.
template <class T> __device__ inline T vload_uniform(const T* p, long long idx) {
  const int z = (int)__builtin_amdgcn_mbcnt_lo(0u, 0u);
  return gld(p + idx + z);
}

// LDS-only wait plus a work-group barrier; outstanding global loads (the
// coefficient stream) stay in flight
__device__ inline void lds_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ inline ChunkMeta unpack_meta(unsigned long long raw) {
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)raw);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(raw >> 32));
  ChunkMeta m;
  m.tile_off = lo;
  m.t_lo = (uint8_t)(hi & 0xFF);
  m.t_hi = (uint8_t)((hi >> 8) & 0xFF);
  m.seg_end = (uint8_t)((hi >> 16) & 0xFF);
  m.bit = (uint8_t)(hi >> 24);
  return m;
}

// term-loop kernels: monomials per partial sum, records staged in LDS at a time
constexpr int kTermGroup = 4096;
__host__ __device__ inline int term_groups(int n_mono) { return n_mono > 0 ? (n_mono + kTermGroup - 1) / kTermGroup : 1; }

struct TermJob {             // one instance's term-loop energy of a batch
  const TermRec* rec;
  int n_mono;
  int W;
  int integer;
  int pad;
  long long B;
  const unsigned long long* bits;  // [W][B]
  void* part;                      // [term_groups][B] partial sums
};
// Bit-sliced term sums.  For each group of 64 replicas term_masks stores,
// per variable v, the 64-bit mask whose bit r is x_{64g + r, v}.  A
// monomial's mask over the group is the AND of its variables' masks, and
// lane r adds w_S when bit r is set; the monomials of a group are added in
// list order.
__host__ __device__ inline size_t term_mask_offset(int n_mono, long long B) {  // bytes into the workspace
  return ((size_t)term_groups(n_mono) * (size_t)B * 8 + 255) & ~(size_t)255;
}
__host__ __device__ inline size_t term_mask_bytes(int n_vars, long long B) {
  return (size_t)((B + 63) / 64) * 64 * (size_t)((n_vars + 63) / 64) * 8;
}

// work-group of 256 threads: 4 waves, one 64-replica group each
__device__ inline void term_masks(const TermJob& J, int rowblock) {
  const int lane = threadIdx.x & 63;
  const long long g = (long long)rowblock * 4 + (threadIdx.x >> 6);
  if (g * 64 >= J.B) return;
  const long long b = g * 64 + lane;
  unsigned long long* masks =
      reinterpret_cast<unsigned long long*>(static_cast<char*>(J.part) + term_mask_offset(J.n_mono, J.B)) +
      g * 64 * J.W;
  for (int w = 0; w < J.W; ++w) {
    const unsigned long long x = b < J.B ? gld(J.bits + (long long)w * J.B + b) : 0ull;
    unsigned long long mine = 0;
    for (int jb = 0; jb < 64; ++jb) {
      const unsigned long long m = __builtin_amdgcn_ballot_w64(((x >> jb) & 1ull) != 0);
      if (lane == jb) mine = m;
    }
    masks[64 * w + lane] = mine;
  }
}

// One 64-replica group per wave; the group's variable masks are copied to LDS.
// Lanes form 64 monomials' masks at once (lane q: monomial m + q, the AND of
// its seven index slots' masks, repeats included), then the wave walks those
// 64 monomials in list order: the monomial's mask, read from its lane, is the
// exec mask of one FP64 (int64) add of its weight, so lane r adds w_S exactly
// when bit r is set, in the same order as a per-lane loop over the list.
template <bool INT>
__device__ inline void term_walk(const TermJob& J, const unsigned long long* sm, int m0, int m1, void* acc_out) {
  const int lane = threadIdx.x & 63;
  typedef const __attribute__((address_space(4))) u4* ConstU4;
  const ConstU4 srec = (ConstU4)J.rec;
  const u4* vrec = reinterpret_cast<const u4*>(J.rec);
  double sf = 0.0;
  long long si = 0;
  // the add runs with exec = (the wave's exec) & mk and restores the saved
  // exec in the same asm statement (the walk is in wave-uniform control flow)
  auto add = [&](unsigned long long mk, const u4& r) {
    const unsigned long long wb = ((unsigned long long)r[3] << 32) | r[2];
    unsigned long long save;
    if (INT)
      asm volatile("s_and_saveexec_b64 %0, %2\n\tv_lshl_add_u64 %1, %1, 0, %3\n\ts_mov_b64 exec, %0"
                   : "=&s"(save), "+v"(si) : "s"(mk), "s"(wb));
    else
      asm volatile("s_and_saveexec_b64 %0, %2\n\tv_add_f64 %1, %3, %1\n\ts_mov_b64 exec, %0"
                   : "=&s"(save), "+v"(sf) : "s"(mk), "s"(__longlong_as_double((long long)wb)));
  };
  for (int m = m0; m < m1; m += 64) {
    const int cnt = m1 - m < 64 ? m1 - m : 64;
    unsigned long long mk = 0;
    if (lane < cnt) {
      const u4 r = vrec[m + lane];
      mk = sm[r[0] & 0xFFu] & sm[(r[0] >> 8) & 0xFFu] & sm[(r[0] >> 16) & 0xFFu] & sm[r[0] >> 24] &
           sm[r[1] & 0xFFu] & sm[(r[1] >> 8) & 0xFFu] & sm[(r[1] >> 16) & 0xFFu];
    }
    const unsigned lo = (unsigned)mk, hi = (unsigned)(mk >> 32);
    auto mask_at = [&](int q) {
      return ((unsigned long long)(unsigned)__builtin_amdgcn_readlane((int)hi, q) << 32) |
             (unsigned)__builtin_amdgcn_readlane((int)lo, q);
    };
    if (cnt == 64) {  // the next four weights load while the current four are added
      u4 n0 = srec[m], n1 = srec[m + 1], n2 = srec[m + 2], n3 = srec[m + 3];
#pragma unroll
      for (int q = 0; q < 64; q += 4) {
        u4 ra = n0, rb = n1, rc = n2, rd = n3;
        asm volatile("" : "+s"(ra), "+s"(rb), "+s"(rc), "+s"(rd));
        if (q + 4 < 64) { n0 = srec[m + q + 4]; n1 = srec[m + q + 5]; n2 = srec[m + q + 6]; n3 = srec[m + q + 7]; }
        add(mask_at(q), ra);
        add(mask_at(q + 1), rb);
        add(mask_at(q + 2), rc);
        add(mask_at(q + 3), rd);
      }
    } else {
      for (int q = 0; q < cnt; ++q) {
        const u4 r = srec[m + q];
        add(mask_at(q), r);
      }
    }
  }
  if (INT)
    *static_cast<long long*>(acc_out) = si;
  else
    *static_cast<double*>(acc_out) = sf;
}

__device__ inline void term_partial(const TermJob& J, int rowblock, int grp) {
  __shared__ unsigned long long sm_masks[4][kMaxVars];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const long long g = (long long)rowblock * 4 + wv;
  if (g * 64 >= J.B) return;
  const long long b = g * 64 + lane;
  const int m0 = grp * kTermGroup;
  const int m1 = m0 + kTermGroup < J.n_mono ? m0 + kTermGroup : J.n_mono;
  const unsigned long long* masks =
      reinterpret_cast<const unsigned long long*>(static_cast<const char*>(J.part) + term_mask_offset(J.n_mono, J.B)) +
      g * 64 * J.W;
  unsigned long long* sm = sm_masks[wv];
  for (int w = 0; w < J.W; ++w) sm[64 * w + lane] = masks[64 * w + lane];
  // the wave's own LDS copy: its writes land before its reads
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (J.integer) {
    long long si;
    term_walk<true>(J, sm, m0, m1, &si);
    if (b < J.B) reinterpret_cast<long long*>(J.part)[(long long)grp * J.B + b] = si;
  } else {
    double sf;
    term_walk<false>(J, sm, m0, m1, &sf);
    if (b < J.B) reinterpret_cast<double*>(J.part)[(long long)grp * J.B + b] = sf;
  }
}


// Arguments of the annealing kernels.  Sweep indices are global within the
// temperature schedule (Philox counters use them); beta and trace rows are
// relative to the call's first sweep; a launch runs sweeps [s_begin, s_end).
struct AnnealParams {
  const AnnealInstDev* insts;
  const AnnealItem* items;
  int n_items;
  int sweeps;                 // sweeps of the call (rows of beta and of the trace)
  int s_first;                // global index of the call's first sweep (row 0)
  int s_begin, s_end;         // global sweeps of this launch
  int cont;                   // 1: best state / energy continue from best_x / best_track
  int mask_s0;                // sweep of attempt-mask row 0
  int mask_rows;              // attempt-mask rows per 16-replica tile
  const double* beta;         // [S] inverse temperatures
  unsigned long long seed;
  const unsigned char* ones;  // a device byte equal to 1 (attempt flag without masks)
  int unif_sweeps;            // blocked kernel: sweep stride of the uniform buffers
};

inline int hip_fail(hipError_t e, std::string* err, const char* what) {
  if (e == hipSuccess) return HOBO_OK;
  *err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? HOBO_ERR_OOM : HOBO_ERR_HIP;
}


// Launch timing (see timing.hip): brackets one kernel launch with two HIP
// events on its stream when timing is enabled and the stream is not capturing.
struct TimedLaunch {
  bool on;
  int kernel;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  TimedLaunch(int k, hipStream_t s);
  ~TimedLaunch();
};

}  // namespace hobo
