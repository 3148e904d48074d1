// gfx950 (CDNA4) kernels of the HOBO engine.
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
#include <string>

#include "hobo_internal.h"
#include "../../include/hobo.h"

namespace hobo {

typedef __bf16 bf16x8 __attribute__((__vector_size__(8 * sizeof(__bf16))));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef int i4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int kLcm = 420;  // lcm(1..7): scales the per-order energy sums to integers

// ------------------------------------------------------------ precision traits
template <int P> struct PT;
template <> struct PT<P_FP32> { static constexpr int RPC = 4, NP = 1, NLD = 2; };
template <> struct PT<P_BF16X2> { static constexpr int RPC = 4, NP = 2, NLD = 2; };
template <> struct PT<P_BF16X3> { static constexpr int RPC = 4, NP = 3, NLD = 3; };
template <> struct PT<P_INT8X4> { static constexpr int RPC = 8, NP = 4, NLD = 4; };

// per-tile B registers: NLD x 16 bytes per lane
template <int P> struct BTile { u4 v[PT<P>::NLD]; };

// accumulator of one 16x16 output tile
template <int P> struct AccT { f4 v; };
template <> struct AccT<P_INT8X4> { i4 v[4]; };

// A operand of one 16-row tile for one chunk
template <int P> struct AOp { u4 v; };  // bf16x8 / 16 int8 / (FP32: low byte = run mask)

// ------------------------------------------------------------ LDS tables
struct Luts {
  u4 bf16[256];         // byte -> eight BF16 values 0 / 1.0
  unsigned long long i8[256];  // byte -> eight INT8 values 0 / 1
};

__device__ inline void build_luts(Luts* L) {
  for (int m = threadIdx.x; m < 256; m += blockDim.x) {
    u4 v;
    for (int d = 0; d < 4; ++d) {
      unsigned lo = (m >> (2 * d)) & 1u, hi = (m >> (2 * d + 1)) & 1u;
      v[d] = (lo ? 0x3F80u : 0u) | (hi ? 0x3F800000u : 0u);
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
    b.v[0] = p[0];
    b.v[1] = p[1];
  } else {
    for (int q = 0; q < PT<P>::NLD; ++q) b.v[q] = *reinterpret_cast<const u4*>(tile + q * 1024 + lane * 16);
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

// value r (0..3) of an accumulator as double (exact for INT8 limbs up to 2^53)
template <int P> __device__ inline double acc_f(const AccT<P>& c, int r) {
  if constexpr (P == P_INT8X4) {
    long long v = (long long)c.v[0][r] + ((long long)c.v[1][r] << 8) + ((long long)c.v[2][r] << 16) +
                  ((long long)c.v[3][r] << 24);
    return (double)v;
  } else {
    return (double)c.v[r];
  }
}
template <int P> __device__ inline long long acc_i(const AccT<P>& c, int r) {
  if constexpr (P == P_INT8X4) {
    return (long long)c.v[0][r] + ((long long)c.v[1][r] << 8) + ((long long)c.v[2][r] << 16) +
           ((long long)c.v[3][r] << 24);
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
    dst[e] = (w < W && r < B) ? bits[(long long)w * B + r] : 0ull;
  }
}

// ============================================================ eval kernel
struct EvalParams {
  const unsigned char* tiles;
  const ChunkMeta* chunks;
  const unsigned long long* runs;
  int nchunks;
  int n_vars;
  int W;
  int ncg;          // column groups
  long long B;
  const unsigned long long* bits;
  void* de_out;     // [B][N] float or int64 (fields)
  void* e_out;      // [B] double or int64
  void* work;       // [ncg][B] partial energies (double or int64), scaled by kLcm in fields mode
  int integer;
  int want_e;
};

template <int P, int RT, int CT, int MODE, int NW>
__global__ __launch_bounds__(64 * NW) void eval_kernel(EvalParams p) {
  constexpr int RPC = PT<P>::RPC;
  __shared__ Luts L;
  __shared__ unsigned long long sbits[NW][RT * 16 * 4];
  build_luts(&L);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, j = lane & 15;
  const long long r0 = ((long long)blockIdx.x * NW + wave) * (RT * 16);
  const int cg = blockIdx.y;
  const int tbase = cg * CT;
  load_bits(sbits[wave], p.bits, p.W, p.B, r0, RT * 16, lane);
  __syncthreads();
  if (r0 >= p.B) return;
  const unsigned char* myb = reinterpret_cast<const unsigned char*>(sbits[wave]);
  const int tb = (P == P_FP32) ? 2048 : (P == P_BF16X2 ? 2048 : (P == P_BF16X3 ? 3072 : 4096));

  AccT<P> acc[RT][CT];
  for (int rt = 0; rt < RT; ++rt)
    for (int t = 0; t < CT; ++t) acc_zero<P>(acc[rt][t]);
  // fields mode: per-order energy bookkeeping (Euler: sum_i x_i g_i^(r) = r E^(r))
  double eacc[RT][4], prevd[RT][4];
  long long eacci[RT][4], previ[RT][4];
  for (int rt = 0; rt < RT; ++rt)
    for (int r = 0; r < 4; ++r) { eacc[rt][r] = 0.0; prevd[rt][r] = 0.0; eacci[rt][r] = 0; previ[rt][r] = 0; }

  BTile<P> bA[CT], bB[CT];
  auto fetch = [&](BTile<P>* b, int c) {
    if (c >= p.nchunks) return;
    ChunkMeta m = p.chunks[c];
    for (int t = 0; t < CT; ++t) {
      int tt = tbase + t;
      if (tt >= m.t_lo && tt < m.t_hi)
        load_tile<P>(b[t], p.tiles + (size_t)(m.tile_off + (tt - m.t_lo)) * tb, lane);
    }
  };
  auto compute = [&](const BTile<P>* b, int c) {
    ChunkMeta m = p.chunks[c];
    int lo = m.t_lo > tbase ? m.t_lo : tbase;
    int hi = m.t_hi < tbase + CT ? m.t_hi : tbase + CT;
    if (hi > lo) {
      AOp<P> a[RT];
      for (int rt = 0; rt < RT; ++rt) a[rt] = gen_a<P>(p.runs, c * RPC, g, myb + (rt * 16 + j) * 32, &L);
      for (int t = 0; t < CT; ++t) {
        int tt = tbase + t;
        if (tt >= lo && tt < hi)
          for (int rt = 0; rt < RT; ++rt) mma<P>(acc[rt][t], a[rt], b[t]);
      }
    }
    if (MODE == M_FIELDS && p.want_e && m.seg_end) {
      const int ord = m.seg_end;
      for (int rt = 0; rt < RT; ++rt)
        for (int r = 0; r < 4; ++r) {
          const unsigned char* rb = myb + (rt * 16 + 4 * g + r) * 32;
          if (p.integer) {
            long long d = 0;
            for (int t = 0; t < CT; ++t) {
              int col = 16 * (tbase + t) + j;
              if (col < p.n_vars && bit_at(rb, col)) d += acc_i<P>(acc[rt][t], r);
            }
            eacci[rt][r] += (long long)(kLcm / ord) * (d - previ[rt][r]);
            previ[rt][r] = d;
          } else {
            double d = 0.0;
            for (int t = 0; t < CT; ++t) {
              int col = 16 * (tbase + t) + j;
              if (col < p.n_vars && bit_at(rb, col)) d += acc_f<P>(acc[rt][t], r);
            }
            eacc[rt][r] += (double)(kLcm / ord) * (d - prevd[rt][r]);
            prevd[rt][r] = d;
          }
        }
    }
  };
  fetch(bA, 0);
  for (int c = 0; c < p.nchunks; c += 2) {
    fetch(bB, c + 1);
    compute(bA, c);
    if (c + 1 < p.nchunks) {
      fetch(bA, c + 2);
      compute(bB, c + 1);
    }
  }

  // ------------------------------------------------------------ epilogue
  for (int rt = 0; rt < RT; ++rt) {
    for (int r = 0; r < 4; ++r) {
      const long long row = r0 + rt * 16 + 4 * g + r;
      const unsigned char* rb = myb + (rt * 16 + 4 * g + r) * 32;
      if (MODE == M_FIELDS && p.de_out) {
        for (int t = 0; t < CT; ++t) {
          int col = 16 * (tbase + t) + j;
          if (row < p.B && col < p.n_vars) {
            int x = bit_at(rb, col);
            if (p.integer) {
              long long gv = acc_i<P>(acc[rt][t], r);
              reinterpret_cast<long long*>(p.de_out)[row * p.n_vars + col] = x ? -gv : gv;
            } else {
              float gv = (float)acc_f<P>(acc[rt][t], r);
              reinterpret_cast<float*>(p.de_out)[row * p.n_vars + col] = x ? -gv : gv;
            }
          }
        }
      }
      if (p.want_e) {
        // per-row energy partial of this column group
        if (p.integer) {
          long long v;
          if (MODE == M_FIELDS) {
            v = eacci[rt][r];
          } else {
            v = 0;
            for (int t = 0; t < CT; ++t) {
              int col = 16 * (tbase + t) + j;
              if (col < p.n_vars && bit_at(rb, col)) v += acc_i<P>(acc[rt][t], r);
            }
          }
          v = group_sum_i(v);
          if (j == 0 && row < p.B) {
            if (p.ncg == 1)
              reinterpret_cast<long long*>(p.e_out)[row] = MODE == M_FIELDS ? v / kLcm : v;
            else
              reinterpret_cast<long long*>(p.work)[(long long)cg * p.B + row] = v;
          }
        } else {
          double v;
          if (MODE == M_FIELDS) {
            v = eacc[rt][r];
          } else {
            v = 0.0;
            for (int t = 0; t < CT; ++t) {
              int col = 16 * (tbase + t) + j;
              if (col < p.n_vars && bit_at(rb, col)) v += acc_f<P>(acc[rt][t], r);
            }
          }
          v = group_sum(v);
          if (j == 0 && row < p.B) {
            if (p.ncg == 1)
              reinterpret_cast<double*>(p.e_out)[row] = MODE == M_FIELDS ? v / (double)kLcm : v;
            else
              reinterpret_cast<double*>(p.work)[(long long)cg * p.B + row] = v;
          }
        }
      }
    }
  }
}

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
// One thread per replica; the monomial list is read uniformly (scalar loads).
// Sums in FP64 (real tensors) or int64 (integer tensors) in monomial order.
__global__ __launch_bounds__(256) void term_energy_kernel(const TermRec* rec, int n_mono, int W,
                                                          long long B, const unsigned long long* bits,
                                                          void* e_out, int integer) {
  long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long x0 = 0, x1 = 0, x2 = 0, x3 = 0;
  if (b < B) {
    x0 = bits[b];
    if (W > 1) x1 = bits[B + b];
    if (W > 2) x2 = bits[2 * B + b];
    if (W > 3) x3 = bits[3 * B + b];
  }
  double sf = 0.0;
  long long si = 0;
  for (int m = 0; m < n_mono; ++m) {
    TermRec r = rec[m];
    bool on = true;
    for (int q = 0; q < r.len; ++q) {
      unsigned v = r.idx[q];
      unsigned long long w = v < 64 ? x0 : (v < 128 ? x1 : (v < 192 ? x2 : x3));
      on = on && ((w >> (v & 63u)) & 1ull);
    }
    if (on) {
      if (integer)
        si += r.w.i;
      else
        sf += r.w.f;
    }
  }
  if (b < B) {
    if (integer)
      reinterpret_cast<long long*>(e_out)[b] = si;
    else
      reinterpret_cast<double*>(e_out)[b] = sf;
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

// Random initial states: bit i of replica b = top bit of word i%4 of
// Philox(counter (b, 0, i/4, 1), key (seed, inst)).
__global__ void init_random_kernel(unsigned long long* x, int n_vars, int W, long long B,
                                   unsigned long long seed, unsigned long long inst) {
  long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)W * B) return;
  int w = (int)(idx / B);
  long long b = idx - (long long)w * B;
  unsigned long long v = 0;
  for (int q = 0; q < 16; ++q) {
    int i0 = 64 * w + 4 * q;
    if (i0 >= n_vars) break;
    U64x4 o = philox((unsigned long long)b, 0ull, (unsigned long long)(i0 >> 2), 1ull, seed, inst);
    for (int e = 0; e < 4; ++e)
      if (i0 + e < n_vars) v |= (o.w[e] >> 63) << ((i0 + e) & 63);
  }
  x[idx] = v;
}

// ============================================================ annealer
struct AnnealParams {
  const AnnealInstDev* insts;
  const AnnealItem* items;
  int n_items;
  int sweeps;
  const double* beta;
  unsigned long long seed;
};

template <int P, int CT, int NW>
__global__ __launch_bounds__(64 * NW) void anneal_kernel(AnnealParams p) {
  constexpr int RPC = PT<P>::RPC;
  __shared__ Luts L;
  __shared__ unsigned long long sbits[NW][64];
  __shared__ unsigned long long sbest[NW][64];
  build_luts(&L);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, j = lane & 15;
  const bool owner = j < 4;
  const int orow = 4 * g + j;  // replica row owned by this lane (if owner)
  unsigned char* myb = reinterpret_cast<unsigned char*>(sbits[wave]);
  const int tb = (P == P_FP32) ? 2048 : (P == P_BF16X2 ? 2048 : (P == P_BF16X3 ? 3072 : 4096));
  const int wave_gid = blockIdx.x * NW + wave;
  const int wave_cnt = gridDim.x * NW;

  for (int it = wave_gid; it < p.n_items; it += wave_cnt) {
    const AnnealItem item = p.items[it];
    const AnnealInstDev I = p.insts[item.inst];
    const long long r0 = (long long)item.tile16 * 16;
    const int N = I.n_vars;
    load_bits(sbits[wave], I.x, I.W, I.B, r0, 16, lane);
    load_bits(sbest[wave], I.x, I.W, I.B, r0, 16, lane);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    const long long myrow = r0 + orow;
    double E = 0.0, bestE = 0.0;
    if (owner && myrow < I.B) E = I.e_track[myrow];
    bestE = E;
    unsigned long long rw[4] = {0, 0, 0, 0};  // Philox words held by this lane

    for (int s = 0; s < p.sweeps; ++s) {
      const double beta = p.beta[s];
      const unsigned char* att = I.attempt ? I.attempt + ((size_t)item.tile16 * p.sweeps + s) * N : nullptr;
      auto next_bit = [&](int from) {
        int b = from;
        if (att)
          while (b < N && !att[b]) ++b;
        return b;
      };
      // flattened stream of (bit, chunk) pairs of this sweep, one chunk prefetched ahead
      int ci = next_bit(0), cc = 0;  // current
      SlabMeta sm{};
      if (ci < N) sm = I.slabs[ci];
      AccT<P> acc[CT];
      for (int t = 0; t < CT; ++t) acc_zero<P>(acc[t]);
      BTile<P> bA[CT], bB[CT];
      auto fetch = [&](BTile<P>* b, int bit, int c) {
        if (bit >= N) return;
        const SlabMeta m2 = I.slabs[bit];
        const ChunkMeta m = I.chunks[m2.chunk0 + c];
        for (int t = 0; t < CT; ++t)
          if (t >= m.t_lo && t < m.t_hi) load_tile<P>(b[t], I.tiles + (size_t)(m.tile_off + (t - m.t_lo)) * tb, lane);
      };
      // philox block for bits i .. i+15 (refreshed when i crosses a multiple of 16)
      int rw_block = -1;
      auto step = [&](const BTile<P>* cur, BTile<P>* nxt) {
        // successor of (ci, cc)
        int ni = ci, nc = cc + 1;
        if (nc >= (int)sm.nchunks) {
          ni = next_bit(ci + 1);
          nc = 0;
        }
        fetch(nxt, ni, nc);
        {
          const ChunkMeta m = I.chunks[sm.chunk0 + cc];
          if (m.t_hi > m.t_lo) {
            AOp<P> a = gen_a<P>(I.runs, (int)(sm.run0 + cc * RPC), g, myb + j * 32, &L);
            for (int t = 0; t < CT; ++t)
              if (t >= m.t_lo && t < m.t_hi) mma<P>(acc[t], a, cur[t]);
          }
        }
        if (cc + 1 >= (int)sm.nchunks) {
          // ---- epilogue of bit ci: g_i = w_i + sum_c x_c G_c, then Metropolis
          const int i = ci;
          if ((i >> 4) != rw_block) {
            rw_block = i >> 4;
            // lane (g, j) draws the block of replica 4g + (j & 3) for bits 16*blk + 4*(j>>2) .. +3
            const long long rr = r0 + 4 * g + (j & 3);
            U64x4 o = philox((unsigned long long)rr, (unsigned long long)s,
                             (unsigned long long)(4 * rw_block + (j >> 2)), 0ull, p.seed, I.inst_id);
            rw[0] = o.w[0]; rw[1] = o.w[1]; rw[2] = o.w[2]; rw[3] = o.w[3];
          }
          double hs[4];
          long long hi4[4];
          for (int r = 0; r < 4; ++r) {
            const unsigned char* rb = myb + (4 * g + r) * 32;
            if (I.integer) {
              long long v = 0;
              for (int t = 0; t < CT; ++t) {
                int col = 16 * t + j;
                if (col < N && bit_at(rb, col)) v += acc_i<P>(acc[t], r);
              }
              hi4[r] = group_sum_i(v);
              hs[r] = 0.0;
            } else {
              double v = 0.0;
              for (int t = 0; t < CT; ++t) {
                int col = 16 * t + j;
                if (col < N && bit_at(rb, col)) v += acc_f<P>(acc[t], r);
              }
              hs[r] = group_sum(v);
              hi4[r] = 0;
            }
          }
          // random word for (row, s, i): held by lane (g, 4*((i>>2)&3) + (j&3))
          const int src = 16 * g + 4 * ((i >> 2) & 3) + (j & 3);
          const unsigned long long word = rw[i & 3];
          const unsigned lo32 = __shfl((unsigned)word, src, 64);
          const unsigned hi32 = __shfl((unsigned)(word >> 32), src, 64);
          if (owner && myrow < I.B) {
            double gval;
            if (I.integer) {
              long long h = j == 0 ? hi4[0] : (j == 1 ? hi4[1] : (j == 2 ? hi4[2] : hi4[3]));
              gval = (double)(sm.a_i + h);
            } else {
              double h = j == 0 ? hs[0] : (j == 1 ? hs[1] : (j == 2 ? hs[2] : hs[3]));
              gval = sm.a_f + h;
            }
            unsigned char* rb = myb + orow * 32;
            const int xi = bit_at(rb, i);
            const double dE = xi ? -gval : gval;
            const unsigned long long r64 = ((unsigned long long)hi32 << 32) | lo32;
            const double u = (double)(r64 >> 11) * 0x1.0p-53;
            bool take = dE <= 0.0;
            if (!take) take = u < exp(-dE * beta);
            if (take) {
              rb[i >> 3] ^= (unsigned char)(1u << (i & 7));
              E += dE;
            }
          }
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
          __builtin_amdgcn_wave_barrier();
          for (int t = 0; t < CT; ++t) acc_zero<P>(acc[t]);
        }
        ci = ni;
        cc = nc;
        if (ci < N && cc == 0) sm = I.slabs[ci];
      };
      fetch(bA, ci, 0);
      while (ci < N) {
        step(bA, bB);
        if (ci >= N) break;
        step(bB, bA);
      }
      // best tracking after the sweep
      if (owner && myrow < I.B && E < bestE) {
        bestE = E;
        for (int w = 0; w < 4; ++w) sbest[wave][orow * 4 + w] = sbits[wave][orow * 4 + w];
      }
      if (I.trace_part) {
        double v = (owner && myrow < I.B) ? bestE : INFINITY;
        for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
        if (lane == 0) I.trace_part[(size_t)item.tile16 * p.sweeps + s] = v;
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      __builtin_amdgcn_wave_barrier();
    }
    // write back
    {
      const int rho = lane >> 2, w = lane & 3;
      const long long r = r0 + rho;
      if (w < I.W && r < I.B) {
        I.x[(long long)w * I.B + r] = sbits[wave][lane];
        I.best_x[(long long)w * I.B + r] = sbest[wave][lane];
      }
    }
    if (owner && myrow < I.B) {
      I.e_track[myrow] = E;
      I.best_track[myrow] = bestE;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
  }
}

__global__ void trace_reduce_kernel(const double* part, double* out, int ntiles, int S) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  double v = INFINITY;
  for (int t = 0; t < ntiles; ++t) v = fmin(v, part[(size_t)t * S + s]);
  out[s] = v;
}

// ============================================================ launchers
static int hip_fail(hipError_t e, std::string* err, const char* what) {
  if (e == hipSuccess) return HOBO_OK;
  *err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? HOBO_ERR_OOM : HOBO_ERR_HIP;
}

size_t eval_workspace_bytes(const Tensor* t, int mode, int64_t B, int ct) {
  (void)mode;
  int T = (t->n_vars + 15) / 16;
  int ncg = (T + ct - 1) / ct;
  return ncg > 1 ? (size_t)ncg * (size_t)B * 8 : 0;
}

template <int P, int RT, int CT, int MODE>
static void launch_eval_t(const EvalParams& ep, int nblk_x, hipStream_t st) {
  constexpr int NW = 4;
  dim3 grid((unsigned)nblk_x, (unsigned)ep.ncg);
  hipLaunchKernelGGL((eval_kernel<P, RT, CT, MODE, NW>), grid, dim3(64 * NW), 0, st, ep);
}

template <int P, int MODE>
static int dispatch_eval_shape(const EvalParams& ep, int rt, int ct, long long B, hipStream_t st) {
  const long long rows_per_block = 4LL * rt * 16;
  int nblk = (int)((B + rows_per_block - 1) / rows_per_block);
#define HOBO_EV(RTV, CTV)                                                   \
  if (rt == RTV && ct == CTV) {                                             \
    launch_eval_t<P, RTV, CTV, MODE>(ep, nblk, st);                         \
    return 0;                                                               \
  }
  HOBO_EV(1, 1) HOBO_EV(1, 2) HOBO_EV(1, 4) HOBO_EV(1, 8)
  HOBO_EV(2, 1) HOBO_EV(2, 2) HOBO_EV(2, 4) HOBO_EV(2, 8)
#undef HOBO_EV
  return -1;
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
  ep.B = a.B;
  ep.bits = reinterpret_cast<const unsigned long long*>(a.bits);
  ep.de_out = a.de_out;
  ep.e_out = a.e_out;
  ep.work = a.work;
  ep.integer = t->integer ? 1 : 0;
  ep.want_e = a.e_out != nullptr;
  int r = -1;
  switch (pk->prec * 4 + pk->mode) {
    case P_FP32 * 4 + M_FIELDS: r = dispatch_eval_shape<P_FP32, M_FIELDS>(ep, rt, ct, a.B, st); break;
    case P_FP32 * 4 + M_ENERGY: r = dispatch_eval_shape<P_FP32, M_ENERGY>(ep, rt, ct, a.B, st); break;
    case P_BF16X2 * 4 + M_FIELDS: r = dispatch_eval_shape<P_BF16X2, M_FIELDS>(ep, rt, ct, a.B, st); break;
    case P_BF16X2 * 4 + M_ENERGY: r = dispatch_eval_shape<P_BF16X2, M_ENERGY>(ep, rt, ct, a.B, st); break;
    case P_BF16X3 * 4 + M_FIELDS: r = dispatch_eval_shape<P_BF16X3, M_FIELDS>(ep, rt, ct, a.B, st); break;
    case P_BF16X3 * 4 + M_ENERGY: r = dispatch_eval_shape<P_BF16X3, M_ENERGY>(ep, rt, ct, a.B, st); break;
    case P_INT8X4 * 4 + M_FIELDS: r = dispatch_eval_shape<P_INT8X4, M_FIELDS>(ep, rt, ct, a.B, st); break;
    case P_INT8X4 * 4 + M_ENERGY: r = dispatch_eval_shape<P_INT8X4, M_ENERGY>(ep, rt, ct, a.B, st); break;
    default: break;
  }
  if (r != 0) {
    *err = "no kernel for this precision / tile shape";
    return HOBO_ERR_UNSUPPORTED;
  }
  int s = hip_fail(hipGetLastError(), err, "eval kernel launch");
  if (s) return s;
  if (ncg > 1 && a.e_out) {
    int scale = pk->mode == M_FIELDS ? kLcm : 1;
    hipLaunchKernelGGL(reduce_partials, dim3((unsigned)((a.B + 255) / 256)), dim3(256), 0, st, a.work, a.e_out,
                       ncg, (long long)a.B, ep.integer, scale);
    s = hip_fail(hipGetLastError(), err, "reduce kernel launch");
  }
  return s;
}

int launch_term_energy(const TermArgs& a, std::string* err) {
  hipStream_t st = (hipStream_t)a.stream;
  int W = (a.t->n_vars + 63) / 64;
  hipLaunchKernelGGL(term_energy_kernel, dim3((unsigned)((a.B + 255) / 256)), dim3(256), 0, st, a.td->d_rec,
                     a.td->n_mono, W, (long long)a.B, reinterpret_cast<const unsigned long long*>(a.bits), a.e_out,
                     a.t->integer ? 1 : 0);
  return hip_fail(hipGetLastError(), err, "term energy launch");
}

}  // namespace hobo

namespace hobo {

// ------------------------------------------------------------ multi-instance helpers
// grid.y = instance; x covers replicas (and words for init)
__global__ void init_random_multi(const InstSmall* in, unsigned long long seed) {
  const InstSmall I = in[blockIdx.y];
  long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)I.W * I.B) return;
  int w = (int)(idx / I.B);
  long long b = idx - (long long)w * I.B;
  unsigned long long v = 0;
  for (int q = 0; q < 16; ++q) {
    int i0 = 64 * w + 4 * q;
    if (i0 >= I.n_vars) break;
    U64x4 o = philox((unsigned long long)b, 0ull, (unsigned long long)(i0 >> 2), 1ull, seed, I.inst_id);
    for (int e = 0; e < 4; ++e)
      if (i0 + e < I.n_vars) v |= (o.w[e] >> 63) << ((i0 + e) & 63);
  }
  I.x[idx] = v;
}

// energies of x (which = 0) or best_x (which = 1) by the term loop: which = 0
// writes the tracked start energy (double), which = 1 the rescored best output
__global__ __launch_bounds__(256) void term_energy_multi(const InstSmall* in, int which) {
  const InstSmall I = in[blockIdx.y];
  long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if ((long long)blockIdx.x * blockDim.x >= I.B) return;
  const unsigned long long* bits = which ? I.best_x : I.x;
  unsigned long long x0 = 0, x1 = 0, x2 = 0, x3 = 0;
  if (b < I.B) {
    x0 = bits[b];
    if (I.W > 1) x1 = bits[I.B + b];
    if (I.W > 2) x2 = bits[2 * I.B + b];
    if (I.W > 3) x3 = bits[3 * I.B + b];
  }
  double sf = 0.0;
  long long si = 0;
  for (int m = 0; m < I.n_mono; ++m) {
    TermRec r = I.rec[m];
    bool on = true;
    for (int q = 0; q < r.len; ++q) {
      unsigned v = r.idx[q];
      unsigned long long w = v < 64 ? x0 : (v < 128 ? x1 : (v < 192 ? x2 : x3));
      on = on && ((w >> (v & 63u)) & 1ull);
    }
    if (on) {
      if (I.integer) si += r.w.i; else sf += r.w.f;
    }
  }
  if (b < I.B) {
    if (which == 0) {
      I.e_track[b] = I.integer ? (double)si : sf;
    } else if (I.best_out) {
      if (I.integer)
        reinterpret_cast<long long*>(I.best_out)[b] = si;
      else
        reinterpret_cast<double*>(I.best_out)[b] = sf;
    }
  }
}

__global__ void trace_reduce_multi(const InstSmall* in, int S) {
  const InstSmall I = in[blockIdx.y];
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S || !I.trace_out) return;
  double v = INFINITY;
  for (int t = 0; t < I.ntiles16; ++t) v = fmin(v, I.trace_part[(size_t)t * S + s]);
  I.trace_out[s] = v;
}

template <int P, int CT, int NW>
static void launch_anneal_t(const AnnealParams& ap, int nblk, hipStream_t st) {
  hipLaunchKernelGGL((anneal_kernel<P, CT, NW>), dim3((unsigned)nblk), dim3(64 * NW), 0, st, ap);
}

template <int P>
static int dispatch_anneal(const AnnealParams& ap, int ct, int nw, int nblk, hipStream_t st) {
#define HOBO_AN(CTV, NWV)                         \
  if (ct == CTV && nw == NWV) {                   \
    launch_anneal_t<P, CTV, NWV>(ap, nblk, st);   \
    return 0;                                     \
  }
  if constexpr (P == P_INT8X4) {
    HOBO_AN(1, 1) HOBO_AN(1, 2) HOBO_AN(1, 4)
    HOBO_AN(2, 1) HOBO_AN(2, 2) HOBO_AN(2, 4)
    HOBO_AN(4, 1) HOBO_AN(4, 2) HOBO_AN(4, 4)
  } else {
    HOBO_AN(1, 1) HOBO_AN(1, 2) HOBO_AN(1, 4)
    HOBO_AN(2, 1) HOBO_AN(2, 2) HOBO_AN(2, 4)
    HOBO_AN(4, 1) HOBO_AN(4, 2) HOBO_AN(4, 4)
    HOBO_AN(8, 1) HOBO_AN(8, 2) HOBO_AN(8, 4)
    HOBO_AN(16, 1) HOBO_AN(16, 2) HOBO_AN(16, 4)
  }
#undef HOBO_AN
  return -1;
}

int anneal_ct_for(int n_vars) {
  int T = (n_vars + 15) / 16;
  int ct = 1;
  while (ct < T) ct *= 2;
  return ct;
}

// Enqueue the whole anneal sequence for instances [i0, i1) of the tables.
int enqueue_anneal_seq(const AnnealTables& tb, int n_inst, int sweeps, uint64_t seed, int init_random,
                       int prec, int ct, int nw, int item0, int nitems, int inst0, int ninst,
                       void* stream, std::string* err) {
  (void)n_inst;
  hipStream_t st = (hipStream_t)stream;
  const InstSmall* sm = tb.d_small + inst0;
  if (init_random) {
    long long wb = (long long)tb.max_W * tb.max_B;
    hipLaunchKernelGGL(init_random_multi, dim3((unsigned)((wb + 255) / 256), (unsigned)ninst), dim3(256), 0, st, sm,
                       (unsigned long long)seed);
  }
  hipLaunchKernelGGL(term_energy_multi, dim3((unsigned)((tb.max_B + 255) / 256), (unsigned)ninst), dim3(256), 0, st,
                     sm, 0);
  AnnealParams ap{};
  ap.insts = tb.d_inst;
  ap.items = tb.d_items + item0;
  ap.n_items = nitems;
  ap.sweeps = sweeps;
  ap.beta = tb.d_beta;
  ap.seed = seed;
  if (nitems > 0) {
    int nblk = (nitems + nw - 1) / nw;
    if (nblk > 4096) nblk = 4096;
    int r = -1;
    switch (prec) {
      case P_FP32: r = dispatch_anneal<P_FP32>(ap, ct, nw, nblk, st); break;
      case P_BF16X2: r = dispatch_anneal<P_BF16X2>(ap, ct, nw, nblk, st); break;
      case P_BF16X3: r = dispatch_anneal<P_BF16X3>(ap, ct, nw, nblk, st); break;
      case P_INT8X4: r = dispatch_anneal<P_INT8X4>(ap, ct, nw, nblk, st); break;
      default: break;
    }
    if (r != 0) {
      *err = "no annealer kernel for this precision / width";
      return HOBO_ERR_UNSUPPORTED;
    }
  }
  hipLaunchKernelGGL(term_energy_multi, dim3((unsigned)((tb.max_B + 255) / 256), (unsigned)ninst), dim3(256), 0, st,
                     sm, 1);
  if (sweeps > 0)
    hipLaunchKernelGGL(trace_reduce_multi, dim3((unsigned)((sweeps + 255) / 256), (unsigned)ninst), dim3(256), 0, st,
                       sm, sweeps);
  return hip_fail(hipGetLastError(), err, "anneal launch");
}

}  // namespace hobo
