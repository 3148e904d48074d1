// The batched energy / local-field contraction kernel (hobo_energy,
// hobo_local_fields), included by one translation unit per precision
// (eval_prec.hip, built once for each precision) so that the many shape
// instantiations compile in parallel.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>
#include <type_traits>

#include "device_common.h"

namespace hobo {

// ============================================================ eval kernel
struct EvalParams {
  const unsigned char* tiles;
  const ChunkMeta* chunks;
  const unsigned long long* runs;
  int nchunks;
  int n_vars;
  int W;
  int ncg;          // column groups
  int n_tiles;      // 16-column tiles
  unsigned n_tile_buf;  // tiles stored in the packed buffer
  long long B;
  const unsigned long long* bits;
  void* de_out;     // [B][N] float or int64 (fields)
  void* e_out;      // [B] double or int64
  void* work;       // [ncg][B] partial energies (double or int64), scaled by kLcm in fields mode
  int integer;
  int want_e;
  double inv_scale;  // 2^-scale_exp of the packed layout (FP16X2)
};

// chunks in flight per wave in the evaluation kernels
template <int P, int CT> constexpr int ring_depth_eval() {
  constexpr int per = CT * PT<P>::NLD * 4 + 4;
  constexpr int d = 160 / per;
  return d < 2 ? 2 : (d > 8 ? 8 : d);
}
constexpr int kEvalMetaBlock = 1024;  // chunk metadata staged in LDS per block

template <int P, int RT, int CT, int MODE, int NW>
__global__ __launch_bounds__(64 * NW) void eval_kernel(EvalParams p) {
  constexpr int RPC = PT<P>::RPC;
  __shared__ Luts L;
  __shared__ unsigned long long sbits[NW][RT * 16 * 4];
  __shared__ ChunkMeta smeta[2][kEvalMetaBlock];
  build_luts<P>(&L);
  const double scl = p.inv_scale;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, j = lane & 15;
  const long long r0 = ((long long)blockIdx.x * NW + wave) * (RT * 16);
  const int cg = blockIdx.y;
  const int tbase = cg * CT;
  load_bits(sbits[wave], p.bits, p.W, p.B, r0, RT * 16, lane);
  {
    // metadata blocks 0 and 1 (the rest are staged as the stream advances)
    const int nb0 = (p.nchunks + kEvalMetaBlock - 1) / kEvalMetaBlock;
    for (int blk = 0; blk < 2 && blk < nb0; ++blk) {
      const int c0 = blk * kEvalMetaBlock;
      const int cnt = p.nchunks - c0 < kEvalMetaBlock ? p.nchunks - c0 : kEvalMetaBlock;
      for (int q = threadIdx.x; q < cnt; q += blockDim.x)
        smeta[blk][q] = __builtin_bit_cast(ChunkMeta, gld(reinterpret_cast<const unsigned long long*>(p.chunks) + c0 + q));
    }
  }
  __syncthreads();
  const unsigned char* myb = reinterpret_cast<const unsigned char*>(sbits[wave]);
  const int tb = (P == P_FP32 || P == P_BF16X2 || P == P_FP16X2) ? 2048 : (P == P_BF16X3 ? 3072 : 4096);

  AccT<P> acc[RT][CT];
  for (int rt = 0; rt < RT; ++rt)
    for (int t = 0; t < CT; ++t) acc_zero<P>(acc[rt][t]);
  // fields mode: per-order energy bookkeeping (Euler: sum_i x_i g_i^(r) = r E^(r))
  // one 64-bit register pair per value: int64 for integer tensors, the bits
  // of a double otherwise
  long long eacc[RT][4], prevv[RT][4];
  for (int rt = 0; rt < RT; ++rt)
    for (int r = 0; r < 4; ++r) { eacc[rt][r] = 0; prevv[rt][r] = 0; }

  // coefficient stream: chunk c's tiles of this column group and run
  // descriptors, D chunks in flight; chunk metadata is fetched one ahead
  constexpr int D = ring_depth_eval<P, CT>();
  struct ESlot {
    BTile<P> b[CT];
    unsigned long long d0, d1;
    int c;
  };
  // chunk metadata comes from LDS (staged kEvalMetaBlock chunks at a time);
  // every chunk issues the same loads into its own ring slot (absent tiles
  // read the zero tile 0), so counted waits keep the later chunks in flight
  const int nblk = (p.nchunks + kEvalMetaBlock - 1) / kEvalMetaBlock;
  auto stage_meta = [&](int blk) {
    const int c0 = blk * kEvalMetaBlock;
    const int cnt = p.nchunks - c0 < kEvalMetaBlock ? p.nchunks - c0 : kEvalMetaBlock;
    for (int q = threadIdx.x; q < cnt; q += blockDim.x)
      smeta[blk & 1][q] = __builtin_bit_cast(ChunkMeta, gld(reinterpret_cast<const unsigned long long*>(p.chunks) + c0 + q));
  };
  auto meta_of = [&](int c) -> ChunkMeta {
    const int blk = c / kEvalMetaBlock;
    return smeta[blk & 1][c - blk * kEvalMetaBlock];
  };
  int pc = 0;
  auto issue = [&](ESlot& sl) {
    const bool valid = pc < p.nchunks;
    const int c = valid ? pc : 0;
    sl.c = valid ? c : -1;
    const ChunkMeta pm = valid ? meta_of(c) : ChunkMeta{};
#pragma unroll
    for (int t = 0; t < CT; ++t) {
      const int tt = tbase + t;
      const bool have = tt >= pm.t_lo && tt < pm.t_hi;
      unsigned idx = have ? pm.tile_off + (unsigned)(tt - pm.t_lo) : 0u;
      idx = idx < p.n_tile_buf ? idx : 0u;  // never outside the tile buffer
      load_tile<P>(sl.b[t], p.tiles + (size_t)idx * tb, lane);
    }
    if constexpr (P == P_INT8X4) {
      sl.d0 = gld(p.runs + c * RPC + 2 * g);
      sl.d1 = gld(p.runs + c * RPC + 2 * g + 1);
    } else {
      sl.d0 = gld(p.runs + c * RPC + g);
    }
    ++pc;
  };
  auto consume = [&](ESlot& sl, auto restage) {
    if (sl.c < 0) return;
    if constexpr (decltype(restage)::value) {
      // entering a metadata block: stage the block after it into the buffer
      // of the block before, once every wave has consumed that block (the
      // first barrier; the producer is fewer than a block ahead, so it does
      // not read it either), and before any producer reaches the staged
      // block (the second)
      if (sl.c % kEvalMetaBlock == 0) {
        const int nb = sl.c / kEvalMetaBlock + 1;
        lds_barrier();
        if (nb < nblk) stage_meta(nb);
        lds_barrier();
      }
    }
    const ChunkMeta m = meta_of(sl.c);
    const int lo = m.t_lo > tbase ? m.t_lo : tbase;
    const int hi = m.t_hi < tbase + CT ? m.t_hi : tbase + CT;
    if (hi > lo) {
      AOp<P> a[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const unsigned char* rb = myb + (rt * 16 + j) * 32;
        if constexpr (P == P_FP32) {
          a[rt].v = u4{run_mask(sl.d0, rb), 0u, 0u, 0u};
        } else if constexpr (P == P_INT8X4) {
          unsigned long long lo8 = L.i8[run_mask(sl.d0, rb)], hi8 = L.i8[run_mask(sl.d1, rb)];
          a[rt].v = u4{(unsigned)lo8, (unsigned)(lo8 >> 32), (unsigned)hi8, (unsigned)(hi8 >> 32)};
        } else {
          a[rt].v = L.bf16[run_mask(sl.d0, rb)];
        }
      }
#pragma unroll
      for (int t = 0; t < CT; ++t) {
        const int tt = tbase + t;
        if (tt >= lo && tt < hi)
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) mma<P>(acc[rt][t], a[rt], sl.b[t]);
      }
    }
    if (MODE == M_FIELDS && p.want_e && m.seg_end) {
      const int ord = m.seg_end;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const unsigned char* rb = myb + (rt * 16 + 4 * g + r) * 32;
          if (p.integer) {
            long long d = 0;
#pragma unroll
            for (int t = 0; t < CT; ++t) {
              int col = 16 * (tbase + t) + j;
              if (col < p.n_vars && bit_at(rb, col)) d += acc_i<P>(acc[rt][t], r, scl);
            }
            eacc[rt][r] += (long long)(kLcm / ord) * (d - prevv[rt][r]);
            prevv[rt][r] = d;
          } else {
            double d = 0.0;
#pragma unroll
            for (int t = 0; t < CT; ++t) {
              int col = 16 * (tbase + t) + j;
              if (col < p.n_vars && bit_at(rb, col)) d += acc_f<P>(acc[rt][t], r, scl);
            }
            const double e = __longlong_as_double(eacc[rt][r]) +
                             (double)(kLcm / ord) * (d - __longlong_as_double(prevv[rt][r]));
            eacc[rt][r] = __double_as_longlong(e);
            prevv[rt][r] = __double_as_longlong(d);
          }
        }
    }
  };
  auto run = [&](auto restage) {
    ESlot ring[D];
#pragma unroll
    for (int d = 0; d < D; ++d) issue(ring[d]);
    while (ring[0].c >= 0) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        consume(ring[d], restage);
        issue(ring[d]);
      }
    }
  };
  if (nblk > 2)
    run(std::integral_constant<bool, true>{});
  else
    run(std::integral_constant<bool, false>{});

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
              long long gv = acc_i<P>(acc[rt][t], r, scl);
              reinterpret_cast<long long*>(p.de_out)[row * p.n_vars + col] = x ? -gv : gv;
            } else {
              float gv = (float)acc_f<P>(acc[rt][t], r, scl);
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
            v = group_sum_i(eacc[rt][r]);
          } else {
            v = 0;
            for (int t = 0; t < CT; ++t) {
              int col = 16 * (tbase + t) + j;
              long long ts = group_sum_i((col < p.n_vars && bit_at(rb, col)) ? acc_i<P>(acc[rt][t], r, scl) : 0);
              v += ts;
              if (p.ncg > 1 && j == 0 && row < p.B && tbase + t < p.n_tiles)
                reinterpret_cast<long long*>(p.work)[(long long)(tbase + t) * p.B + row] = ts;
            }
          }
          if (j == 0 && row < p.B) {
            if (p.ncg == 1)
              reinterpret_cast<long long*>(p.e_out)[row] = MODE == M_FIELDS ? v / kLcm : v;
            else if (MODE == M_FIELDS)
              reinterpret_cast<long long*>(p.work)[(long long)cg * p.B + row] = v;
          }
        } else {
          double v;
          if (MODE == M_FIELDS) {
            v = group_sum(__longlong_as_double(eacc[rt][r]));
          } else {
            // per 16-column tile sums added in column order: the result does
            // not depend on how tiles are grouped into waves
            v = 0.0;
            for (int t = 0; t < CT; ++t) {
              int col = 16 * (tbase + t) + j;
              double ts = group_sum((col < p.n_vars && bit_at(rb, col)) ? acc_f<P>(acc[rt][t], r, scl) : 0.0);
              v += ts;
              if (p.ncg > 1 && j == 0 && row < p.B && tbase + t < p.n_tiles)
                reinterpret_cast<double*>(p.work)[(long long)(tbase + t) * p.B + row] = ts;
            }
          }
          if (j == 0 && row < p.B) {
            if (p.ncg == 1)
              reinterpret_cast<double*>(p.e_out)[row] = MODE == M_FIELDS ? v / (double)kLcm : v;
            else if (MODE == M_FIELDS)
              reinterpret_cast<double*>(p.work)[(long long)cg * p.B + row] = v;
          }
        }
      }
    }
  }
}

template <int P, int RT, int CT, int MODE>
inline void launch_eval_t(const EvalParams& ep, int nblk_x, hipStream_t st) {
  constexpr int NW = 4;
  dim3 grid((unsigned)nblk_x, (unsigned)ep.ncg);
  TimedLaunch tl(MODE == M_FIELDS ? 1 : 2, st);
  hipLaunchKernelGGL((eval_kernel<P, RT, CT, MODE, NW>), grid, dim3(64 * NW), 0, st, ep);
}

template <int P, int MODE>
inline int dispatch_eval_shape(const EvalParams& ep, int rt, int ct, long long B, hipStream_t st) {
  const long long rows_per_block = 4LL * rt * 16;
  int nblk = (int)((B + rows_per_block - 1) / rows_per_block);
#define HOBO_EV(RTV, CTV)                                                   \
  if (rt == RTV && ct == CTV) {                                             \
    launch_eval_t<P, RTV, CTV, MODE>(ep, nblk, st);                         \
    return 0;                                                               \
  }
  HOBO_EV(1, 1) HOBO_EV(1, 2) HOBO_EV(1, 4) HOBO_EV(1, 8)
  HOBO_EV(2, 1) HOBO_EV(2, 2) HOBO_EV(2, 4) HOBO_EV(2, 8)
  HOBO_EV(4, 1) HOBO_EV(4, 2) HOBO_EV(4, 4)
#undef HOBO_EV
  return -1;
}


// shape dispatch of one precision for both modes (defined in eval_prec.hip)
template <int P> int dispatch_eval_prec(const EvalParams& ep, int mode, int rt, int ct, long long B, hipStream_t st);

}  // namespace hobo
