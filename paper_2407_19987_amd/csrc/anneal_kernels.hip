// Batched single-flip Metropolis annealing (hobo_anneal_batch): the
// persistent multi-instance annealing kernel and its setup / finish kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>
#include <type_traits>

#include "device_common.h"

namespace hobo {

// ============================================================ annealer (per-bit slabs)
// k-th 16-column tile of wave w among cs waves, folded (w, 2cs-1-w, 2cs+w, ...)
// so that the triangular layouts give every wave the same amount of work
__host__ __device__ inline int wave_tile(int k, int w, int cs) { return k * cs + ((k & 1) ? cs - 1 - w : w); }

// ring depth of the coefficient stream (chunks in flight per wave)
// (eight-wave groups run two waves per SIMD and get half the registers)
template <int P, int CTW, int CS> constexpr int ring_depth() {
  constexpr int per = CTW * PT<P>::NLD * 4 + (P == P_INT8X4 ? 5 : 3);
  constexpr int d = (CS >= 8 ? 88 : 176) / per;
  return d < 2 ? 2 : (d > 16 ? 16 : d);
}

template <int P, int CTW> struct Slot {
  BTile<P> b[CTW];
  unsigned long long d0, d1;  // run descriptors of this lane's group
  unsigned att;               // 1 if the chunk's variable is visited this sweep
  int s, c;                   // sweep and chunk index (c < 0: empty)
};

// Chunk metadata is staged in LDS in blocks of kMetaBlock chunks; the last
// block absorbs the remainder (up to 2 kMetaBlock - 1 chunks), so no block is
// shorter than the ring depth and the producer never enters a block before
// the consumer has staged it.
constexpr int kMetaBlock = 512;
constexpr int kTraceEpoch = 256;  // sweeps whose trace values wait in LDS

// One work-group anneals 16 replicas.  Its CS waves split the 16-column tiles
// of every slab (wave_tile); each wave streams its tiles of the sweep's chunk
// sequence through a register ring D chunks deep.  Every chunk issues the
// same loads into its own ring slot (absent tiles read the zero tile 0) and
// the chunk metadata comes from LDS (staged kMetaBlock chunks at a time), so
// the compiler's counted waits keep the later chunks in flight.  At the end of
// a slab each wave writes its per-tile row sums to LDS; after one barrier
// every wave adds the tiles in column order and takes the same Metropolis
// decisions on its own copy of the bits, so no second barrier is needed.
template <int P, int CTW, int CS>
__global__ __launch_bounds__(64 * CS) void anneal_kernel(AnnealParams p) {
  constexpr int RPC = PT<P>::RPC;
  constexpr int D = ring_depth<P, CTW, CS>();
  __shared__ Luts L;
  __shared__ unsigned long long sbits[CS][64];
  __shared__ unsigned long long sbest[64];
  __shared__ double spart[2][16][16];
  __shared__ double sa[256];
  __shared__ ChunkMeta smeta[2][2 * kMetaBlock];
  __shared__ double strace[kTraceEpoch];
  __shared__ double sbeta[kTraceEpoch];
  build_luts<P>(&L);
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, j = lane & 15;
  const bool owner = j < 4;
  const int orow = 4 * g + j;
  unsigned char* myb = reinterpret_cast<unsigned char*>(sbits[w]);
  const int tb = (P == P_FP32 || P == P_BF16X2 || P == P_FP16X2) ? 2048 : (P == P_BF16X3 ? 3072 : 4096);
  int buf = 0;

  for (int it = blockIdx.x; it < p.n_items; it += gridDim.x) {
    const AnnealItem item = p.items[it];
    const AnnealInstDev I = p.insts[item.inst];
    const long long r0 = (long long)item.tile16 * 16;
    const int N = I.n_vars;
    const int T = (N + 15) >> 4;
    const int C = (int)I.n_chunks;
    const int S = p.sweeps;
    const int nblk = C / kMetaBlock > 1 ? C / kMetaBlock : 1;
    auto blk_of = [&](int c) { return c / kMetaBlock < nblk ? c / kMetaBlock : nblk - 1; };

    // stage metadata block `blk` (of the chunk list) into buffer `slot`
    auto stage_meta = [&](int blk, int slot) {
      const int c0 = blk * kMetaBlock;
      const int cnt = blk == nblk - 1 ? C - c0 : kMetaBlock;
      for (int q = threadIdx.x; q < cnt; q += blockDim.x)
        smeta[slot][q] = __builtin_bit_cast(ChunkMeta, gld(reinterpret_cast<const unsigned long long*>(I.chunks) + c0 + q));
    };
    load_bits(sbits[w], I.x, I.W, I.B, r0, 16, lane);
    if (w == 0) load_bits(sbest, p.cont ? I.best_x : I.x, I.W, I.B, r0, 16, lane);
    for (int q = threadIdx.x; q < N; q += blockDim.x) sa[q] = gld(&I.slabs[q].a_f);
    {  // the first two blocks of the stream, in the buffers their position selects
      const int par = nblk > 2 ? (int)(((long long)p.s_begin * nblk) & 1) : 0;
      if (C > 0) stage_meta(0, par);
      if (nblk > 1) stage_meta(1, par ^ 1);
    }
    const long long myrow = r0 + orow;
    const bool live_row = owner && myrow < I.B;
    double E = 0.0, bestE = 0.0;
    if (live_row) {
      E = gld(I.e_track + myrow);
      bestE = p.cont ? gld(I.best_track + myrow) : E;
    }
    unsigned long long rw[4] = {0, 0, 0, 0};
    int rw_key = -1;  // (sweep, 16-bit block) of the Philox words held
    __syncthreads();

    AccT<P> acc[CTW];
#pragma unroll
    for (int k = 0; k < CTW; ++k) acc_zero<P>(acc[k]);
    const unsigned char* att_base =
        I.attempt ? I.attempt + ((size_t)item.tile16 * p.mask_rows - p.mask_s0) * N : p.ones;
    const int att_on = I.attempt ? 1 : 0;
    // with at most two blocks both stay staged (buffer = block); with more,
    // blocks are restaged in stream order and alternate buffers
    auto meta_of = [&](int s, int c) -> ChunkMeta {
      const int blk = blk_of(c);
      const int bufi = nblk > 2 ? (int)(((long long)s * nblk + blk) & 1) : blk;
      return smeta[bufi][c - blk * kMetaBlock];
    };

    // ---- producer cursor: sweep ps, chunk pc (advanced without division)
    int ps = 0, pc = 0, ps_end = 0;
    auto issue = [&](Slot<P, CTW>& sl) {
      const bool valid = ps < ps_end;
      const int c = valid ? pc : 0;
      const int s = valid ? ps : 0;
      sl.c = valid ? c : -1;
      sl.s = s;
      const ChunkMeta m = valid ? meta_of(s, c) : ChunkMeta{};
#pragma unroll
      for (int k = 0; k < CTW; ++k) {
        const int t = wave_tile(k, w, CS);
        const bool have = t < T && t >= m.t_lo && t < m.t_hi;
        unsigned idx = have ? m.tile_off + (unsigned)(t - m.t_lo) : 0u;
        idx = idx < I.n_tiles ? idx : 0u;  // never outside the tile buffer
        load_tile<P>(sl.b[k], I.tiles + (size_t)idx * tb, lane);
      }
      if constexpr (P == P_INT8X4) {
        sl.d0 = gld(I.runs + c * RPC + 2 * g);
        sl.d1 = gld(I.runs + c * RPC + 2 * g + 1);
      } else {
        sl.d0 = gld(I.runs + c * RPC + g);
      }
      sl.att = vload_uniform(att_base, att_on ? (long long)s * N + m.bit : 0);
      if (valid && ++pc == C) {
        pc = 0;
        ++ps;
      }
    };

    int cs_cur = p.s_begin;  // sweep the consumer is in
    auto end_sweep = [&](int s) {
      if (live_row && E < bestE) {
        bestE = E;
        if (w == 0)
          for (int q = 0; q < 4; ++q) sbest[orow * 4 + q] = sbits[0][orow * 4 + q];
      }
      if (w == 0) {
        // kept in LDS: a global store here would make the stream's counted waits imprecise
        double v = live_row ? bestE : INFINITY;
        for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
        if (lane == 0) strace[s % kTraceEpoch] = v;
      }
    };

    // RESTAGE: the chunk list has more than two metadata blocks, so they are
    // restaged as the stream advances (a separate copy of the stream loop,
    // so the common case carries no staging branch in its hot path)
    auto consume = [&](Slot<P, CTW>& sl, auto restage) {
      if (sl.c < 0) return;
      while (sl.s > cs_cur) end_sweep(cs_cur++);
      if constexpr (decltype(restage)::value) {
        // entering a metadata block: stage the block after it into the buffer
        // of the block before, once every wave has consumed that block (the
        // first barrier; the producers are fewer than kMetaBlock chunks ahead,
        // so none of them reads it either), and before any producer reaches
        // the staged block (the second)
        if (sl.c % kMetaBlock == 0 && sl.c / kMetaBlock < nblk) {
          const long long gb = (long long)sl.s * nblk + sl.c / kMetaBlock + 1;
          lds_barrier();
          if (gb < (long long)S * nblk) stage_meta((int)(gb % nblk), (int)(gb & 1));
          lds_barrier();
        }
      }
      if (!__builtin_amdgcn_readfirstlane(sl.att)) return;
      const ChunkMeta m = meta_of(sl.s, sl.c);
      {
        AOp<P> a;
        const unsigned char* rb = myb + j * 32;
        if constexpr (P == P_FP32) {
          a.v = u4{run_mask(sl.d0, rb), 0u, 0u, 0u};
        } else if constexpr (P == P_INT8X4) {
          unsigned long long lo8 = L.i8[run_mask(sl.d0, rb)], hi8 = L.i8[run_mask(sl.d1, rb)];
          a.v = u4{(unsigned)lo8, (unsigned)(lo8 >> 32), (unsigned)hi8, (unsigned)(hi8 >> 32)};
        } else {
          a.v = L.bf16[run_mask(sl.d0, rb)];
        }
#pragma unroll
        for (int k = 0; k < CTW; ++k) {
          const int t = wave_tile(k, w, CS);
          if (t < T && t >= m.t_lo && t < m.t_hi) mma<P>(acc[k], a, sl.b[k]);
        }
      }
      if (!m.seg_end) return;
      // ---- end of the slab of bit i: g_i = w_i + sum_c x_c G_c, then Metropolis
      const int i = m.bit;
#pragma unroll
      for (int k = 0; k < CTW; ++k) {
        const int t = wave_tile(k, w, CS);
        if (t < T) {
          double v[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int col = 16 * t + j;
            v[r] = (col < N && bit_at(myb + (4 * g + r) * 32, col)) ? acc_f<P>(acc[k], r, I.inv_scale) : 0.0;
          }
          const double rs = rowsum4(v[0], v[1], v[2], v[3], j);
          if ((j & 3) == 0) spart[buf][t][4 * g + (j >> 2)] = rs;
        }
        acc_zero<P>(acc[k]);
      }
      const int key = (sl.s << 4) | (i >> 4);
      if (key != rw_key) {
        rw_key = key;
        // lane (g, j) draws the words of replica 4g + (j & 3) for bits 16*(i/16) + 4*(j>>2) .. +3
        const long long rr = r0 + 4 * g + (j & 3);
        U64x4 o = philox((unsigned long long)rr, (unsigned long long)sl.s,
                         (unsigned long long)(4 * (i >> 4) + (j >> 2)), 0ull, p.seed, I.inst_id);
        rw[0] = o.w[0]; rw[1] = o.w[1]; rw[2] = o.w[2]; rw[3] = o.w[3];
      }
      // the word of (row 4g + j, bit i) sits in lane (g, 4*((i>>2)&3) + j) for j < 4
      const unsigned long long word = rw[i & 3];
      unsigned lo32 = (unsigned)word, hi32 = (unsigned)(word >> 32);
      switch ((i >> 2) & 3) {
        case 1: lo32 = dpp_u<kDppRowRor12>(lo32); hi32 = dpp_u<kDppRowRor12>(hi32); break;
        case 2: lo32 = dpp_u<kDppRowRor8b>(lo32); hi32 = dpp_u<kDppRowRor8b>(hi32); break;
        case 3: lo32 = dpp_u<kDppRowRor4>(lo32); hi32 = dpp_u<kDppRowRor4>(hi32); break;
        default: break;
      }
      lds_barrier();
      if (live_row) {
        double h = 0.0;
        for (int t = 0; t < T; ++t) h += spart[buf][t][orow];
        const double gval = sa[i] + h;
        unsigned char* rb = myb + orow * 32;
        const double dE = bit_at(rb, i) ? -gval : gval;
        const unsigned long long r64 = ((unsigned long long)hi32 << 32) | lo32;
        const double u = (double)(r64 >> 11) * 0x1.0p-53;
        bool take = dE <= 0.0;
        if (!take) take = u < exp(-dE * sbeta[sl.s % kTraceEpoch]);
        if (take) {
          rb[i >> 3] ^= (unsigned char)(1u << (i & 7));
          E += dE;
        }
      }
      buf ^= 1;
    };

    auto run = [&](auto restage) {
      Slot<P, CTW> ring[D];
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
    // the run in epochs of kTraceEpoch sweeps; the trace leaves LDS between them
    for (int s0 = p.s_begin; s0 < p.s_end; s0 += kTraceEpoch) {
      const int s1 = p.s_end - s0 < kTraceEpoch ? p.s_end : s0 + kTraceEpoch;
      ps = s0;
      pc = 0;
      ps_end = C > 0 ? s1 : s0;
      // inverse temperatures of this epoch (the stream reads them from LDS)
      __syncthreads();
      for (int q = threadIdx.x; q < s1 - s0; q += blockDim.x) sbeta[(s0 + q) % kTraceEpoch] = gld(p.beta + (s0 - p.s_first) + q);
      __syncthreads();
      if (nblk > 2)
        run(std::integral_constant<bool, true>{});
      else
        run(std::integral_constant<bool, false>{});
      while (cs_cur < s1) end_sweep(cs_cur++);
      if (I.trace_part && w == 0 && lane == 0)
        for (int s = s0; s < s1; ++s) I.trace_part[(size_t)item.tile16 * S + (s - p.s_first)] = strace[s % kTraceEpoch];
    }

    // write back (wave 0 holds the outputs; all waves hold identical states)
    if (w == 0) {
      const int rho = lane >> 2, q = lane & 3;
      const long long r = r0 + rho;
      if (q < I.W && r < I.B) {
        I.x[(long long)q * I.B + r] = sbits[0][lane];
        I.best_x[(long long)q * I.B + r] = sbest[lane];
      }
      if (live_row) {
        I.e_track[myrow] = E;
        I.best_track[myrow] = bestE;
      }
    }
    __syncthreads();
  }
}

#ifndef HOBO_SLAB_PREC
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

// Term-loop energies of x (which = 0, written to the tracked start energy)
// or of best_x (which = 1, written to the rescored output); grid.z = instance
__device__ inline TermJob term_job(const InstSmall& I, int which) {
  TermJob J{};
  J.rec = I.rec;
  J.n_mono = I.n_mono;
  J.W = I.W;
  J.integer = I.integer;
  J.B = I.B;
  J.bits = which ? I.best_x : I.x;
  J.part = I.term_part;
  return J;
}

__global__ __launch_bounds__(256) void term_masks_multi(const InstSmall* in, int which) {
  const InstSmall I = in[blockIdx.y];
  if ((long long)blockIdx.x * 256 >= I.B) return;
  term_masks(term_job(I, which), blockIdx.x);
}

__global__ __launch_bounds__(256) void term_partial_multi(const InstSmall* in, int which) {
  const InstSmall I = in[blockIdx.z];
  if ((long long)blockIdx.x * 256 >= I.B || (int)blockIdx.y * kTermGroup >= I.n_mono) return;
  term_partial(term_job(I, which), blockIdx.x, blockIdx.y);
}

__global__ void term_reduce_multi(const InstSmall* in, int which) {
  const InstSmall I = in[blockIdx.y];
  const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= I.B) return;
  const int G = term_groups(I.n_mono);
  double sf = 0.0;
  long long si = 0;
  for (int q = 0; q < G; ++q) {
    if (I.integer)
      si += reinterpret_cast<const long long*>(I.term_part)[(long long)q * I.B + b];
    else
      sf += reinterpret_cast<const double*>(I.term_part)[(long long)q * I.B + b];
  }
  if (I.n_mono == 0) { sf = 0.0; si = 0; }
  if (which == 0) {
    I.e_track[b] = I.integer ? (double)si : sf;
  } else if (which == 2) {
    I.best_track[b] = I.integer ? (double)si : sf;
  } else if (I.best_out) {
    if (I.integer)
      reinterpret_cast<long long*>(I.best_out)[b] = si;
    else
      reinterpret_cast<double*>(I.best_out)[b] = sf;
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

#endif  // !HOBO_SLAB_PREC

template <int P, int CTW, int CS>
static void launch_anneal_t(const AnnealParams& ap, int nblk, hipStream_t st) {
  TimedLaunch tl(0, st);
  hipLaunchKernelGGL((anneal_kernel<P, CTW, CS>), dim3((unsigned)nblk), dim3(64 * CS), 0, st, ap);
}

// one precision's shape dispatch (each defined in the build of that precision)
template <int P> int dispatch_anneal_prec(const AnnealParams& ap, int ctw, int cs, int nblk, hipStream_t st);

#ifdef HOBO_SLAB_PREC
// this translation unit instantiates one precision's per-bit kernels (the
// file is compiled once per precision, so they build in parallel)
template <>
int dispatch_anneal_prec<HOBO_SLAB_PREC>(const AnnealParams& ap, int ctw, int cs, int nblk, hipStream_t st) {
  constexpr int P = HOBO_SLAB_PREC;
#define HOBO_AN(CTWV, CSV)                          \
  if (ctw == CTWV && cs == CSV) {                   \
    launch_anneal_t<P, CTWV, CSV>(ap, nblk, st);    \
    return 0;                                       \
  }
  HOBO_AN(1, 1) HOBO_AN(2, 1) HOBO_AN(4, 1) HOBO_AN(8, 1) HOBO_AN(16, 1)
  HOBO_AN(1, 2) HOBO_AN(2, 2) HOBO_AN(4, 2) HOBO_AN(8, 2)
  HOBO_AN(1, 4) HOBO_AN(2, 4) HOBO_AN(3, 4) HOBO_AN(4, 4)
  HOBO_AN(1, 8) HOBO_AN(2, 8)
#undef HOBO_AN
  return -1;
}

#else
void anneal_shape(int T, int cs_req, int* ctw, int* cs) {
  int c = cs_req;
  // default: one wave per column tile, up to eight waves (deepest rings)
  if (c != 1 && c != 2 && c != 4 && c != 8) c = T >= 8 ? 8 : (T >= 4 ? 4 : (T >= 2 ? 2 : 1));
  int per = (T + c - 1) / c;
  int w;
  if (c == 1) w = per <= 1 ? 1 : per <= 2 ? 2 : per <= 4 ? 4 : per <= 8 ? 8 : 16;
  else if (c == 2) w = per <= 1 ? 1 : per <= 2 ? 2 : per <= 4 ? 4 : 8;
  else if (c == 4) w = per;  // 1..4 are all instantiated
  else w = per <= 1 ? 1 : 2;
  *ctw = w;
  *cs = c;
}

int launch_anneal_block(const AnnealParams& ap, int prec, int nw, int nblk, hipStream_t st);
void launch_anneal_uniforms(const AnnealParams& ap, hipStream_t st);

// The annealing sequence of one launch plan, in three parts: random start
// states and start energies (FP64 / int64 term sums); the sweeps (blocked
// kernel items in windows, then per-bit slab kernel items); the FP64 rescore
// of the best states and the per-sweep trace minima.
int enqueue_anneal_setup(const AnnealTables& tb, const AnnealPlan& pl, void* stream, std::string* err) {
  hipStream_t st = (hipStream_t)stream;
  const InstSmall* sm = tb.d_small + pl.inst0;
  const unsigned ni = (unsigned)pl.ninst;
  if (pl.init_random) {
    long long wb = (long long)tb.max_W * tb.max_B;
    hipLaunchKernelGGL(init_random_multi, dim3((unsigned)((wb + 255) / 256), ni), dim3(256), 0, st, sm,
                       (unsigned long long)pl.seed);
  }
  const unsigned rb = (unsigned)((tb.max_B + 255) / 256);
  hipLaunchKernelGGL(term_masks_multi, dim3(rb, ni), dim3(256), 0, st, sm, 0);
  hipLaunchKernelGGL(term_partial_multi, dim3(rb, (unsigned)tb.max_groups, ni), dim3(256), 0, st, sm, 0);
  hipLaunchKernelGGL(term_reduce_multi, dim3(rb, ni), dim3(256), 0, st, sm, 0);
  if (pl.cont) {
    hipLaunchKernelGGL(term_masks_multi, dim3(rb, ni), dim3(256), 0, st, sm, 2);
    hipLaunchKernelGGL(term_partial_multi, dim3(rb, (unsigned)tb.max_groups, ni), dim3(256), 0, st, sm, 2);
    hipLaunchKernelGGL(term_reduce_multi, dim3(rb, ni), dim3(256), 0, st, sm, 2);
  }
  return hip_fail(hipGetLastError(), err, "anneal setup");
}

// Sweeps [s_begin, s_end) of the plan; attempt-mask row 0 is sweep mask_s0
// and every 16-replica group has mask_rows rows.  `cont`: the best states
// continue from an earlier part of the run.
int enqueue_anneal_sweeps(const AnnealTables& tb, const AnnealPlan& pl, int s_begin, int s_end, int mask_s0,
                          int mask_rows, int cont, void* stream, std::string* err) {
  hipStream_t st = (hipStream_t)stream;
  AnnealParams ap{};
  ap.insts = tb.d_inst;
  ap.sweeps = pl.sweeps;
  ap.s_first = pl.s_first;
  ap.mask_s0 = mask_s0;
  ap.mask_rows = mask_rows;
  ap.beta = tb.d_beta;
  ap.seed = pl.seed;
  ap.ones = tb.d_ones;
  if (pl.n_blk > 0) {
    ap.items = tb.d_items + pl.item0;
    ap.n_items = pl.n_blk;
    const int nblk = pl.n_blk < 2048 ? pl.n_blk : 2048;
    const int win0 = pl.masked ? anneal_mask_window() : anneal_sweep_window();
    const int win = tb.unif_sweeps > 0 && tb.unif_sweeps < win0 ? tb.unif_sweeps : win0;
    ap.unif_sweeps = tb.unif_sweeps;
    int s0 = s_begin;
    do {  // at least one launch: with no sweeps it writes the start states back as the best ones
      ap.s_begin = s0;
      ap.s_end = s_end - s0 < win ? s_end : s0 + win;
      ap.cont = (cont || s0 > s_begin) ? 1 : 0;
      // the window's Metropolis uniforms first (a kernel of their own)
      if (ap.s_end > ap.s_begin) launch_anneal_uniforms(ap, st);
      if (launch_anneal_block(ap, pl.prec, pl.nw_blk, nblk, st) != 0) {
        *err = "no blocked annealer kernel for this precision / width";
        return HOBO_ERR_UNSUPPORTED;
      }
      s0 += win;
    } while (s0 < s_end);
  }
  if (pl.n_slab > 0) {
    ap.items = tb.d_items + pl.item0 + pl.n_blk;
    ap.n_items = pl.n_slab;
    ap.s_begin = s_begin;
    ap.s_end = s_end;
    ap.cont = cont;
    const int nblk = pl.n_slab < 2048 ? pl.n_slab : 2048;  // one work-group per 16 replicas, persistent beyond
    int r = -1;
    switch (pl.prec) {
      case P_FP32: r = dispatch_anneal_prec<P_FP32>(ap, pl.ct, pl.nw, nblk, st); break;
      case P_BF16X2: r = dispatch_anneal_prec<P_BF16X2>(ap, pl.ct, pl.nw, nblk, st); break;
      case P_BF16X3: r = dispatch_anneal_prec<P_BF16X3>(ap, pl.ct, pl.nw, nblk, st); break;
      case P_FP16X2: r = dispatch_anneal_prec<P_FP16X2>(ap, pl.ct, pl.nw, nblk, st); break;
      case P_INT8X4: r = dispatch_anneal_prec<P_INT8X4>(ap, pl.ct, pl.nw, nblk, st); break;
      default: break;
    }
    if (r != 0) {
      *err = "no annealer kernel for this precision / width";
      return HOBO_ERR_UNSUPPORTED;
    }
  }
  return hip_fail(hipGetLastError(), err, "anneal launch");
}

int enqueue_anneal_finish(const AnnealTables& tb, const AnnealPlan& pl, void* stream, std::string* err) {
  hipStream_t st = (hipStream_t)stream;
  const InstSmall* sm = tb.d_small + pl.inst0;
  const unsigned ni = (unsigned)pl.ninst;
  const unsigned rb = (unsigned)((tb.max_B + 255) / 256);
  hipLaunchKernelGGL(term_masks_multi, dim3(rb, ni), dim3(256), 0, st, sm, 1);
  hipLaunchKernelGGL(term_partial_multi, dim3(rb, (unsigned)tb.max_groups, ni), dim3(256), 0, st, sm, 1);
  hipLaunchKernelGGL(term_reduce_multi, dim3(rb, ni), dim3(256), 0, st, sm, 1);
  if (pl.sweeps > 0)
    hipLaunchKernelGGL(trace_reduce_multi, dim3((unsigned)((pl.sweeps + 255) / 256), ni), dim3(256), 0, st,
                       sm, pl.sweeps);
  return hip_fail(hipGetLastError(), err, "anneal finish");
}

int enqueue_anneal_seq(const AnnealTables& tb, const AnnealPlan& pl, void* stream, std::string* err) {
  if (int s = enqueue_anneal_setup(tb, pl, stream, err)) return s;
  if (int s = enqueue_anneal_sweeps(tb, pl, pl.s_first, pl.s_first + pl.sweeps, pl.s_first, pl.sweeps, pl.cont,
                                    stream, err))
    return s;
  return enqueue_anneal_finish(tb, pl, stream, err);
}

#endif  // HOBO_SLAB_PREC

}  // namespace hobo
