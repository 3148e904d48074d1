// Blocked single-flip Metropolis annealing (hobo_anneal_batch) for instances
// of order <= 3 in the FP32 / BF16 precisions.
//
// A sweep visits the variables in order, 16 at a time.  For a block J of 16
// consecutive variables and the state x0 at the block's start, the matrix
// cores compute for 16 replicas
//   g_a(x0)       = sum_{S containing a} w_S prod_{S minus a} x0       (a in J)
//   H_ab(x0)      = sum_{S containing a, b} w_S prod_{S minus a, b} x0  (a < b in J)
// and the block's order-3 coefficients w_abc (a, b, c in J) come from a
// table.  Because the energy is multilinear, the field of bit a after the
// flips of earlier bits c of the block (x_c -> x_c + d_c, d_c in {-1, 0, 1})
// is exactly
//   g_a = g_a(x0) + sum_c d_c H_ac(x0) + sum_{c < c'} d_c d_c' w_{acc'},
// so the 16 sequential decisions run in registers: after a flip of c every
// later field takes g_a += d_c Hc_ac and every later coupling takes
// Hc_ab += d_c w_abc.  The chain of states, flip changes and decisions is the
// same as visiting one variable at a time.
//
// Work-group: 16 replicas, NW waves.  Phase 1 (all waves): the field tile is
// split over the waves by chunks, the 8 pair tiles by tile; every wave streams
// its chunks through a register ring that runs continuously across blocks
// and sweeps (loads do not depend on the state).  Phase 2 (wave 0): the 16
// decisions, lane = 4 * replica + s, sub-lane s holding bits s, s+4, s+8,
// s+12 of the block.  Meanwhile another wave stages the next block's
// coefficient table and its Philox uniforms -log(u).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "device_common.h"

namespace hobo {

constexpr int kRing = 8;       // chunks in flight per wave
constexpr int kMaskWin = 64;   // sweeps per launch when attempt masks are used
constexpr int kSweepWin = 256; // sweeps per launch otherwise (their trace waits in LDS)

template <int P> struct BSlot {
  BTile<P> b;
  unsigned long long d;  // run descriptor of this lane's K group
  int kind;              // 0 chunk, 1 chunk closing its list, 2 padding, 3 end of stream
  int tgt;               // list of the chunk: 0 fields, 1 + t pair tile t
  int ord;               // active-block ordinal of the slot
};

template <int HT> struct BProd {  // producer cursor (wave-uniform, scalar registers)
  int ord, s, q;         // active-block ordinal, its sweep and block
  int k, padded;         // next slot of the block, the block's padded slot count
  int cnt_g;             // field chunks of this wave (chunk g0 + k * NW)
  unsigned g0;
  int hs[HT], hn[HT];    // pair-tile m of this wave: slots hs .. hs + hn - 1 after the field chunks
  unsigned hc0[HT];      // its first chunk
};

template <int CTRL> __device__ inline int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
// value of sub-lane o of each quad (quad_perm o, o, o, o)
__device__ inline int quad_bcast(int v, int o) {
  switch (o) {
    case 0: return dpp_i<0x00>(v);
    case 1: return dpp_i<0x55>(v);
    case 2: return dpp_i<0xAA>(v);
    default: return dpp_i<0xFF>(v);
  }
}

// Eight-monomial mask of a run with at most one prefix variable (all runs of
// an order <= 3 instance's block lists): the run's byte of the replica's bits,
// cleared when the prefix bit is 0; constant and padding runs give 1 and 0.
__device__ inline unsigned run_mask1(unsigned long long d, const unsigned char* rb) {
  const unsigned np = (unsigned)(d >> 8) & 0xFFu;
  const unsigned pv = (unsigned)(d >> 16) & 0xFFu;
  const unsigned m = rb[(unsigned)d & 0x1Fu];
  const unsigned pb = (rb[pv >> 3] >> (pv & 7u)) & 1u;
  const unsigned v = (np == 1u && !pb) ? 0u : m;
  return np == kRunConst ? 1u : (np == kRunNull ? 0u : v);
}

template <int P, int NW>
__global__ __launch_bounds__(64 * NW) void anneal_block_kernel(AnnealParams p) {
  constexpr int D = kRing;
  constexpr int RPC = PT<P>::RPC;
  constexpr int TB = P == P_FP32 ? 2048 : (P == P_BF16X2 ? 2048 : 3072);
  constexpr int HT = (kPairTiles + NW - 1) / NW;  // pair tiles per wave
  __shared__ Luts L;
  __shared__ unsigned long long sbits[64];  // 16 replicas x 32 bytes
  __shared__ unsigned long long sbest[64];
  __shared__ float sG[NW][16][17];          // per-wave partial fields [rep][bit]
  __shared__ float sH[128][17];             // pair couplings [pair][rep]
  __shared__ __attribute__((aligned(16))) float sC[2][4096];  // order-3 table of the block [c][a][b]
  __shared__ double sL[2][16][17];          // -log(u) [rep][bit]
  __shared__ BlockMeta sBM[kMaxVars / kBlockBits];
  __shared__ unsigned short sAM[kMaskWin][kMaxVars / kBlockBits];  // attempted bits per (sweep, block)
  __shared__ unsigned short sAL[kMaskWin * (kMaxVars / kBlockBits)];  // active (sweep, block), stream order
  __shared__ int sNA;                                                  // their number
  __shared__ double strace[kSweepWin];  // per-sweep tile minima, written back after the launch's sweeps

  build_luts(&L);
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // wave index, uniform
  const int g = lane >> 4, j = lane & 15;
  // phase-2 layout
  const int rep = lane >> 2, sub = lane & 3;

  for (int it = blockIdx.x; it < p.n_items; it += gridDim.x) {
    __syncthreads();
    const AnnealItem item = p.items[it];
    const AnnealInstDev I = p.insts[item.inst];
    const long long r0 = (long long)item.tile16 * 16;
    const int N = I.n_vars;
    const int NB = I.nblocks;
    const bool masked = I.attempt != nullptr;
    for (int q = threadIdx.x; q < NB; q += blockDim.x) sBM[q] = I.blocks[q];
    if (masked) {  // attempted bits of every (sweep, block) of this launch
      const int ns = p.s_end - p.s_begin;
      for (int e = threadIdx.x; e < ns * NB; e += blockDim.x) {
        const int sr = e / NB, q = e - sr * NB;
        const unsigned char* m =
            I.attempt + ((size_t)item.tile16 * p.mask_rows + (size_t)(p.s_begin + sr - p.mask_s0)) * N + 16 * q;
        const int nb = N - 16 * q < 16 ? N - 16 * q : 16;
        unsigned v = 0;
        for (int c = 0; c < nb; ++c) v |= (gld(m + c) ? 1u : 0u) << c;
        sAM[sr][q] = (unsigned short)v;
      }
    }
    if (w == 0) {
      load_bits(sbits, I.x, I.W, I.B, r0, 16, lane);
      load_bits(sbest, p.cont ? I.best_x : I.x, I.W, I.B, r0, 16, lane);
    }
    __syncthreads();

    auto block_bits = [&](int s, int q) -> unsigned {
      const unsigned nb = __builtin_amdgcn_readfirstlane(sBM[q].nbits);
      const unsigned full = (1u << nb) - 1u;
      return masked ? __builtin_amdgcn_readfirstlane((unsigned)sAM[s - p.s_begin][q]) & full : full;
    };
    // the active blocks of the launch, in stream order: every (sweep, block)
    // without masks; with masks the list of those with an attempted bit
    if (masked) {
      if (w == 0) {
        const int tot = (p.s_end - p.s_begin) * NB;
        int cnt = 0;
        for (int b0 = 0; b0 < tot; b0 += 64) {
          const int e = b0 + lane;
          const int sr = e / (NB > 0 ? NB : 1), q = e - sr * NB;
          const bool act = e < tot && ((unsigned)sAM[sr][q] & ((1u << sBM[q].nbits) - 1u)) != 0u;
          const unsigned long long bal = __builtin_amdgcn_ballot_w64(act);
          const int pos = cnt + (int)__builtin_popcountll(bal & ((1ull << lane) - 1ull));
          if (act) sAL[pos] = (unsigned short)((sr << 4) | q);
          cnt += (int)__builtin_popcountll(bal);
        }
        if (lane == 0) sNA = cnt;
      }
      __syncthreads();
    }
    const int nact = masked ? __builtin_amdgcn_readfirstlane(sNA) : (p.s_end - p.s_begin) * NB;
    // (sweep, block) of active ordinal o, given those of o - 1
    auto step_block = [&](int o, int& s, int& q) {
      if (masked) {
        const int v = __builtin_amdgcn_readfirstlane((int)sAL[o]);
        s = p.s_begin + (v >> 4);
        q = v & 15;
      } else if (++q == NB) {
        q = 0;
        ++s;
      }
    };

    auto stage_block = [&](int s, int q, int bf, int tid, int nthr, bool do_u) {
      const u4* src = reinterpret_cast<const u4*>(I.triples + (size_t)q * 4096);
      u4* dst = reinterpret_cast<u4*>(sC[bf]);
      for (int e = tid; e < 1024; e += nthr) dst[e] = gld(src + e);
      if (do_u && tid < 64) {
        // lane (rep, grp) draws the four words of bits 16q + 4 grp .. +3
        const int rp = tid >> 2, gp = tid & 3;
        U64x4 o = philox((unsigned long long)(r0 + rp), (unsigned long long)s,
                         (unsigned long long)(4 * q + gp), 0ull, p.seed, I.inst_id);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const double u = (double)(o.w[e] >> 11) * 0x1.0p-53;
          sL[bf][rp][4 * gp + e] = u > 0.0 ? -log(u) : INFINITY;
        }
      }
    };

    // ---- state of the 16 replicas (wave 0, phase-2 layout)
    const long long myrow = r0 + rep;
    const bool live = myrow < I.B;
    double E = 0.0, bestE = 0.0;
    if (w == 0 && live) {
      E = gld(I.e_track + myrow);
      bestE = p.cont ? gld(I.best_track + myrow) : E;
    }

    // ---- producer: straight-line, scalar; block changes every `padded` slots
    BProd<HT> pr{};
    auto setup_block = [&]() {
      const BlockMeta& m = sBM[pr.q];
      const int ng = __builtin_amdgcn_readfirstlane((int)m.nchunks[0]);
      const int npt = __builtin_amdgcn_readfirstlane((int)m.npt);
      pr.cnt_g = ng > w ? (ng - w + NW - 1) / NW : 0;
      pr.g0 = __builtin_amdgcn_readfirstlane(m.chunk0[0]) + (unsigned)w;
      int tot = 0;
#pragma unroll
      for (int mm = 0; mm < HT; ++mm) {
        const int t = w + mm * NW;
        const bool ok = t < npt;
        pr.hs[mm] = tot;
        pr.hn[mm] = ok ? __builtin_amdgcn_readfirstlane((int)m.nchunks[1 + (ok ? t : 0)]) : 0;
        pr.hc0[mm] = ok ? __builtin_amdgcn_readfirstlane(m.chunk0[1 + (ok ? t : 0)]) : 0u;
        tot += pr.hn[mm];
      }
      tot += pr.cnt_g;
      pr.padded = tot <= D ? D : (tot + D - 1) / D * D;
      pr.k = 0;
    };
    // the producer enters its next active block; its slot counts are whole
    // rounds of D, so this happens only between rounds
    auto advance = [&]() {
      if (pr.k == pr.padded) {
        ++pr.ord;
        if (pr.ord < nact) {
          step_block(pr.ord, pr.s, pr.q);
          setup_block();
        }
        pr.k = 0;
      }
    };
    auto issue = [&](BSlot<P>& sl) {
      const int k = pr.k;
      unsigned c = 0;
      int kind = 2, tgt = 0;
      if (k < pr.cnt_g) {
        c = pr.g0 + (unsigned)(k * NW);
        kind = k == pr.cnt_g - 1 ? 1 : 0;
      } else {
        const int kk = k - pr.cnt_g;
#pragma unroll
        for (int mm = 0; mm < HT; ++mm)
          if (kk >= pr.hs[mm] && kk < pr.hs[mm] + pr.hn[mm]) {
            c = pr.hc0[mm] + (unsigned)(kk - pr.hs[mm]);
            kind = kk == pr.hs[mm] + pr.hn[mm] - 1 ? 1 : 0;
            tgt = 1 + w + mm * NW;
          }
      }
      pr.k = k + 1;
      if (pr.ord >= nact) {  // past the last block
        kind = 3;
        c = 0;
      }
      sl.kind = __builtin_amdgcn_readfirstlane(kind);
      sl.tgt = __builtin_amdgcn_readfirstlane(tgt);
      sl.ord = __builtin_amdgcn_readfirstlane(pr.ord);
      unsigned tix = kind <= 1 ? c + 1u : 0u;
      tix = tix < I.n_tiles ? tix : 0u;  // never outside the tile buffer
      load_tile<P>(sl.b, I.tiles + (size_t)tix * TB, lane);
      sl.d = gld(I.runs + (size_t)c * RPC + g);
    };

    pr.ord = 0;
    pr.s = p.s_begin;
    pr.q = 0;
    if (nact > 0) {
      if (masked) step_block(0, pr.s, pr.q);
      setup_block();
    }
    int co = 0, cs = pr.s, cq = pr.q;  // consumer: active ordinal, sweep, block
    int bf = 0;                        // buffer of the consumer block's table and uniforms
    if (co < nact) stage_block(cs, cq, 0, threadIdx.x, blockDim.x, true);
    BSlot<P> ring[D];
#pragma unroll
    for (int d = 0; d < D; ++d) issue(ring[d]);
    __syncthreads();

    AccT<P> acc;
    acc_zero<P>(acc);
    const unsigned char* rb = reinterpret_cast<const unsigned char*>(sbits) + j * 32;
    int s_prev = p.s_begin;  // sweeps before s_prev are closed

    auto end_sweep = [&](int s) {
      if (w == 0) {
        if (live && sub == 0 && E < bestE) {
          bestE = E;
          for (int qq = 0; qq < 4; ++qq) sbest[rep * 4 + qq] = sbits[rep * 4 + qq];
        }
        double v = live ? bestE : INFINITY;
        for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
        // kept in LDS: a global store here would make the stream's counted waits imprecise
        if (lane == 0) strace[s - p.s_begin] = v;
      }
    };

    while (co < nact) {
      while (s_prev < cs) end_sweep(s_prev++);
      const int q = cq;
      const unsigned amask = block_bits(cs, q);
      const BlockMeta& bmq = sBM[q];
      // ---- phase 1: zero this wave's outputs, then stream the block's chunks
      for (int e = lane; e < 256; e += 64) sG[w][e >> 4][e & 15] = 0.0f;
      for (int t = w; t < (int)bmq.npt; t += NW)
        for (int e = lane; e < 256; e += 64) sH[16 * t + (e & 15)][e >> 4] = 0.0f;
      // whole rounds of D slots belong to one block (its slot count is padded)
      while (ring[0].ord == co) {
        advance();
        // one round: the operand of slot d + 1 is generated before the
        // matrix-core work of slot d, so its LDS reads overlap that work
        auto gen = [&](const BSlot<P>& sl) {
          // every slot's registers are consumed on every path (padding slots
          // multiply a zero operand), so the counted waits stay exact
          const unsigned m1 = run_mask1(sl.d, rb);
          const unsigned msk = sl.kind <= 1 ? m1 : 0u;
          AOp<P> a;
          if constexpr (P == P_FP32) {
            a.v = u4{msk, 0u, 0u, 0u};
          } else {
            a.v = L.bf16[msk];
          }
          return a;
        };
        AOp<P> an = gen(ring[0]);
#pragma unroll
        for (int d = 0; d < D; ++d) {
          BSlot<P>& sl = ring[d];
          const AOp<P> a = an;
          if (d + 1 < D) an = gen(ring[d + 1 < D ? d + 1 : 0]);
          mma<P>(acc, a, sl.b);
          if (sl.kind == 1) {  // the chunk closes its list: fields [rep][bit], pairs [pair][rep]
            if (sl.tgt == 0) {
#pragma unroll
              for (int r = 0; r < 4; ++r) sG[w][4 * g + r][j] = acc.v[r];
            } else {
#pragma unroll
              for (int r = 0; r < 4; ++r) sH[16 * (sl.tgt - 1) + j][4 * g + r] = acc.v[r];
            }
            acc_zero<P>(acc);
          }
          issue(sl);
        }
      }
      lds_barrier();
      // ---- the next active block, for the staging wave
      int ns = cs, nq = cq;
      if (co + 1 < nact) step_block(co + 1, ns, nq);
      if (w == 0) {
        // ---- phase 2: sixteen sequential decisions
        const double beta = gld(p.beta + (cs - p.s_first));
        float gq[4];
        float hc[4][16];
        double lu[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int a = sub + 4 * i;
          float v = 0.0f;
#pragma unroll
          for (int ww = 0; ww < NW; ++ww) v += sG[ww][rep][a];
          gq[i] = v;
          lu[i] = sL[bf][rep][a];
#pragma unroll
          for (int b = 0; b < 16; ++b) {
            if (b < 4 * i + 3) {
              const int pc = b < a ? pair_col(b, a) : 0;
              const float h = sH[pc][rep];
              hc[i][b] = b < a ? h : 0.0f;
            }
          }
        }
        unsigned char* myb = reinterpret_cast<unsigned char*>(sbits) + rep * 32 + 2 * q;
        unsigned xb = (unsigned)myb[0] | ((unsigned)myb[1] << 8);
        const float* tri = sC[bf];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          if (!((amask >> c) & 1u)) continue;  // not attempted (or past the last variable)
          const int ic = c >> 2;
          const unsigned xc = (xb >> c) & 1u;
          const float gc = gq[ic];
          const float dE = xc ? -gc : gc;
          const bool take = dE <= 0.0f || (double)dE * beta < lu[ic];
          // the owner of bit c is sub-lane c & 3 of each replica's quad
          const int tk = quad_bcast(take ? 1 : 0, c & 3);
          const float dEo = __int_as_float(quad_bcast(__float_as_int(dE), c & 3));
          if (tk) {
            xb ^= 1u << c;
            E += (double)dEo;
          }
          if (__builtin_amdgcn_ballot_w64(tk != 0)) {  // any flip among the 16 replicas
            const float dl = tk ? (xc ? -1.0f : 1.0f) : 0.0f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              if (4 * i + 3 > c) {
                const int a = sub + 4 * i;
                gq[i] = fmaf(dl, hc[i][c], gq[i]);
                const float* row = tri + (c * 16 + a) * 16;
#pragma unroll
                for (int b = 0; b < 16; ++b)
                  if (b > c && b < 4 * i + 3) hc[i][b] = fmaf(dl, row[b], hc[i][b]);
              }
            }
          }
        }
        if (sub == 0) {
          myb[0] = (unsigned char)(xb & 0xFFu);
          myb[1] = (unsigned char)(xb >> 8);
        }
        if (NW == 1 && co + 1 < nact) stage_block(ns, nq, bf ^ 1, lane, 64, true);
      } else if (co + 1 < nact) {
        // the other waves stage the next block's triple table and uniforms
        stage_block(ns, nq, bf ^ 1, threadIdx.x - 64, 64 * (NW - 1), true);
      }
      // every load issued so far has landed (the ring's were issued before
      // phase 2): the stream loop then starts from a known count of
      // outstanding loads and keeps its ring in flight
      __builtin_amdgcn_s_waitcnt(0x0F70);
      lds_barrier();
      bf ^= 1;
      ++co;
      cs = ns;
      cq = nq;
    }
    while (s_prev < p.s_end) end_sweep(s_prev++);

    // write back (wave 0)
    if (w == 0) {
      if (I.trace_part)
        for (int s = p.s_begin + lane; s < p.s_end; s += 64)
          I.trace_part[(size_t)item.tile16 * p.sweeps + (s - p.s_first)] = strace[s - p.s_begin];
      const int rho = lane >> 2, qw = lane & 3;
      const long long r = r0 + rho;
      if (qw < I.W && r < I.B) {
        I.x[(long long)qw * I.B + r] = sbits[lane];
        I.best_x[(long long)qw * I.B + r] = sbest[lane];
      }
      if (live && sub == 0) {
        I.e_track[myrow] = E;
        I.best_track[myrow] = bestE;
      }
    }
  }
}

template <int P, int NW>
static void launch_block_t(const AnnealParams& ap, int nblk, hipStream_t st) {
  TimedLaunch tl(0, st);
  hipLaunchKernelGGL((anneal_block_kernel<P, NW>), dim3((unsigned)nblk), dim3(64 * NW), 0, st, ap);
}

int launch_anneal_block(const AnnealParams& ap, int prec, int nw, int nblk, hipStream_t st) {
#define HOBO_AB(PV, NWV)                     \
  if (prec == PV && nw == NWV) {             \
    launch_block_t<PV, NWV>(ap, nblk, st);   \
    return 0;                                \
  }
  HOBO_AB(P_FP32, 1) HOBO_AB(P_FP32, 2) HOBO_AB(P_FP32, 4) HOBO_AB(P_FP32, 8)
  HOBO_AB(P_BF16X2, 1) HOBO_AB(P_BF16X2, 2) HOBO_AB(P_BF16X2, 4) HOBO_AB(P_BF16X2, 8)
  HOBO_AB(P_BF16X3, 1) HOBO_AB(P_BF16X3, 2) HOBO_AB(P_BF16X3, 4) HOBO_AB(P_BF16X3, 8)
#undef HOBO_AB
  return -1;
}

int anneal_mask_window() { return kMaskWin; }
int anneal_sweep_window() { return kSweepWin; }

}  // namespace hobo
