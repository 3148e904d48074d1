// Blocked single-flip Metropolis annealing (hobo_anneal_batch) for instances
// of order <= 3 in the FP32 / BF16 precisions.
//
// A sweep visits the variables in order, 16 at a time.  For a block J of 16
// consecutive variables and the state x0 at the block's start, the matrix
// cores compute for 16 replicas
//   H_ab(x0)      = sum_{S containing a, b} w_S prod_{S minus a, b} x0  (a < b in J)
//   F_a(x0)       = sum of w_S prod_{S minus a} x0 over the S containing a
//                   and no other variable of J, minus the same over the S
//                   containing a and two others of J                    (a in J)
// and the decision wave completes the fields as
//   g_a(x0)       = F_a(x0) + sum_{b in J, b != a} x0_b H_ab(x0)
// (the terms with one other variable b of J are in x0_b H_ab once, those
// with two are there twice), so the field list carries about a fifth fewer
// rows.  The block's order-3 coefficients w_abc (a, b, c in J) come from a
// table.  Because the energy is multilinear, the field of bit a after the
// flips of earlier bits c of the block (x_c -> x_c + d_c, d_c in {-1, 0, 1})
// is exactly
//   g_a = g_a(x0) + sum_c d_c H_ac(x0) + sum_{c < c'} d_c d_c' w_{acc'},
// so the 16 sequential decisions run in registers: after a flip of c every
// later field takes g_a += d_c Hc_ac and every later coupling takes
// Hc_ab += d_c w_abc.  The chain of states, flip changes and decisions is the
// same as visiting one variable at a time.
//
// Work-group: 16 replicas, NW waves in two roles.  Waves 1 .. NW-1 stream:
// the field tile is split over them by chunks, the 8 pair tiles by tile, and
// every streaming wave keeps its chunks in flight through a register ring
// that runs continuously across blocks and sweeps (loads do not depend on the
// state).  Wave 0 decides: it holds the replicas' energies, stages the
// block's order-3 table (straight from global memory into LDS) and its
// Philox uniforms -log(u) while the others stream, then takes the 16
// decisions, lane = 4 * replica + s, sub-lane s holding bits s, s+4, s+8,
// s+12 of the block.  The roles' registers never live at the same time, so
// the kernel fits four waves per SIMD.  Each block's field list starts with
// the chunks that read no bit of the block before it in the sweep: the
// streaming waves compute those while wave 0 still decides that block.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "device_common.h"

namespace hobo {

constexpr int kRing = 8;       // chunks in flight per wave
constexpr int kBufferFlags = 0x00020000;  // buffer resource word 3: raw byte-addressed data
constexpr int kMaskWin = 64;   // sweeps per launch when attempt masks are used
constexpr int kSweepWin = 256; // sweeps per launch otherwise (their trace waits in LDS)

template <int P> struct BSlot {
  BTile<P> b;
  unsigned d;            // low word of the run descriptor of this lane's K group (all its fields here)
  int kind;              // 0 chunk, 1 chunk closing its list, 2 padding, 3 end of stream
  int tgt;               // list of the chunk: 0 fields, 1 + t pair tile t
  int ord;               // active-block ordinal of the slot
};

struct BProd {  // producer cursor (wave-uniform, scalar registers)
  int ord, s, q;   // active-block ordinal, its sweep and block
  int k;           // next slot of the block
  int pe, padded;  // the block's early slots and all its slots (whole rounds)
  unsigned off;    // first slot word of the block in the schedule
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

// A pointer every lane holds, in scalar registers.
template <class T> __device__ inline void* uniform_ptr(T* p) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v), hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return reinterpret_cast<void*>(((unsigned long long)hi << 32) | lo);
}

// Lane id read from the hardware counter where it is needed (the asm is not
// hoisted): values derived from it once and kept across the item loop would
// hold registers in both roles.
__device__ inline int lane_id() {
  int v;
  asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(v));
  return v;
}

// Eight-monomial mask of a run with at most one prefix variable (all runs of
// an order <= 3 instance's block lists): the run's byte of the replica's bits,
// cleared when the prefix bit is 0; constant and padding runs give 1 and 0.
__device__ inline unsigned run_mask1(unsigned d, const unsigned char* rb) {  // rb[16 k] = byte k
  const unsigned np = (unsigned)(d >> 8) & 0xFFu;
  const unsigned pv = (unsigned)(d >> 16) & 0xFFu;
  const unsigned m = rb[16u * ((unsigned)d & 0x1Fu)];
  const unsigned pb = (rb[16u * (pv >> 3)] >> (pv & 7u)) & 1u;
  const unsigned v = (np == 1u && !pb) ? 0u : m;
  return np == kRunConst ? 1u : (np == kRunNull ? 0u : v);
}

// Eight- and sixteen-wave groups keep to 128 VGPRs (four waves per SIMD);
// the two- and four-wave forms, whose streaming waves each carry more of the
// block, may use twice that and run two waves per SIMD.
template <int P, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW >= 8 ? 4 : 2))) void anneal_block_kernel(
    AnnealParams p) {
  static_assert(NW >= 2, "one decision wave and at least one streaming wave");
  // with sixteen waves, wave 1 stages the next block's table and uniforms
  // while wave 0 decides; narrower groups let wave 0 stage its own block
  constexpr bool STAGER = NW == 16;
  constexpr int NS = NW - 1 - (STAGER ? 1 : 0);  // streaming waves (the last NS)
  constexpr int W0 = NW - NS;                    // first streaming wave
  constexpr int NBUF = STAGER ? 2 : 1;           // buffers of the staged table and uniforms
  constexpr int D = kRing;
  constexpr int RPC = PT<P>::RPC;
  constexpr int TB = P == P_BF16X3 ? 3072 : 2048;
  // FP16X2 tiles and tables hold the coefficients times 2^scale_exp
  constexpr bool SCALED = P == P_FP16X2;
  static_assert(D == kBlockRing, "the schedule is built in rounds of the ring depth");
  __shared__ unsigned long long sbits[64];  // 16 replicas x 32 bytes
  // the same bits byte-transposed, [byte][replica]: the streaming waves' reads
  // of one byte position for 16 replicas fall in 4 consecutive banks
  __shared__ __attribute__((aligned(16))) unsigned char sbT[32][16];
  // nibble -> four BF16 (FP16) values 0 / 1.0 (16 entries x 8 bytes: every entry in
  // its own two banks, so the operand reads never conflict)
  __shared__ unsigned long long sNib[16];
  __shared__ unsigned long long sbest[64];
  // per-streaming-wave partial fields, [rep][4 * sub + i] holds bit sub + 4 i
  // (two buffers: a block's early chunks run while the decisions of the one
  // before it still read its fields)
  __shared__ __attribute__((aligned(16))) float sG[2][NS][16][16];
  // pair couplings [rep][a][b], stored at both (a, b) and (b, a); replicas
  // 260 floats apart (no bank conflicts when the decision wave reads its
  // rows as float4)
  constexpr int kHRep = 260;
  __shared__ __attribute__((aligned(16))) float sH[16 * kHRep];
  __shared__ unsigned short sPC[128];  // pair column -> (a << 8) | b (unused columns -> 0)
  __shared__ __attribute__((aligned(16))) float sC[NBUF][4096];  // order-3 table of the block [c][a][b]
  __shared__ __attribute__((aligned(16))) double sL[NBUF][16][16];  // -log(u) [rep][bit]
  __shared__ BlockMeta sBM[kMaxVars / kBlockBits];
  __shared__ unsigned short sAM[kMaskWin][kMaxVars / kBlockBits];  // attempted bits per (sweep, block)
  __shared__ unsigned short sAL[kMaskWin * (kMaxVars / kBlockBits)];  // active (sweep, block), stream order
  __shared__ int sNA;                                                  // their number
  // schedule header of each (block, streaming wave): first slot word, then
  // (early slots << 16) | slots
  __shared__ uint2 sHdr[kMaxVars / kBlockBits][NS];
  __shared__ double strace[kSweepWin];  // per-sweep tile minima, written back after the launch's sweeps

  for (int n = threadIdx.x; n < 16; n += blockDim.x) {
    unsigned long long v = 0;
    for (int i = 0; i < 4; ++i) v |= (unsigned long long)(((n >> i) & 1) ? one16<P>() : 0u) << (16 * i);
    sNib[n] = v;
  }
  for (int e = threadIdx.x; e < 128; e += blockDim.x) {
    unsigned v = 0;
    for (int a = 1; a < 16; ++a)
      for (int b = 0; b < a; ++b)
        if (pair_col(b, a) == e) v = (unsigned)(a << 8 | b);
    sPC[e] = (unsigned short)v;
  }
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // wave index, uniform

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
      const unsigned char* sb = reinterpret_cast<const unsigned char*>(sbits);
      for (int t = lane; t < 512; t += 64) sbT[t >> 4][t & 15] = sb[(t & 15) * 32 + (t >> 4)];
    }
    // the streaming waves only ever add their results to zeroed outputs;
    // wave 0 clears each output again once it has read it
    for (int e = threadIdx.x; e < 2 * NS * 64; e += blockDim.x)
      reinterpret_cast<f4*>(&sG[0][0][0][0])[e] = f4{0.f, 0.f, 0.f, 0.f};
    for (int e = threadIdx.x; e < 16 * kHRep / 4; e += blockDim.x)
      reinterpret_cast<f4*>(&sH[0])[e] = f4{0.f, 0.f, 0.f, 0.f};
    __syncthreads();

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
    for (int e = threadIdx.x; e < NB * NS; e += blockDim.x)
      sHdr[e / NS][e % NS] = uint2{gld(I.sched_hdr + 2 * e), gld(I.sched_hdr + 2 * e + 1)};
    __syncthreads();
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
    int cs = p.s_begin, cq = 0;  // sweep and block of active ordinal 0
    if (masked && nact > 0) step_block(0, cs, cq);

    // Staging of block (s, q) into buffer bf, by one wave: its order-3
    // table, straight from global memory into LDS (no registers; in LDS once
    // the wave's loads have drained), and the uniforms -log(u) of its 16 x 16
    // decisions.
    auto stage_table = [&](int q, int bf) {
      const int lane = lane_id();
      const float* src = I.triples + (size_t)q * 4096;
#pragma unroll
      for (int e = 0; e < 16; ++e)
        __builtin_amdgcn_global_load_lds(src + 256 * e + 4 * lane,
                                         (__attribute__((address_space(3))) void*)(&sC[bf][256 * e]), 16, 0, 0);
    };
    // the uniforms come from the window's buffer (anneal_uniforms_kernel), 2 KB
    auto stage_uniforms = [&](int s, int q, int bf) {
      const int lane = lane_id();
      const double* src = I.unif + ((size_t)item.tile16 * p.unif_sweeps + (s - p.s_begin)) * ((size_t)NB * 256) +
                          (size_t)q * 256;
#pragma unroll
      for (int e = 0; e < 2; ++e)
        __builtin_amdgcn_global_load_lds(src + 128 * e + 2 * lane,
                                         (__attribute__((address_space(3))) void*)(&sL[bf][0][0] + 128 * e), 16, 0,
                                         0);
    };
    auto drain = []() { __builtin_amdgcn_s_waitcnt(0x0F70); };  // vmcnt(0)

    // Every role passes two work-group barriers per active block: A when the
    // block's fields and couplings are in LDS, B when its decisions are.  The
    // streaming waves run a block's early part (field chunks that read no bit
    // of the block before) between A and B of the block before.
    if (w == 0) {
      // ================= decision wave: replica state, decisions
      // (raised priority: its chain of decisions is the one the others wait for)
      __builtin_amdgcn_s_setprio(2);
      const int lane = lane_id();
      const int rep = lane >> 2, sub = lane & 3;
      const long long myrow = r0 + rep;
      const bool live = myrow < I.B;
      double E = 0.0, bestE = 0.0;
      if (live) {
        E = gld(I.e_track + myrow);
        bestE = p.cont ? gld(I.best_track + myrow) : E;
      }
      int s_prev = p.s_begin;  // sweeps before s_prev are closed
      auto end_sweep = [&](int s) {
        if (live && sub == 0 && E < bestE) {
          bestE = E;
          for (int qq = 0; qq < 4; ++qq) sbest[rep * 4 + qq] = sbits[rep * 4 + qq];
        }
        double v = live ? bestE : INFINITY;
        for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
        if (lane == 0) strace[s - p.s_begin] = v;
      };
      for (int co = 0; co < nact; ++co) {
        if (co > 0) step_block(co, cs, cq);
        while (s_prev < cs) end_sweep(s_prev++);
        const int q = cq;
        // per-block lane layout (its LDS addresses are not kept across blocks)
        const int lane = lane_id();
        const int rep = lane >> 2, sub = lane & 3;
        const unsigned nbq = __builtin_amdgcn_readfirstlane(sBM[q].nbits);
        const unsigned full = (1u << nbq) - 1u;
        const unsigned amask =
            masked ? __builtin_amdgcn_readfirstlane((unsigned)sAM[cs - p.s_begin][q]) & full : full;
        const int bf = STAGER ? (co & 1) : 0;
        // while the streaming waves compute the block's fields: its table and uniforms
        if (!STAGER) {
          stage_table(q, 0);
          stage_uniforms(cs, q, 0);
          drain();
        }
        // in the scaled units of FP16X2 flip changes the inverse temperature
        // carries the factor 2^-scale_exp (exact), so the test is unchanged
        const double beta = SCALED ? gld(p.beta + (cs - p.s_first)) * I.inv_scale : gld(p.beta + (cs - p.s_first));
        lds_barrier();  // A
        // ---- sixteen sequential decisions, sub-lane s holding bits s, s+4, s+8, s+12
        float gq[4];
        float hc[4][16];
        double lu[4];
        {
          const int gb = co & 1;
          f4 acc4 = *reinterpret_cast<const f4*>(&sG[gb][0][rep][4 * sub]);
#pragma unroll
          for (int ww = 1; ww < NS; ++ww) acc4 += *reinterpret_cast<const f4*>(&sG[gb][ww][rep][4 * sub]);
#pragma unroll
          for (int i = 0; i < 4; ++i) gq[i] = acc4[i];
#pragma unroll
          for (int ww = 0; ww < NS; ++ww) reinterpret_cast<f4*>(&sG[gb][ww][0][0])[lane] = f4{0.f, 0.f, 0.f, 0.f};
        }
        unsigned char* myb = reinterpret_cast<unsigned char*>(sbits) + rep * 32 + 2 * q;
        unsigned xb = (unsigned)myb[0] | ((unsigned)myb[1] << 8);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int a = sub + 4 * i;
          lu[i] = sL[bf][rep][a];
#pragma unroll
          for (int b = 0; b < 16; ++b) {
            if (b < 4 * i + 3) {
              const float h = sH[rep * kHRep + a * 16 + b];
              hc[i][b] = b < a ? h : 0.0f;
            }
          }
        }
        // The field list leaves out the terms with exactly one other bit b of
        // the block and holds the block's triples negated: adding
        // sum_b x0_b H_ab(x0) completes g_a(x0).  Row a of H (stored at both
        // (a, b) and (b, a)) is read as four float4, two rows at a time (a
        // loop of two steps, with the lane layout read again, keeps the
        // decision chain's registers free).
        {
          const int ln = lane_id();
          const int rp = ln >> 2, sb = ln & 3;
          const unsigned char* xr = reinterpret_cast<const unsigned char*>(sbits) + rp * 32 + 2 * q;
          const unsigned x0 = (unsigned)xr[0] | ((unsigned)xr[1] << 8);
#pragma unroll 1
          for (int i2 = 0; i2 < 4; i2 += 2) {
            float corr[2] = {0.0f, 0.0f};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int a = sb + 4 * (i2 + h);
#pragma unroll
              for (int k = 0; k < 4; ++k) {
                const f4 v = *reinterpret_cast<const f4*>(&sH[rp * kHRep + a * 16 + 4 * k]);
#pragma unroll
                for (int e = 0; e < 4; ++e)
                  corr[h] += (4 * k + e != a && ((x0 >> (4 * k + e)) & 1u)) ? v[e] : 0.0f;
              }
            }
            if (i2 == 0) {
              gq[0] += corr[0];
              gq[1] += corr[1];
            } else {
              gq[2] += corr[0];
              gq[3] += corr[1];
            }
          }
        }
        for (int e = lane; e < 16 * kHRep / 4; e += 64)
          reinterpret_cast<f4*>(&sH[0])[e] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          if (!((amask >> c) & 1u)) continue;  // not attempted (or past the last variable)
          // the order-3 rows w_{c a b} this step may need (b = c+1 .. 4i+2), read
          // as float4 before the decision so that their latency overlaps it
          f4 rw[4][4];
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int k = 0; k < 4; ++k)
              if (4 * i + 3 > c && k >= ((c + 1) >> 2) && k <= i)
                rw[i][k] = *reinterpret_cast<const f4*>(&sC[bf][(c * 16 + sub + 4 * i) * 16 + 4 * k]);
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
            E += SCALED ? (double)dEo * I.inv_scale : (double)dEo;
          }
          if (__builtin_amdgcn_ballot_w64(tk != 0)) {  // any flip among the 16 replicas
            const float dl = tk ? (xc ? -1.0f : 1.0f) : 0.0f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              if (4 * i + 3 > c) {
                gq[i] = fmaf(dl, hc[i][c], gq[i]);
#pragma unroll
                for (int b = 0; b < 16; ++b)
                  if (b > c && b < 4 * i + 3) hc[i][b] = fmaf(dl, rw[i][b >> 2][b & 3], hc[i][b]);
              }
            }
          }
        }
        if (sub == 0) {
          myb[0] = (unsigned char)(xb & 0xFFu);
          myb[1] = (unsigned char)(xb >> 8);
          sbT[2 * q][rep] = (unsigned char)(xb & 0xFFu);
          sbT[2 * q + 1][rep] = (unsigned char)(xb >> 8);
        }
        lds_barrier();  // B
      }
      while (s_prev < p.s_end) end_sweep(s_prev++);

      // write back
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
      __builtin_amdgcn_s_setprio(0);
    } else if (STAGER && w == 1) {
      // ================= staging wave.  Blocks 0 and 1 before the loop; then
      // block o + 2 goes out right after B(o), when its buffers are free, and
      // has landed by B(o + 1): a whole block's time for the loads.
      int s2 = cs, q2 = cq;  // the last block sent
      if (nact > 0) {
        stage_table(cq, 0);
        stage_uniforms(cs, cq, 0);
      }
      if (nact > 1) {
        step_block(1, s2, q2);
        stage_table(q2, 1);
        stage_uniforms(s2, q2, 1);
      }
      drain();
      for (int co = 0; co < nact; ++co) {
        lds_barrier();  // A
        drain();
        lds_barrier();  // B
        if (co + 2 < nact) {
          step_block(co + 2, s2, q2);
          stage_table(q2, co & 1);
          stage_uniforms(s2, q2, co & 1);
        }
      }
    } else {
      // ================= streaming waves: the block's fields and couplings
      const int ws = w - W0;
      const int lane = lane_id();
      const int g = lane >> 4, j = lane & 15;
      // producer: the wave's slot words of the current block, one round (D
      // words, one scalar load) at a time; a block's slots are whole rounds
      BProd pr{};
      auto setup_block = [&]() {
        const uint2 h = sHdr[pr.q][ws];
        pr.off = __builtin_amdgcn_readfirstlane(h.x);
        const unsigned cnt = __builtin_amdgcn_readfirstlane(h.y);
        pr.pe = (int)(cnt >> 16);
        pr.padded = (int)(cnt & 0xFFFFu);
        pr.k = 0;
      };
      // the producer enters its next active block (only between rounds)
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
      unsigned wd[D];  // slot words of the round being issued
      // (branch-free: a branch here leaves the compiler's counted waits for
      // the ring's loads imprecise, and every round would drain the ring)
      auto fetch = [&]() {
        const bool past = pr.ord >= nact;  // past the last block: end slots
        typedef const __attribute__((address_space(4))) u4* ConstU4;
        const ConstU4 sp = (ConstU4)(I.sched + (past ? 0u : pr.off + (unsigned)pr.k));
        const u4 a = sp[0], b = sp[1];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          wd[d] = past ? kSlotEnd : a[d];
          wd[4 + d] = past ? kSlotEnd : b[d];
        }
      };
      // tiles and run words through buffer resources: the slot's offset is
      // a scalar, the lane's part a constant register (reads past the end
      // return zero)
      const __amdgpu_buffer_rsrc_t tiles_rs = __builtin_amdgcn_make_buffer_rsrc(
          uniform_ptr(I.tiles), 0, (int)__builtin_amdgcn_readfirstlane(I.n_tiles * (unsigned)TB), kBufferFlags);
      const __amdgpu_buffer_rsrc_t runs_rs = __builtin_amdgcn_make_buffer_rsrc(
          uniform_ptr(I.runs), 0, __builtin_amdgcn_readfirstlane(I.n_chunks * RPC * 8), kBufferFlags);
      auto issue = [&](BSlot<P>& sl, unsigned word) {
        const unsigned tix = word & 0xFFFFFu;  // tile (chunk + 1; 0 = the zero tile)
        sl.kind = (int)((word >> 20) & 3u);
        sl.tgt = (int)(word >> 22);
        sl.ord = 2 * pr.ord + (pr.k >= pr.pe ? 1 : 0);  // (block, part)
        ++pr.k;
        const int toff = __builtin_amdgcn_readfirstlane((int)(tix * (unsigned)TB));
        const int roff = __builtin_amdgcn_readfirstlane((int)((tix ? tix - 1u : 0u) * (unsigned)(RPC * 8)));
        if constexpr (P == P_FP32) {
#pragma unroll
          for (int q = 0; q < 2; ++q)
            sl.b.v[q] = __builtin_bit_cast(u4, __builtin_amdgcn_raw_buffer_load_b128(tiles_rs, lane * 32 + 16 * q, toff, 0));
        } else {
#pragma unroll
          for (int q = 0; q < PT<P>::NLD; ++q)
            sl.b.v[q] = __builtin_bit_cast(u4, __builtin_amdgcn_raw_buffer_load_b128(tiles_rs, q * 1024 + lane * 16, toff, 0));
        }
        sl.d = __builtin_amdgcn_raw_buffer_load_b32(runs_rs, g * 8, roff, 0);
      };

      pr.ord = 0;
      pr.s = cs;
      pr.q = cq;
      if (nact > 0) setup_block();
      BSlot<P> ring[D];
      fetch();
      // the priming loads stay in slot order: the loop's counted waits are
      // merged with this entry state, so a reordered priming would make
      // every round wait for all of its loads
#pragma unroll
      for (int d = 0; d < D; ++d) {
        issue(ring[d], wd[d]);
        __builtin_amdgcn_sched_barrier(0);
      }

      AccT<P> acc;
      acc_zero<P>(acc);
      const unsigned char* rb = &sbT[0][j];
      // one round of D slots: the operand of slot d + 1 is generated before
      // the matrix-core work of slot d, so its LDS reads overlap that work
      auto round = [&](float* myG) {
        advance();
        fetch();
        auto gen = [&](const BSlot<P>& sl) {
          // every slot's registers are consumed on every path (padding slots
          // multiply a zero operand), so the counted waits stay exact
          const unsigned m1 = run_mask1(sl.d, rb);
          const unsigned msk = sl.kind <= 1 ? m1 : 0u;
          AOp<P> a;
          if constexpr (P == P_FP32) {
            a.v = u4{msk, 0u, 0u, 0u};
          } else {
            const unsigned long long lo = sNib[msk & 15u], hi = sNib[msk >> 4];
            a.v = u4{(unsigned)lo, (unsigned)(lo >> 32), (unsigned)hi, (unsigned)(hi >> 32)};
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
          if (sl.kind == 1) {  // the chunk closes its list: fields [rep][sub][i], pairs [rep][a][b]
            if (sl.tgt == 0) {
#pragma unroll
              for (int r = 0; r < 4; ++r) myG[16 * r] = acc.v[r];
            } else {
              const unsigned ab = sPC[16 * (sl.tgt - 1) + j];
              float* dst = &sH[4 * g * kHRep + (ab >> 8) * 16 + (ab & 0xFFu)];
              float* dsu = &sH[4 * g * kHRep + (ab & 0xFFu) * 16 + (ab >> 8)];  // the symmetric entry
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                dst[kHRep * r] = acc.v[r];
                dsu[kHRep * r] = acc.v[r];
              }
            }
            acc_zero<P>(acc);
          }
          issue(sl, wd[d]);
        }
      };
      for (int co = 0; co < nact; ++co) {
        if (co > 0) step_block(co, cs, cq);
        // this lane's field outputs in the block's buffer, rebuilt from the
        // lane id every block (kept live across the block loop, the address
        // would be spilled, and reloading it would drain the load ring)
        const int ln = lane_id();
        float* myG = &sG[co & 1][ws][0][0] + (ln >> 4) * 64 + 4 * (ln & 3) + ((ln >> 2) & 3);
        // ---- early part: field chunks that read no bit of the block before,
        // while that block's decisions are taken (whole rounds per part)
        while (ring[0].ord == 2 * co) round(myG);
        if (co > 0) lds_barrier();  // B of the block before
        // ---- late part: the other field chunks and the pair tiles
        while (ring[0].ord == 2 * co + 1) round(myG);
        lds_barrier();  // A
      }
      if (nact > 0) lds_barrier();  // B of the last block
    }
  }
}

// one precision's launcher (each defined in the build of that precision)
template <int P> int launch_anneal_block_p(const AnnealParams& ap, int nw, int nblk, hipStream_t st);

template <int P, int NW>
static void launch_block_t(const AnnealParams& ap, int nblk, hipStream_t st) {
  TimedLaunch tl(0, st);
  hipLaunchKernelGGL((anneal_block_kernel<P, NW>), dim3((unsigned)nblk), dim3(64 * NW), 0, st, ap);
}

#ifdef HOBO_BLOCK_PREC
// this translation unit instantiates one precision's kernels (the file is
// compiled once per precision of the blocked annealer, so they build in parallel)
template <>
int launch_anneal_block_p<HOBO_BLOCK_PREC>(const AnnealParams& ap, int nw, int nblk, hipStream_t st) {
  switch (nw) {
    case 2: launch_block_t<HOBO_BLOCK_PREC, 2>(ap, nblk, st); return 0;
    case 4: launch_block_t<HOBO_BLOCK_PREC, 4>(ap, nblk, st); return 0;
    case 8: launch_block_t<HOBO_BLOCK_PREC, 8>(ap, nblk, st); return 0;
    case 16: launch_block_t<HOBO_BLOCK_PREC, 16>(ap, nblk, st); return 0;
    default: return -1;
  }
}
#else
int launch_anneal_block(const AnnealParams& ap, int prec, int nw, int nblk, hipStream_t st) {
  switch (prec) {
    case P_FP32: return launch_anneal_block_p<P_FP32>(ap, nw, nblk, st);
    case P_BF16X2: return launch_anneal_block_p<P_BF16X2>(ap, nw, nblk, st);
    case P_BF16X3: return launch_anneal_block_p<P_BF16X3>(ap, nw, nblk, st);
    case P_FP16X2: return launch_anneal_block_p<P_FP16X2>(ap, nw, nblk, st);
    default: return -1;
  }
}

// -log(u) of every (replica, sweep, bit) of a blocked launch window, one
// work-group per (sweep, 16-replica item): thread (q, rep, grp) draws the
// four Philox words of bits 16q + 4 grp .. +3 (counter: replica, sweep,
// 4q + grp, tag 0) and stores them at [item][sweep][q][rep][bit].
__global__ __launch_bounds__(256) void anneal_uniforms_kernel(AnnealParams p) {
  const int sr = blockIdx.y;
  const int s = p.s_begin + sr;
  for (int it = blockIdx.x; it < p.n_items; it += gridDim.x) {
    const AnnealItem item = p.items[it];
    const AnnealInstDev* I = p.insts + item.inst;
    const int NB = I->nblocks;
    const unsigned long long inst_id = I->inst_id;
    double* dst = I->unif + ((size_t)item.tile16 * p.unif_sweeps + sr) * ((size_t)NB * 256);
    const long long r0 = (long long)item.tile16 * 16;
    for (int u = threadIdx.x; u < NB * 64; u += blockDim.x) {
      const int q = u >> 6, rep = (u >> 2) & 15, grp = u & 3;
      const U64x4 o = philox((unsigned long long)(r0 + rep), (unsigned long long)s, (unsigned long long)(4 * q + grp),
                             0ull, p.seed, inst_id);
      double v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const double uu = (double)(o.w[e] >> 11) * 0x1.0p-53;
        v[e] = uu > 0.0 ? -log(uu) : INFINITY;
      }
      double* d = dst + q * 256 + rep * 16 + 4 * grp;
      *reinterpret_cast<d2*>(d) = d2{v[0], v[1]};
      *reinterpret_cast<d2*>(d + 2) = d2{v[2], v[3]};
    }
  }
}

void launch_anneal_uniforms(const AnnealParams& ap, hipStream_t st) {
  const unsigned gx = (unsigned)(ap.n_items < 4096 ? ap.n_items : 4096);
  hipLaunchKernelGGL(anneal_uniforms_kernel, dim3(gx, (unsigned)(ap.s_end - ap.s_begin)), dim3(256), 0, st, ap);
}

int anneal_mask_window() { return kMaskWin; }
int anneal_sweep_window() { return kSweepWin; }
#endif  // HOBO_BLOCK_PREC

}  // namespace hobo
