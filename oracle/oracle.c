/*
 * CPU oracle for the HOBO energy / single-flip / Metropolis hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously-correct C.  It shares no
 * code with the GPU library and is never linked into it; only the tests, the
 * smoke check and the benchmark's CPU-baseline leg load it.
 *
 * Every instance is a canonical monomial list (sorted, distinct variables per
 * monomial, constant term removed) in CSR form:
 *   monomial m has variables mono_idx[mono_ptr[m] .. mono_ptr[m+1]) and
 *   coefficient coeff[m].
 * Coefficients arrive as int64 fixed-point numbers together with a binary
 * scale `s`: the real coefficient is coeff[m] * 2^-s (s = 0 for integer
 * instances).  All sums are then exact in __int128 and a real result is
 * rounded once, at the end, to the nearest double.
 *
 * Bit vectors arrive word-major, [W][B] uint64: variable i of row b is bit
 * (i & 63) of word bits[(i >> 6) * B + b].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;
typedef unsigned __int128 u128;

static inline int bit_of(const uint64_t* bits, int64_t B, int64_t b, int i) {
  return (int)((bits[(int64_t)(i >> 6) * B + b] >> (i & 63)) & 1u);
}

static void row_to_bytes(const uint64_t* bits, int64_t B, int64_t b, int n, unsigned char* x) {
  for (int i = 0; i < n; ++i) x[i] = (unsigned char)bit_of(bits, B, b, i);
}

/* Round an exact fixed-point value acc * 2^-s to the nearest double. */
static double fixed_to_double(i128 acc, int s) {
  /* (double) of an __int128 rounds to nearest (libgcc); ldexp is exact here
   * because |acc| * 2^-s stays far from the subnormal range for the
   * coefficient magnitudes this oracle accepts. */
  return ldexp((double)acc, -s);
}

/* ---------------------------------------------------------------------- *
 * Energy, by definition: E(x) = sum_S w_S prod_{i in S} x_i
 * (the paper's Sec. II.B polynomial; the constant is excluded, it is the
 * offset returned with the tensor).
 * ---------------------------------------------------------------------- */
static i128 energy_row(int n_mono, const int64_t* mono_ptr, const int32_t* mono_idx,
                       const int64_t* coeff, const unsigned char* x) {
  i128 acc = 0;
  for (int m = 0; m < n_mono; ++m) {
    int on = 1;
    for (int64_t p = mono_ptr[m]; p < mono_ptr[m + 1]; ++p)
      if (!x[mono_idx[p]]) { on = 0; break; }
    if (on) acc += (i128)coeff[m];
  }
  return acc;
}

/* out_i64 (if non-null) receives exact integers (requires s == 0 and range);
 * out_f64 (if non-null) receives the correctly rounded real value. */
int orc_energy(int n_vars, int n_mono, const int64_t* mono_ptr, const int32_t* mono_idx,
               const int64_t* coeff, int s, int64_t B, const uint64_t* bits,
               int64_t* out_i64, double* out_f64) {
  int overflow = 0;
#pragma omp parallel for schedule(static) reduction(| : overflow)
  for (int64_t b = 0; b < B; ++b) {
    unsigned char x[4096];
    row_to_bytes(bits, B, b, n_vars, x);
    i128 e = energy_row(n_mono, mono_ptr, mono_idx, coeff, x);
    if (out_i64) {
      if (e > (i128)INT64_MAX || e < (i128)INT64_MIN) overflow = 1;
      out_i64[b] = (int64_t)e;
    }
    if (out_f64) out_f64[b] = fixed_to_double(e, s);
  }
  return overflow ? -1 : 0;
}

/* ---------------------------------------------------------------------- *
 * Local fields and single-flip changes, by definition:
 *   g_i(x)  = sum_{S containing i} w_S prod_{j in S, j != i} x_j
 *   dE_i(x) = E(x with bit i flipped) - E(x) = (1 - 2 x_i) g_i(x)
 * (the multilinear polynomial is affine in each x_i with slope g_i).
 * ---------------------------------------------------------------------- */
int orc_fields(int n_vars, int n_mono, const int64_t* mono_ptr, const int32_t* mono_idx,
               const int64_t* coeff, int s, int64_t B, const uint64_t* bits,
               int64_t* g_i64, double* g_f64, int64_t* de_i64, double* de_f64) {
  int overflow = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(| : overflow)
  for (int64_t b = 0; b < B; ++b) {
    unsigned char x[4096];
    i128* g = (i128*)calloc((size_t)n_vars, sizeof(i128));
    row_to_bytes(bits, B, b, n_vars, x);
    for (int m = 0; m < n_mono; ++m) {
      for (int64_t p = mono_ptr[m]; p < mono_ptr[m + 1]; ++p) {
        int i = mono_idx[p];
        int on = 1;
        for (int64_t q = mono_ptr[m]; q < mono_ptr[m + 1]; ++q)
          if (q != p && !x[mono_idx[q]]) { on = 0; break; }
        if (on) g[i] += (i128)coeff[m];
      }
    }
    for (int i = 0; i < n_vars; ++i) {
      i128 de = x[i] ? -g[i] : g[i];
      if (g_i64) {
        if (g[i] > (i128)INT64_MAX || g[i] < (i128)INT64_MIN) overflow = 1;
        g_i64[b * n_vars + i] = (int64_t)g[i];
      }
      if (de_i64) de_i64[b * n_vars + i] = (int64_t)de;
      if (g_f64) g_f64[b * n_vars + i] = fixed_to_double(g[i], s);
      if (de_f64) de_f64[b * n_vars + i] = fixed_to_double(de, s);
    }
    free(g);
  }
  return overflow ? -1 : 0;
}

/* ---------------------------------------------------------------------- *
 * Exhaustive minimisation over all 2^n states (n <= 30), visiting them in
 * reflected Gray-code order so that consecutive states differ in one bit;
 * the energy is carried exactly from one state to the next by dE_i above.
 * Writes the minimum (fixed point), the number of minimisers, and up to
 * `cap` minimising states as integers (bit i = variable i).
 * ---------------------------------------------------------------------- */
int orc_brute_force(int n_vars, int n_mono, const int64_t* mono_ptr, const int32_t* mono_idx,
                    const int64_t* coeff, int64_t* min_hi, uint64_t* min_lo, int64_t* n_min,
                    uint64_t* argmins, int64_t cap) {
  if (n_vars > 30) return -1;
  /* incidence lists: monomials containing each variable */
  int64_t* cnt = (int64_t*)calloc((size_t)n_vars + 1, sizeof(int64_t));
  for (int m = 0; m < n_mono; ++m)
    for (int64_t p = mono_ptr[m]; p < mono_ptr[m + 1]; ++p) cnt[mono_idx[p] + 1]++;
  for (int i = 0; i < n_vars; ++i) cnt[i + 1] += cnt[i];
  int* inc = (int*)malloc(sizeof(int) * (size_t)(cnt[n_vars] + 1));
  int64_t* fill = (int64_t*)calloc((size_t)n_vars, sizeof(int64_t));
  for (int m = 0; m < n_mono; ++m)
    for (int64_t p = mono_ptr[m]; p < mono_ptr[m + 1]; ++p) {
      int i = mono_idx[p];
      inc[cnt[i] + fill[i]++] = m;
    }
  unsigned char x[64];
  memset(x, 0, sizeof(x));
  i128 e = 0; /* E(0) = 0: every monomial has at least one variable */
  i128 best = e;
  int64_t nbest = 1;
  uint64_t state = 0;
  if (cap > 0) argmins[0] = 0;
  uint64_t total = 1ull << n_vars;
  for (uint64_t t = 1; t < total; ++t) {
    int i = __builtin_ctzll(t); /* Gray code: bit flipped at step t */
    i128 g = 0;
    for (int64_t a = cnt[i]; a < cnt[i + 1]; ++a) {
      int m = inc[a];
      int on = 1;
      for (int64_t q = mono_ptr[m]; q < mono_ptr[m + 1]; ++q)
        if (mono_idx[q] != i && !x[mono_idx[q]]) { on = 0; break; }
      if (on) g += (i128)coeff[m];
    }
    e += x[i] ? -g : g;
    x[i] ^= 1;
    state ^= 1ull << i;
    if (e < best) {
      best = e;
      nbest = 0;
    }
    if (e == best) {
      if (nbest < cap) argmins[nbest] = state;
      nbest++;
    }
  }
  *min_hi = (int64_t)(best >> 64);
  *min_lo = (uint64_t)best;
  *n_min = nbest;
  free(cnt);
  free(inc);
  free(fill);
  return 0;
}

/* ---------------------------------------------------------------------- *
 * Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
 * 64x64->128 multiplications (multipliers M0, M1), a word permutation and a
 * key XOR, with the two key words bumped by the Weyl constants W0, W1
 * between rounds.
 * ---------------------------------------------------------------------- */
#define PHILOX_M0 0xD2E7470EE14C6C93ull
#define PHILOX_M1 0xCA5A826395121157ull
#define PHILOX_W0 0x9E3779B97F4A7C15ull
#define PHILOX_W1 0xBB67AE8584CAA73Bull

void orc_philox4x64(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]) {
  uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint64_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    u128 p0 = (u128)PHILOX_M0 * c0;
    u128 p1 = (u128)PHILOX_M1 * c2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n1 = lo1;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    uint64_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* uniform double in [0, 1) from the top 53 bits of a 64-bit word */
static inline double u01(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }

/* Random word for (replica b, sweep s, variable i, stream tag):
 * counter (b, s, i / 4, tag), key (seed, instance), word i % 4. */
static inline uint64_t draw(uint64_t seed, uint64_t inst, uint64_t b, uint64_t s, int i, uint64_t tag) {
  uint64_t c[4] = {b, s, (uint64_t)(i >> 2), tag}, k[2] = {seed, inst}, o[4];
  orc_philox4x64(c, k, o);
  return o[i & 3];
}

/* ---------------------------------------------------------------------- *
 * Batched single-flip Metropolis simulated annealing (the paper's
 * Sec. II.D.1 search, with the schedule, scan order and acceptance rule the
 * paper leaves open fixed as follows):
 *   - temperatures temps[s], one per sweep (the caller passes the schedule);
 *   - a sweep visits variables 0, 1, ..., n-1 in order;
 *   - visiting i: dE = (1 - 2 x_i) g_i(x), exact; accept iff dE <= 0 or
 *     u < exp(-dE * beta) with beta = 1 / T and u from draw(seed, inst, b,
 *     s, i, 0), all in double precision; on acceptance flip x_i and add dE
 *     to E;
 *   - initial state: given, or bit i = top bit of draw(seed, inst, b, 0, i, 1);
 *   - best state: the initial one, then after every sweep the current state
 *     if its energy is strictly lower.
 * Learned-proposal gating (attempt masks): if `attempt` is non-null it holds,
 * per (replica group of 16, sweep, variable), 0/1 whether the variable is
 * visited in that sweep by that group; skipped variables are not drawn for.
 * Outputs: final bits, best bits, exact best energies (fixed point),
 * per-sweep trace of min over replicas of the best energy (double).
 * Optional margin_out [B][S]: for replica b and sweep s, the smallest over
 * the sweep's decisions of |dE beta + ln u| / (beta A), where A is the sum of
 * |w_S| over the monomials S containing i whose other variables are set (so
 * that |dE| <= A).  The acceptance test is dE beta < -ln u (for dE <= 0 it
 * always holds), so any evaluation of dE whose error stays below that
 * fraction of A takes the same decision.  +inf when A = 0 or u = 0.
 * ---------------------------------------------------------------------- */
int orc_anneal(int n_vars, int n_mono, const int64_t* mono_ptr, const int32_t* mono_idx,
               const int64_t* coeff, int s_scale, int64_t B, int S, const double* temps,
               uint64_t seed, uint64_t inst, int init_given, uint64_t* bits_inout,
               uint64_t* best_bits_out, int64_t* best_hi, uint64_t* best_lo, double* trace_out,
               const unsigned char* attempt, int64_t* n_accept_out, int s0, double* margin_out) {
  if (n_vars > 4096) return -1;
  int64_t* cnt = (int64_t*)calloc((size_t)n_vars + 1, sizeof(int64_t));
  for (int m = 0; m < n_mono; ++m)
    for (int64_t p = mono_ptr[m]; p < mono_ptr[m + 1]; ++p) cnt[mono_idx[p] + 1]++;
  for (int i = 0; i < n_vars; ++i) cnt[i + 1] += cnt[i];
  int* inc = (int*)malloc(sizeof(int) * (size_t)(cnt[n_vars] + 1));
  int64_t* fill = (int64_t*)calloc((size_t)n_vars, sizeof(int64_t));
  for (int m = 0; m < n_mono; ++m)
    for (int64_t p = mono_ptr[m]; p < mono_ptr[m + 1]; ++p) {
      int i = mono_idx[p];
      inc[cnt[i] + fill[i]++] = m;
    }
  double* tr = (double*)malloc(sizeof(double) * (size_t)(S > 0 ? S : 1) * (size_t)(B > 0 ? B : 1));
  int W = (n_vars + 63) / 64;
  int64_t total_acc = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total_acc)
  for (int64_t b = 0; b < B; ++b) {
    unsigned char x[4096], bx[4096];
    if (init_given) {
      row_to_bytes(bits_inout, B, b, n_vars, x);
    } else {
      for (int i = 0; i < n_vars; ++i) x[i] = (unsigned char)(draw(seed, inst, (uint64_t)b, 0, i, 1) >> 63);
    }
    i128 e = energy_row(n_mono, mono_ptr, mono_idx, coeff, x);
    i128 best = e;
    memcpy(bx, x, (size_t)n_vars);
    for (int s = 0; s < S; ++s) {
      double beta = 1.0 / temps[s]; /* inverse temperature of this sweep */
      double mmin = INFINITY;
      for (int i = 0; i < n_vars; ++i) {
        if (attempt && !attempt[((size_t)(b / 16) * (size_t)S + (size_t)s) * (size_t)n_vars + (size_t)i]) continue;
        i128 g = 0, ga = 0;
        for (int64_t a = cnt[i]; a < cnt[i + 1]; ++a) {
          int m = inc[a];
          int on = 1;
          for (int64_t q = mono_ptr[m]; q < mono_ptr[m + 1]; ++q)
            if (mono_idx[q] != i && !x[mono_idx[q]]) { on = 0; break; }
          if (on) {
            g += (i128)coeff[m];
            ga += (i128)(coeff[m] < 0 ? -coeff[m] : coeff[m]);
          }
        }
        i128 de = x[i] ? -g : g;
        double ded = fixed_to_double(de, s_scale);
        double u = u01(draw(seed, inst, (uint64_t)b, (uint64_t)(s0 + s), i, 0));
        if (margin_out && ga != 0 && u > 0.0) {
          double m = fabs(ded * beta + log(u)) / (beta * fixed_to_double(ga, s_scale));
          if (m < mmin) mmin = m;
        }
        if (ded <= 0.0 || u < exp(-ded * beta)) {
          x[i] ^= 1;
          e += de;
          total_acc++;
        }
      }
      if (margin_out) margin_out[(size_t)b * (size_t)S + (size_t)s] = mmin;
      if (e < best) {
        best = e;
        memcpy(bx, x, (size_t)n_vars);
      }
      tr[(size_t)b * (size_t)S + (size_t)s] = fixed_to_double(best, s_scale);
    }
    for (int w = 0; w < W; ++w) {
      uint64_t v = 0, bv = 0;
      for (int i = 64 * w; i < n_vars && i < 64 * (w + 1); ++i) {
        v |= (uint64_t)x[i] << (i & 63);
        bv |= (uint64_t)bx[i] << (i & 63);
      }
      bits_inout[(int64_t)w * B + b] = v;
      best_bits_out[(int64_t)w * B + b] = bv;
    }
    best_hi[b] = (int64_t)(best >> 64);
    best_lo[b] = (uint64_t)best;
  }
  if (trace_out) {
    for (int s = 0; s < S; ++s) {
      double mn = INFINITY;
      for (int64_t b = 0; b < B; ++b) {
        double v = tr[(size_t)b * (size_t)S + (size_t)s];
        if (v < mn) mn = v;
      }
      trace_out[s] = mn;
    }
  }
  if (n_accept_out) *n_accept_out = total_acc;
  free(tr);
  free(cnt);
  free(inc);
  free(fill);
  return 0;
}

/* Number of OpenMP threads the oracle will use (1 without OpenMP). */
int orc_num_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the following oracle calls (timing on one core or on all). */
void orc_set_threads(int n) {
#ifdef _OPENMP
  extern void omp_set_num_threads(int);
  omp_set_num_threads(n > 0 ? n : 1);
#else
  (void)n;
#endif
}
