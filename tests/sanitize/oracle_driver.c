/* Driver for the address / undefined-behaviour sanitizer build of the CPU
 * oracle (oracle/oracle.c): energies, fields, brute force and the annealer
 * with decision margins on a seeded random order-3 instance. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_energy(int, int, const int64_t*, const int32_t*, const int64_t*, int, int64_t, const uint64_t*, int64_t*,
               double*);
int orc_fields(int, int, const int64_t*, const int32_t*, const int64_t*, int, int64_t, const uint64_t*, int64_t*,
               double*, int64_t*, double*);
int orc_brute_force(int, int, const int64_t*, const int32_t*, const int64_t*, int64_t*, uint64_t*, int64_t*, uint64_t*,
                    int64_t);
int orc_anneal(int, int, const int64_t*, const int32_t*, const int64_t*, int, int64_t, int, const double*, uint64_t,
               uint64_t, int, uint64_t*, uint64_t*, int64_t*, uint64_t*, double*, const unsigned char*, int64_t*, int,
               double*);

static uint64_t st = 88172645463325252ull;
static uint64_t nxt(void) {
  st ^= st << 13;
  st ^= st >> 7;
  st ^= st << 17;
  return st;
}

int main(void) {
  enum { N = 12, B = 40, S = 6 };
  int64_t ptr[600];
  int32_t idx[1800];
  int64_t co[600];
  int nm = 0, ni = 0;
  ptr[0] = 0;
  for (int a = 0; a < N; ++a)
    for (int b = a; b < N; ++b)
      for (int c = b; c < N; ++c) {
        if (nxt() % 3) continue;
        idx[ni++] = a;
        if (b > a) idx[ni++] = b;
        if (c > b) idx[ni++] = c;
        co[nm] = (int64_t)(nxt() % 11) - 5;
        ptr[++nm] = ni;
      }
  uint64_t bits[B], best[B];
  for (int b = 0; b < B; ++b) bits[b] = nxt() & ((1ull << N) - 1);
  int64_t e[B], g[B * N], de[B * N], bh[B];
  uint64_t bl[B], args[64];
  double ef[B], trace[S], margin[B * S], temps[S];
  int rc = 0;
  rc |= orc_energy(N, nm, ptr, idx, co, 0, B, bits, e, ef);
  rc |= orc_fields(N, nm, ptr, idx, co, 0, B, bits, g, NULL, de, NULL);
  int64_t mh, nmin;
  uint64_t ml;
  rc |= orc_brute_force(N, nm, ptr, idx, co, &mh, &ml, &nmin, args, 64);
  for (int s = 0; s < S; ++s) temps[s] = 3.0 / (1 + s);
  int64_t acc;
  rc |= orc_anneal(N, nm, ptr, idx, co, 0, B, S, temps, 5, 0, 1, bits, best, bh, bl, trace, NULL, &acc, 0, margin);
  printf("oracle driver: rc %d, %d monomials, min %lld (%lld minimisers), %lld accepts\n", rc, nm, (long long)ml,
         (long long)nmin, (long long)acc);
  return rc != 0;
}
