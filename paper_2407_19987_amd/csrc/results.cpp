// Result aggregation of a sampling run (the unique states of a batch with
// their energies and occurrence counts, ordered by energy): the host-side
// step after hobo_anneal_batch that turns `shots` replicas into the result
// list the paper prints for each worked problem (Sec. V).
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "hobo_internal.h"
#include "../../include/hobo.h"

namespace hobo {

int aggregate_states(int n_vars, int64_t B, const uint64_t* x_bits, const void* energies, int is_integer,
                     int64_t* n_unique, int64_t* rep_out, int64_t* count_out, std::string* err) {
  const int W = (n_vars + 63) / 64;
  // energies as exact keys: int64, or the double's bits mapped to an
  // order-preserving unsigned integer (NaN is refused)
  std::vector<uint64_t> ekey((size_t)B);
  for (int64_t b = 0; b < B; ++b) {
    if (is_integer) {
      const int64_t v = static_cast<const int64_t*>(energies)[b];
      ekey[(size_t)b] = (uint64_t)v ^ 0x8000000000000000ull;
    } else {
      const double d = static_cast<const double*>(energies)[b];
      if (d != d) {
        *err = "energy " + std::to_string(b) + " is NaN";
        return HOBO_ERR_INVALID_ARG;
      }
      uint64_t u;
      std::memcpy(&u, &d, 8);
      if (u == 0x8000000000000000ull) u = 0;  // -0.0 sorts with +0.0
      ekey[(size_t)b] = (u >> 63) ? ~u : (u | 0x8000000000000000ull);
    }
  }
  // the bit vector as a sequence x_0, x_1, ... compared lexicographically:
  // within a word the lowest variable is the least significant bit, so the
  // word is compared with its bits reversed
  auto rev = [](uint64_t v) {
    v = ((v >> 1) & 0x5555555555555555ull) | ((v & 0x5555555555555555ull) << 1);
    v = ((v >> 2) & 0x3333333333333333ull) | ((v & 0x3333333333333333ull) << 2);
    v = ((v >> 4) & 0x0F0F0F0F0F0F0F0Full) | ((v & 0x0F0F0F0F0F0F0F0Full) << 4);
    v = ((v >> 8) & 0x00FF00FF00FF00FFull) | ((v & 0x00FF00FF00FF00FFull) << 8);
    v = ((v >> 16) & 0x0000FFFF0000FFFFull) | ((v & 0x0000FFFF0000FFFFull) << 16);
    return (v >> 32) | (v << 32);
  };
  std::vector<uint64_t> key((size_t)B * (size_t)W);
  for (int64_t b = 0; b < B; ++b)
    for (int w = 0; w < W; ++w) key[(size_t)b * W + w] = rev(x_bits[(size_t)w * (size_t)B + (size_t)b]);
  std::vector<int64_t> ord((size_t)B);
  std::iota(ord.begin(), ord.end(), 0);
  auto less = [&](int64_t a, int64_t b) {
    if (ekey[(size_t)a] != ekey[(size_t)b]) return ekey[(size_t)a] < ekey[(size_t)b];
    for (int w = 0; w < W; ++w) {
      const uint64_t ka = key[(size_t)a * W + w], kb = key[(size_t)b * W + w];
      if (ka != kb) return ka < kb;
    }
    return a < b;  // the first replica of a state represents it
  };
  std::sort(ord.begin(), ord.end(), less);
  auto same_state = [&](int64_t a, int64_t b) {
    for (int w = 0; w < W; ++w)
      if (key[(size_t)a * W + w] != key[(size_t)b * W + w]) return false;
    return true;
  };
  int64_t u = 0;
  for (int64_t p = 0; p < B;) {
    int64_t q = p + 1;
    while (q < B && ekey[(size_t)ord[(size_t)p]] == ekey[(size_t)ord[(size_t)q]] &&
           same_state(ord[(size_t)p], ord[(size_t)q]))
      ++q;
    rep_out[u] = ord[(size_t)p];
    count_out[u] = q - p;
    ++u;
    p = q;
  }
  *n_unique = u;
  return HOBO_OK;
}

}  // namespace hobo
