// Host-side canonicalisation of a raw HOBO term list (HOBOTAN Sec. II.B, III.C):
// every term is a coefficient on a product of binary variables; because
// x_i^2 = x_i for binary x, a term's index multiset reduces to a set, terms
// with equal sets are summed, the empty set is the constant offset, and zero
// sums are dropped.  The order k of the instance is the largest set size.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <unordered_map>
#include <utility>

#include "hobo_internal.h"
#include "../../include/hobo.h"

namespace hobo {

namespace {

// Exact sum of doubles, rounded once to the nearest double (ties to even).
// Every finite double is an integer multiple of 2^-1074, so the sum is kept
// as one wide two's-complement integer in units of 2^-1074 (a Kulisch-style
// long accumulator: 2098 bits cover the whole double range, the rest is
// headroom for carries of up to 2^60 terms).  Duplicate monomials and the
// constant terms go through it, so their sums do not depend on term order.
class ExactSum {
 public:
  static constexpr int kLimbs = 35;  // 2240 bits
  ExactSum() { std::memset(l_, 0, sizeof(l_)); }
  void add(double d) {
    if (d == 0.0) return;
    int e = 0;
    const double m = std::frexp(std::fabs(d), &e);        // |d| = m 2^e, 0.5 <= m < 1
    uint64_t M = (uint64_t)std::ldexp(m, 53);              // 53-bit integer significand
    int sh = e - 53 + 1074;                                 // |d| = M 2^(sh - 1074)
    if (sh < 0) {                                           // subnormal: M has trailing zeros
      M >>= -sh;
      sh = 0;
    }
    const int q = sh >> 6, b = sh & 63;
    const uint64_t lo = M << b, hi = b ? (M >> (64 - b)) : 0;
    if (d > 0)
      add_at(q, lo, hi);
    else
      sub_at(q, lo, hi);
  }
  // nearest double of the exact sum (+-inf if it is out of range)
  double value() const {
    uint64_t v[kLimbs];
    std::memcpy(v, l_, sizeof(v));
    const bool neg = (v[kLimbs - 1] >> 63) != 0;
    if (neg) {  // two's-complement magnitude
      unsigned carry = 1;
      for (int i = 0; i < kLimbs; ++i) {
        const uint64_t x = ~v[i] + carry;
        carry = (carry && x == 0) ? 1u : 0u;
        v[i] = x;
      }
    }
    int top = -1;  // highest set bit
    for (int i = kLimbs - 1; i >= 0 && top < 0; --i)
      if (v[i]) top = 64 * i + 63 - __builtin_clzll(v[i]);
    if (top < 0) return 0.0;
    auto bit = [&](int p) { return (int)((v[p >> 6] >> (p & 63)) & 1u); };
    double r;
    if (top < 53) {  // exact: fewer than 54 significant bits
      uint64_t x = v[0];
      r = std::ldexp((double)x, -1074);
    } else {
      const int cut = top - 52;  // bits below `cut` are rounded off
      uint64_t q = 0;
      for (int p = top; p >= cut; --p) q = (q << 1) | (uint64_t)bit(p);
      const int half = bit(cut - 1);
      bool sticky = false;  // any set bit below the half-way bit
      for (int p = 0; p <= cut - 2 && !sticky; ++p) sticky = bit(p) != 0;
      if (half && (sticky || (q & 1u))) ++q;
      r = std::ldexp((double)q, cut - 1074);
    }
    return neg ? -r : r;
  }

 private:
  void add_at(int q, uint64_t lo, uint64_t hi) {
    unsigned __int128 c = (unsigned __int128)l_[q] + lo;
    l_[q] = (uint64_t)c;
    c = (unsigned __int128)l_[q + 1] + hi + (uint64_t)(c >> 64);
    l_[q + 1] = (uint64_t)c;
    uint64_t carry = (uint64_t)(c >> 64);
    for (int i = q + 2; carry && i < kLimbs; ++i) carry = (++l_[i] == 0) ? 1u : 0u;
  }
  void sub_at(int q, uint64_t lo, uint64_t hi) {
    uint64_t borrow = l_[q] < lo ? 1u : 0u;
    l_[q] -= lo;
    const unsigned __int128 need = (unsigned __int128)hi + borrow;
    borrow = (unsigned __int128)l_[q + 1] < need ? 1u : 0u;
    l_[q + 1] -= (uint64_t)need;
    for (int i = q + 2; borrow && i < kLimbs; ++i) borrow = (l_[i]-- == 0) ? 1u : 0u;
  }
  uint64_t l_[kLimbs];
};

}  // namespace

int canonicalize(int n_vars, int max_order, int64_t n_terms, const int64_t* term_ptr,
                 const int32_t* term_idx, const void* coeff, int coeff_type, Tensor* t,
                 std::string* err) {
  const bool integer = coeff_type == HOBO_COEFF_INT64;
  const int64_t* ci = static_cast<const int64_t*>(coeff);
  const double* cf = static_cast<const double*>(coeff);

  std::unordered_map<std::string, size_t> where;
  std::vector<std::string> keys;
  std::vector<int64_t> acc_i;
  std::vector<double> acc_f;  // real: the first value of each monomial
  std::vector<std::pair<size_t, double>> dup_f;  // real: further values (slot, value)
  int64_t off_i = 0;
  ExactSum off_f;
  std::vector<int> buf;
  for (int64_t term = 0; term < n_terms; ++term) {
    int64_t a = term_ptr[term], b = term_ptr[term + 1];
    buf.assign(term_idx + a, term_idx + b);
    std::sort(buf.begin(), buf.end());
    buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
    if ((int)buf.size() > kMaxOrder) {
      *err = "term " + std::to_string(term) + " has " + std::to_string(buf.size()) +
             " distinct variables; at most " + std::to_string(kMaxOrder) + " are supported";
      return HOBO_ERR_ORDER;
    }
    if (integer) {
      if (!std::isfinite((double)ci[term])) return HOBO_ERR_INVALID_ARG;
    } else if (!std::isfinite(cf[term])) {
      *err = "coefficient of term " + std::to_string(term) + " is not finite";
      return HOBO_ERR_INVALID_ARG;
    }
    if (buf.empty()) {
      if (integer) {
        if (__builtin_add_overflow(off_i, ci[term], &off_i)) {
          *err = "integer offset overflows int64";
          return HOBO_ERR_RANGE;
        }
      } else {
        off_f.add(cf[term]);
      }
      continue;
    }
    std::string key(buf.size(), '\0');
    for (size_t j = 0; j < buf.size(); ++j) key[j] = (char)(uint8_t)buf[j];
    auto it = where.find(key);
    size_t slot;
    const bool fresh = it == where.end();
    if (fresh) {
      slot = keys.size();
      where.emplace(key, slot);
      keys.push_back(key);
      acc_i.push_back(0);
      acc_f.push_back(0.0);
    } else {
      slot = it->second;
    }
    if (integer) {
      if (__builtin_add_overflow(acc_i[slot], ci[term], &acc_i[slot])) {
        *err = "integer coefficient sum overflows int64";
        return HOBO_ERR_RANGE;
      }
    } else if (fresh) {
      acc_f[slot] = cf[term];
    } else {
      dup_f.emplace_back(slot, cf[term]);
    }
  }
  // duplicate real monomials: the exact sum of all their values, rounded once
  if (!dup_f.empty()) {
    std::stable_sort(dup_f.begin(), dup_f.end(),
                     [](const std::pair<size_t, double>& a, const std::pair<size_t, double>& b) {
                       return a.first < b.first;
                     });
    for (size_t i = 0; i < dup_f.size();) {
      const size_t slot = dup_f[i].first;
      ExactSum es;
      es.add(acc_f[slot]);
      for (; i < dup_f.size() && dup_f[i].first == slot; ++i) es.add(dup_f[i].second);
      acc_f[slot] = es.value();
      if (!std::isfinite(acc_f[slot])) {
        *err = "a real coefficient sum overflows double";
        return HOBO_ERR_RANGE;
      }
    }
  }
  // keep non-zero monomials, ordered by (size, lexicographic)
  std::vector<size_t> order;
  for (size_t s = 0; s < keys.size(); ++s)
    if (integer ? acc_i[s] != 0 : acc_f[s] != 0.0) order.push_back(s);
  std::sort(order.begin(), order.end(), [&](size_t x, size_t y) {
    if (keys[x].size() != keys[y].size()) return keys[x].size() < keys[y].size();
    return std::memcmp(keys[x].data(), keys[y].data(), keys[x].size()) < 0;
  });
  int k = 0;
  for (size_t s : order) k = std::max<int>(k, (int)keys[s].size());
  if (max_order > 0 && k > max_order) {
    *err = "instance has order " + std::to_string(k) + " > max_order " + std::to_string(max_order);
    return HOBO_ERR_ORDER;
  }
  t->n_vars = n_vars;
  t->order = k;
  t->integer = integer;
  t->mono_ptr.assign(1, 0);
  t->mono_idx.clear();
  t->w_i.clear();
  t->w_f.clear();
  t->n_per_order.assign((size_t)k + 1, 0);
  t->abs_sum = 0;
  t->var_abs_max = 0;
  t->w_lo = t->w_hi = 0;
  t->row_norm.assign((size_t)n_vars, 0.0);
  std::vector<unsigned __int128> var_abs(integer ? (size_t)n_vars : 0, 0);
  for (size_t s : order) {
    const std::string& key = keys[s];
    for (char c : key) t->mono_idx.push_back((uint8_t)c);
    t->mono_ptr.push_back((int64_t)t->mono_idx.size());
    double w = integer ? (double)acc_i[s] : acc_f[s];
    t->w_i.push_back(integer ? acc_i[s] : 0);
    t->w_f.push_back(w);
    t->n_per_order[key.size()]++;
    if (integer) {
      const __int128 v = acc_i[s];
      t->abs_sum += (unsigned __int128)(v < 0 ? -v : v);
      for (char c : key) var_abs[(uint8_t)c] += (unsigned __int128)(v < 0 ? -v : v);
      t->w_lo = std::min(t->w_lo, acc_i[s]);
      t->w_hi = std::max(t->w_hi, acc_i[s]);
    }
    for (char c : key) t->row_norm[(uint8_t)c] += w * w;
  }
  for (const auto& v : var_abs) t->var_abs_max = std::max(t->var_abs_max, v);
  t->row_norm_max = 0.0;
  for (auto& v : t->row_norm) {
    v = std::sqrt(v);
    t->row_norm_max = std::max(t->row_norm_max, v);
  }
  t->offset_i = off_i;
  const double off_real = off_f.value();
  if (!integer && !std::isfinite(off_real)) {
    *err = "the constant offset overflows double";
    return HOBO_ERR_RANGE;
  }
  t->offset_f = integer ? (double)off_i : off_real;
  return HOBO_OK;
}

}  // namespace hobo
