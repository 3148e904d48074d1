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

#include "hobo_internal.h"
#include "../../include/hobo.h"

namespace hobo {

int canonicalize(int n_vars, int max_order, int64_t n_terms, const int64_t* term_ptr,
                 const int32_t* term_idx, const void* coeff, int coeff_type, Tensor* t,
                 std::string* err) {
  const bool integer = coeff_type == HOBO_COEFF_INT64;
  const int64_t* ci = static_cast<const int64_t*>(coeff);
  const double* cf = static_cast<const double*>(coeff);

  std::unordered_map<std::string, size_t> where;
  std::vector<std::string> keys;
  std::vector<int64_t> acc_i;
  std::vector<double> acc_f;
  int64_t off_i = 0;
  double off_f = 0.0;
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
        off_f += cf[term];
      }
      continue;
    }
    std::string key(buf.size(), '\0');
    for (size_t j = 0; j < buf.size(); ++j) key[j] = (char)(uint8_t)buf[j];
    auto it = where.find(key);
    size_t slot;
    if (it == where.end()) {
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
    } else {
      acc_f[slot] += cf[term];
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
  t->row_norm.assign((size_t)n_vars, 0.0);
  for (size_t s : order) {
    const std::string& key = keys[s];
    for (char c : key) t->mono_idx.push_back((uint8_t)c);
    t->mono_ptr.push_back((int64_t)t->mono_idx.size());
    double w = integer ? (double)acc_i[s] : acc_f[s];
    t->w_i.push_back(integer ? acc_i[s] : 0);
    t->w_f.push_back(w);
    t->n_per_order[key.size()]++;
    for (char c : key) t->row_norm[(uint8_t)c] += w * w;
  }
  t->row_norm_max = 0.0;
  for (auto& v : t->row_norm) {
    v = std::sqrt(v);
    t->row_norm_max = std::max(t->row_norm_max, v);
  }
  t->offset_i = off_i;
  t->offset_f = integer ? (double)off_i : off_f;
  return HOBO_OK;
}

}  // namespace hobo
