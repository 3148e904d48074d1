// Host-side driver for the address / undefined-behaviour sanitizer build of
// the library's host code: the canonicaliser, the result aggregation and the
// tensor-train decomposition, on seeded random inputs (repeated variables,
// duplicate and cancelling terms, empty terms, real and integer
// coefficients).  Built with g++ only (no device code): the device
// destructors the linked files need are defined here as no-ops, since no
// device memory is ever allocated.
#include <cstdint>
#include <cstdio>
#include <memory>
#include <random>
#include <string>
#include <vector>

#include "hobo_internal.h"

namespace hobo {
Packed::~Packed() {}
TermsDev::~TermsDev() {}
GDDev::~GDDev() {}
BlockSchedule::~BlockSchedule() {}
Tensor::~Tensor() {}
}  // namespace hobo

extern "C" hipError_t hipFree(void*) { return hipSuccess; }
extern "C" hipError_t hipMalloc(void** p, size_t) {
  *p = nullptr;
  return hipErrorOutOfMemory;
}
extern "C" hipError_t hipMemcpy(void*, const void*, size_t, hipMemcpyKind) { return hipErrorInvalidValue; }
extern "C" hipError_t hipGetLastError() { return hipSuccess; }

int main() {
  std::mt19937_64 rng(7);
  int failures = 0;
  for (int trial = 0; trial < 200; ++trial) {
    const int n = 1 + (int)(rng() % 20), k = 1 + (int)(rng() % 5);
    const int64_t nt = (int64_t)(rng() % 300);
    std::vector<int64_t> ptr{0};
    std::vector<int32_t> idx;
    std::vector<int64_t> ci;
    std::vector<double> cf;
    for (int64_t t = 0; t < nt; ++t) {
      const int len = (int)(rng() % (k + 1));  // 0 = constant
      for (int q = 0; q < len; ++q) idx.push_back((int32_t)(rng() % n));  // repeats allowed
      ptr.push_back((int64_t)idx.size());
      ci.push_back((int64_t)(rng() % 17) - 8);
      cf.push_back((double)((int64_t)(rng() % 2001) - 1000) / 64.0);
    }
    const bool integer = trial % 2 == 0;
    hobo::Tensor t;
    std::string err;
    int st = hobo::canonicalize(n, 0, nt, ptr.data(), idx.data(), integer ? (const void*)ci.data() : (const void*)cf.data(),
                                integer ? 0 : 1, &t, &err);
    if (st != 0) {
      std::printf("canonicalize failed: %s\n", err.c_str());
      ++failures;
      continue;
    }
    // result aggregation over a batch with repeats
    const int64_t B = 1 + (int64_t)(rng() % 500);
    const int W = (n + 63) / 64;
    std::vector<uint64_t> bits((size_t)W * B);
    std::vector<int64_t> ei((size_t)B);
    for (int64_t b = 0; b < B; ++b) {
      const uint64_t v = rng() % 7;  // few distinct states
      bits[(size_t)b] = v & ((n >= 64) ? ~0ull : ((1ull << n) - 1ull));
      ei[(size_t)b] = (int64_t)bits[(size_t)b] * 3 - 5;
    }
    int64_t nu = 0;
    std::vector<int64_t> rep((size_t)B), cnt((size_t)B);
    if (hobo::aggregate_states(n, B, bits.data(), ei.data(), 1, &nu, rep.data(), cnt.data(), &err) != 0) ++failures;
    // TT decomposition of the dense tensor (small cases)
    if (t.n_mono() > 0 && n <= 8) {
      std::unique_ptr<hobo::TTDev> tt;
      st = hobo::tt_decompose(&t, &tt, &err);
      if (st != 0 && st != 8) {  // 8: a rank beyond the kernel limit is a refusal, not an error
        std::printf("tt_decompose failed: %s\n", err.c_str());
        ++failures;
      }
    }
  }
  std::printf("host driver: %d failures\n", failures);
  return failures ? 1 : 0;
}
