// Gradient-descent search (Sec. II.D.2): the per-variable record lists of
// the gradient kernel, built on the host from the canonical monomials, and
// the C-ABI calls hobo_gd_gradient / hobo_gd_batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "hobo_internal.h"
#include "../../include/hobo.h"

namespace hobo {

GDDev::~GDDev() {
  if (d_ptr) (void)hipFree(d_ptr);
  if (d_rec) (void)hipFree(d_rec);
}

int get_gd(Tensor* t, GDDev** out, std::string* err) {
  std::lock_guard<std::mutex> lock(t->mu);
  if (t->gd) {
    *out = t->gd.get();
    return HOBO_OK;
  }
  const int n = t->n_vars, nm = t->n_mono();
  std::vector<int32_t> ptr((size_t)n + 1, 0);
  for (int m = 0; m < nm; ++m)
    for (int64_t q = t->mono_ptr[m]; q < t->mono_ptr[m + 1]; ++q) ptr[(size_t)t->mono_idx[q] + 1]++;
  for (int i = 0; i < n; ++i) ptr[(size_t)i + 1] += ptr[(size_t)i];
  std::vector<GDRec> rec((size_t)ptr[(size_t)n]);
  std::vector<int32_t> fill((size_t)n, 0);
  for (int m = 0; m < nm; ++m) {  // monomial order within every variable's list
    const uint8_t* s = t->mono_idx.data() + t->mono_ptr[m];
    const int len = (int)(t->mono_ptr[m + 1] - t->mono_ptr[m]);
    for (int a = 0; a < len; ++a) {
      GDRec r{};
      r.w = t->w_f[m];
      for (int b = 0; b < len; ++b)
        if (b != a) r.o[r.n++] = s[b];
      const int i = s[a];
      rec[(size_t)(ptr[(size_t)i] + fill[(size_t)i]++)] = r;
    }
  }
  std::unique_ptr<GDDev> gd(new GDDev());
  gd->n_vars = n;
  auto up = [&](const void* src, size_t bytes, void** dst) -> int {
    if (hipMalloc(dst, std::max<size_t>(bytes, 16)) != hipSuccess) {
      (void)hipGetLastError();
      *err = "hipMalloc of the gradient records failed";
      return HOBO_ERR_OOM;
    }
    if (bytes && hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) {
      *err = "hipMemcpy of the gradient records failed";
      return HOBO_ERR_HIP;
    }
    gd->bytes += bytes;
    return HOBO_OK;
  };
  if (int s = up(ptr.data(), ptr.size() * sizeof(int32_t), reinterpret_cast<void**>(&gd->d_ptr))) return s;
  if (int s = up(rec.data(), rec.size() * sizeof(GDRec), reinterpret_cast<void**>(&gd->d_rec))) return s;
  *out = gd.get();
  t->gd = std::move(gd);
  return HOBO_OK;
}

}  // namespace hobo
