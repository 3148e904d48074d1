// C-ABI entry points of the HOBO engine (declared in include/hobo.h).
// Every argument is checked on the host before any HIP call; failures return
// a status code and leave a thread-local message for hobo_last_error().
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <iterator>
#include <list>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hobo_internal.h"
#include "../../include/hobo.h"

struct hobo_tensor {
  hobo::Tensor t;
};

namespace {

thread_local std::string g_err;

hobo_status fail(hobo_status code, const std::string& msg) {
  g_err = msg;
  return code;
}
hobo_status ok() { return HOBO_OK; }

hobo_status hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return HOBO_OK;
  (void)hipGetLastError();
  return fail(e == hipErrorOutOfMemory ? HOBO_ERR_OOM : HOBO_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

hobo_status need_device() {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return fail(HOBO_ERR_NO_DEVICE, "no HIP device available");
  }
  return HOBO_OK;
}

// inverse temperature of sweep s of an L-sweep geometric schedule,
// T_s = T_0 (T_end / T_0)^(s / (L - 1)) (Sec. II.D.1 reading), beta_s = 1 / T_s
// The blocked annealer completes a field from the couplings (sum_b x_b H_ab
// over the block, with the block's triples counted twice and taken back
// once), so its FP32 partial sums reach up to three times the variable's
// sum |w|: integer fields stay exact while that is below 2^24.
bool blocked_exact(const hobo::Tensor& t) {
  return !t.integer || t.var_abs_max * 3 < ((unsigned __int128)1 << 24);
}

double schedule_beta(double t_start, double t_end, int64_t s, int64_t L) {
  const double T = L == 1 ? t_start : t_start * std::pow(t_end / t_start, (double)s / (double)(L - 1));
  return 1.0 / T;
}

bool valid_prec(int p) { return p >= HOBO_PREC_FP32 && p <= HOBO_PREC_FP16X2; }

// Tile shape of the evaluation kernels: 16*rt replicas x 16*ct columns per
// wave.  Narrower column groups give more waves when B is small.
int tuned_shape(const hobo::Tensor& t, int kernel, int prec, int64_t B) {
  std::lock_guard<std::mutex> lock(const_cast<hobo::Tensor&>(t).mu);
  auto it = t.tuned.find(hobo::tune_key(kernel, prec, B));
  return it == t.tuned.end() ? 0 : it->second;
}

void eval_shape(const hobo::Tensor& t, int prec, int64_t B, int* rt, int* ct, int kernel = 0) {
  if (kernel) {
    if (int sh = tuned_shape(t, kernel, prec, B)) {
      *rt = sh >> 4;
      *ct = sh & 15;
      return;
    }
  }
  int T = (t.n_vars + 15) / 16;
  int c = 1;
  while (c < T && c < 8) c *= 2;
  if (prec == HOBO_PREC_INT8X4 && c > 4) c = 4;
  auto waves = [&](int cc, int rr) { return ((B + 16 * rr - 1) / (16 * rr)) * ((T + cc - 1) / cc); };
  while (c > 1 && waves(c, 1) < 1024) c /= 2;
  // The energy contraction gains from several row tiles per wave once the
  // grid is full; the fields contraction keeps one per-bit accumulator per
  // row tile and loses more to register pressure than it gains in reuse.
  int r = 1;
  if (kernel != hobo::TK_FIELDS) r = waves(c, 4) >= 2048 ? 4 : (waves(c, 2) >= 2048 ? 2 : 1);
  if (r == 4 && c > 4) c = 4;
  const char* env_rt = std::getenv("HOBO_EVAL_RT");
  const char* env_ct = std::getenv("HOBO_EVAL_CT");
  if (env_rt) {
    int v = std::atoi(env_rt);
    r = v >= 4 ? 4 : (v >= 2 ? 2 : 1);
  }
  if (r == 4 && c > 4) c = 4;
  if (env_ct) {
    int v = std::atoi(env_ct);
    c = v >= 8 ? 8 : v >= 4 ? 4 : v >= 2 ? 2 : 1;
    if (prec == HOBO_PREC_INT8X4 && c > 4) c = 4;
  }
  if (r == 4 && c > 4) c = 4;  // instantiated shapes: rt 4 with up to 4 column tiles
  *rt = r;
  *ct = c;
}

hobo_status check_bits_args(const hobo_tensor* t, const void* x_bits, int64_t B, int32_t precision) {
  if (!t) return fail(HOBO_ERR_INVALID_ARG, "tensor is NULL");
  if (!x_bits) return fail(HOBO_ERR_INVALID_ARG, "x_bits is NULL");
  if (B < 1) return fail(HOBO_ERR_INVALID_ARG, "B must be >= 1");
  if (B > (int64_t)1 << 40) return fail(HOBO_ERR_INVALID_ARG, "B too large");
  if (!valid_prec(precision)) return fail(HOBO_ERR_INVALID_ARG, "unknown precision");
  if (precision == HOBO_PREC_INT8X4 && !t->t.integer)
    return fail(HOBO_ERR_PRECISION, "INT8X4 precision needs an integer tensor");
  if (precision != HOBO_PREC_FP64) {
    std::string err;
    if (int s = hobo::check_prec(&t->t, precision, &err)) return fail(s, err);
  }
  return HOBO_OK;
}

// ------------------------------------------------------------ graph cache
// Annealing setups (device tables, workspace, captured graph) are cached by
// their full argument list, so repeated identical calls only enqueue kernels
// (or launch the graph).  Entries that name a tensor die with it.
// At most kAnnealKeep setups are kept, and the older ones together hold at
// most kAnnealKeepBytes of workspace (calls that differ only in the seed each
// make a setup).
constexpr size_t kAnnealKeep = 16;
constexpr size_t kAnnealKeepBytes = (size_t)4 << 30;
struct AnnealEntry {
  std::vector<uint64_t> key;
  int32_t mode = 0;
  void* work = nullptr;
  size_t bytes = 0;  // workspace size
  hobo::AnnealTables tb;
  std::vector<hobo::AnnealPlan> plans;  // PERSISTENT / GRAPH: one plan; PER_INSTANCE: one per instance
  hipGraphExec_t exec = nullptr;
  // LEARNED proposal: per-instance fields layout, row norms and workspaces
  struct Learn {
    hobo::Packed* fields = nullptr;
    const hobo::Tensor* t = nullptr;
    const double* rnorm = nullptr;
    void* de = nullptr;
    unsigned char* mask = nullptr;
    const uint64_t* x = nullptr;
    int64_t B = 0;
    int rt = 1, ct = 1;
  };
  std::vector<Learn> learn;
  std::vector<double> beta;  // inverse temperatures of the call's sweeps
  int refresh = 0;
  const float* mlp = nullptr;
  float lthr = 0.0f;
  double p_floor = 0.0;
  int precision = 0;
};

// The whole sequence of one plan; with the LEARNED proposal every `refresh`
// sweeps the fields of the current states feed the network and the next
// segment's attempt masks.
int enqueue_plan(const AnnealEntry& e, const hobo::AnnealPlan& pl, void* stream, std::string* err) {
  if (e.refresh == 0) return hobo::enqueue_anneal_seq(e.tb, pl, stream, err);
  if (int s = hobo::enqueue_anneal_setup(e.tb, pl, stream, err)) return s;
  const int s_end = pl.s_first + pl.sweeps;
  if (pl.sweeps == 0) {
    if (int s = hobo::enqueue_anneal_sweeps(e.tb, pl, pl.s_first, pl.s_first, pl.s_first, 0, pl.cont, stream, err))
      return s;
  }
  for (int s0 = pl.s_first; s0 < s_end; s0 += e.refresh) {
    const int len = std::min(e.refresh, s_end - s0);
    const double beta0 = e.beta[(size_t)(s0 - pl.s_first)];
    for (int j = pl.inst0; j < pl.inst0 + pl.ninst; ++j) {
      const AnnealEntry::Learn& L = e.learn[(size_t)j];
      hobo::EvalArgs a{L.fields, L.t, L.x, L.B, L.de, nullptr, nullptr, L.rt, L.ct, stream};
      if (int s = hobo::launch_eval(a, err)) return s;
      if (int s = hobo::proposal_masks(e.mlp, reinterpret_cast<const unsigned long long*>(L.x), L.B, L.t->n_vars,
                                       L.de, L.t->integer ? 1 : 0, beta0, L.rnorm, e.lthr, e.p_floor, pl.seed,
                                       (unsigned long long)j, s0, len, L.mask, (hipStream_t)stream, err))
        return s;
    }
    if (int s = hobo::enqueue_anneal_sweeps(e.tb, pl, s0, s0 + len, s0, len, pl.cont || s0 > pl.s_first, stream,
                                            err))
      return s;
  }
  return hobo::enqueue_anneal_finish(e.tb, pl, stream, err);
}
std::mutex g_anneal_mu;
std::list<AnnealEntry> g_anneal;  // most recent first

void release_entry(AnnealEntry& e) {
  (void)hipDeviceSynchronize();
  if (e.exec) (void)hipGraphExecDestroy(e.exec);
  if (e.work) (void)hipFree(e.work);
  e.exec = nullptr;
  e.work = nullptr;
}

}  // namespace

extern "C" {

const char* hobo_last_error(void) { return g_err.c_str(); }

hobo_status hobo_timing_enable(int32_t enable) {
  g_err.clear();
  hobo::timing_enable(enable);
  return ok();
}

hobo_status hobo_timing_read(int32_t kernel, double* total_ms, int64_t* launches) {
  g_err.clear();
  if (!total_ms || !launches) return fail(HOBO_ERR_INVALID_ARG, "NULL argument");
  if (kernel < 0 || kernel > 2) return fail(HOBO_ERR_INVALID_ARG, "kernel id must be 0, 1 or 2");
  if (int s = hobo::timing_read(kernel, total_ms, launches)) return fail(s, "event timing failed");
  return ok();
}
const char* hobo_version(void) { return "hobo-mi355x 0.1 (gfx950)"; }

hobo_status hobo_build_tensor(int32_t n_vars, int32_t max_order, int64_t n_terms, const int64_t* term_ptr,
                              const int32_t* term_idx, const void* coeff, int32_t coeff_type, hobo_tensor** out,
                              void* offset_out) {
  g_err.clear();
  if (!out) return fail(HOBO_ERR_INVALID_ARG, "out is NULL");
  if (n_vars < 1 || n_vars > hobo::kMaxVars)
    return fail(HOBO_ERR_INVALID_ARG, "n_vars must be in [1, 256]");
  if (max_order < 0) return fail(HOBO_ERR_INVALID_ARG, "max_order must be >= 0");
  if (n_terms < 0) return fail(HOBO_ERR_INVALID_ARG, "n_terms must be >= 0");
  if (coeff_type != HOBO_COEFF_INT64 && coeff_type != HOBO_COEFF_F64)
    return fail(HOBO_ERR_INVALID_ARG, "unknown coeff_type");
  if (!term_ptr) return fail(HOBO_ERR_INVALID_ARG, "term_ptr is NULL");
  if (n_terms > 0 && !coeff) return fail(HOBO_ERR_INVALID_ARG, "coeff is NULL");
  if (term_ptr[0] != 0) return fail(HOBO_ERR_INVALID_ARG, "term_ptr[0] must be 0");
  for (int64_t i = 0; i < n_terms; ++i)
    if (term_ptr[i + 1] < term_ptr[i]) return fail(HOBO_ERR_INVALID_ARG, "term_ptr must be non-decreasing");
  const int64_t nnz = term_ptr[n_terms];
  if (nnz > 0 && !term_idx) return fail(HOBO_ERR_INVALID_ARG, "term_idx is NULL");
  for (int64_t p = 0; p < nnz; ++p)
    if (term_idx[p] < 0 || term_idx[p] >= n_vars)
      return fail(HOBO_ERR_INVALID_ARG, "variable index " + std::to_string(term_idx[p]) + " outside [0, n_vars)");
  if (coeff_type == HOBO_COEFF_F64) {
    const double* c = static_cast<const double*>(coeff);
    for (int64_t i = 0; i < n_terms; ++i)
      if (!std::isfinite(c[i])) return fail(HOBO_ERR_INVALID_ARG, "non-finite coefficient");
  }
  hobo_tensor* h = new (std::nothrow) hobo_tensor();
  if (!h) return fail(HOBO_ERR_OOM, "host allocation failed");
  std::string err;
  int st = hobo::canonicalize(n_vars, max_order, n_terms, term_ptr, term_idx, coeff, coeff_type, &h->t, &err);
  if (st != HOBO_OK) {
    delete h;
    return fail(st, err);
  }
  int dev = -1;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) {
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
  }
  (void)hipGetLastError();
  h->t.device = dev;
  if (offset_out) {
    if (h->t.integer)
      *static_cast<int64_t*>(offset_out) = h->t.offset_i;
    else
      *static_cast<double*>(offset_out) = h->t.offset_f;
  }
  *out = h;
  return ok();
}

hobo_status hobo_free_tensor(hobo_tensor* t) {
  g_err.clear();
  if (!t) return ok();
  {
    std::lock_guard<std::mutex> lock(g_anneal_mu);
    for (auto it = g_anneal.begin(); it != g_anneal.end();) {
      bool uses = false;
      for (auto v : it->key) uses = uses || v == (uint64_t)(uintptr_t)t;
      if (uses) {
        release_entry(*it);
        it = g_anneal.erase(it);
      } else {
        ++it;
      }
    }
  }
  delete t;
  return ok();
}

hobo_status hobo_tensor_info_get(const hobo_tensor* t, hobo_tensor_info* info) {
  g_err.clear();
  if (!t || !info) return fail(HOBO_ERR_INVALID_ARG, "NULL argument");
  std::memset(info, 0, sizeof(*info));
  info->n_vars = t->t.n_vars;
  info->order = t->t.order;
  info->is_integer = t->t.integer ? 1 : 0;
  info->n_monomials = t->t.n_mono();
  for (size_t r = 0; r < t->t.n_per_order.size() && r < 8; ++r) info->n_per_order[r] = t->t.n_per_order[r];
  info->offset_i64 = t->t.offset_i;
  info->offset_f64 = t->t.offset_f;
  int64_t bytes = 0;
  hobo_tensor* tm = const_cast<hobo_tensor*>(t);
  {
    std::lock_guard<std::mutex> lock(tm->t.mu);
    for (auto& kv : tm->t.packed) bytes += (int64_t)kv.second->bytes;
    if (tm->t.terms) bytes += (int64_t)tm->t.terms->bytes;
  }
  info->device_bytes = bytes;
  return ok();
}

hobo_status hobo_tensor_monomials(const hobo_tensor* t, int64_t* mono_ptr, int64_t ptr_cap, int32_t* mono_idx,
                                  int64_t idx_cap, void* weights, int64_t w_cap) {
  g_err.clear();
  if (!t) return fail(HOBO_ERR_INVALID_ARG, "tensor is NULL");
  const hobo::Tensor& T = t->t;
  const int64_t nm = T.n_mono();
  if (mono_ptr) {
    if (ptr_cap < nm + 1) return fail(HOBO_ERR_INVALID_ARG, "mono_ptr capacity too small");
    for (int64_t m = 0; m <= nm; ++m) mono_ptr[m] = T.mono_ptr[(size_t)m];
  }
  if (mono_idx) {
    if (idx_cap < (int64_t)T.mono_idx.size()) return fail(HOBO_ERR_INVALID_ARG, "mono_idx capacity too small");
    for (size_t p = 0; p < T.mono_idx.size(); ++p) mono_idx[p] = T.mono_idx[p];
  }
  if (weights) {
    if (w_cap < nm) return fail(HOBO_ERR_INVALID_ARG, "weights capacity too small");
    for (int64_t m = 0; m < nm; ++m) {
      if (T.integer)
        static_cast<int64_t*>(weights)[m] = T.w_i[(size_t)m];
      else
        static_cast<double*>(weights)[m] = T.w_f[(size_t)m];
    }
  }
  return ok();
}

hobo_status hobo_tensor_export_dense(const hobo_tensor* t, void* host_out, int64_t capacity) {
  g_err.clear();
  if (!t || !host_out) return fail(HOBO_ERR_INVALID_ARG, "NULL argument");
  const hobo::Tensor& T = t->t;
  const int k = std::max(T.order, 1);
  double total = std::pow((double)T.n_vars, (double)k);
  if (total > (double)(1 << 26)) return fail(HOBO_ERR_INVALID_ARG, "N^k exceeds 2^26");
  int64_t n = (int64_t)total;
  if (capacity < n) return fail(HOBO_ERR_INVALID_ARG, "capacity smaller than N^k");
  if (T.integer)
    std::memset(host_out, 0, (size_t)n * sizeof(int64_t));
  else
    std::memset(host_out, 0, (size_t)n * sizeof(double));
  for (int m = 0; m < T.n_mono(); ++m) {
    const uint8_t* s = T.mono_idx.data() + T.mono_ptr[(size_t)m];
    int len = (int)(T.mono_ptr[(size_t)m + 1] - T.mono_ptr[(size_t)m]);
    // the smallest variable fills the leading k - len + 1 slots (Sec. III.C)
    int64_t flat = 0;
    for (int q = 0; q < k; ++q) {
      int v = q < k - len ? s[0] : s[q - (k - len)];
      flat = flat * T.n_vars + v;
    }
    if (T.integer)
      static_cast<int64_t*>(host_out)[flat] = T.w_i[(size_t)m];
    else
      static_cast<double*>(host_out)[flat] = T.w_f[(size_t)m];
  }
  return ok();
}

hobo_status hobo_tensor_layout_info(hobo_tensor* t, int32_t fn, int32_t precision, hobo_layout_info* out) {
  g_err.clear();
  if (!t || !out) return fail(HOBO_ERR_INVALID_ARG, "NULL argument");
  if (fn != 1 && fn != 2 && fn != 4) return fail(HOBO_ERR_INVALID_ARG, "fn must be 1, 2 or 4");
  if (!hobo::tiled_prec(precision)) return fail(HOBO_ERR_PRECISION, "no tiled layout for this precision");
  std::string err;
  if (int s = hobo::check_prec(&t->t, precision, &err)) return fail(s, err);
  if (t->t.n_mono() == 0) {
    std::memset(out, 0, sizeof(*out));
    return ok();
  }
  if (hobo_status s = need_device()) return s;
  int mode = fn == 1 ? hobo::M_ENERGY : fn == 2 ? hobo::M_FIELDS : hobo::M_SLABS;
  if (fn == 4 && t->t.order <= 3 && precision != HOBO_PREC_INT8X4 && blocked_exact(t->t)) mode = hobo::M_BLOCKS;
  hobo::Packed* pk;
  if (int s = hobo::get_packed(&t->t, mode, precision, &pk, &err)) return fail(s, err);
  const int64_t k_rows = precision == HOBO_PREC_INT8X4 ? 64 : 32;
  const int64_t passes = precision == HOBO_PREC_FP32 ? 1
                         : precision == HOBO_PREC_BF16X3 ? 3
                         : precision == HOBO_PREC_INT8X4 ? 4 : 2;
  out->chunks = pk->nchunks;
  out->tiles = pk->ntiles > 0 ? pk->ntiles - 1 : 0;
  out->issued_flops = out->tiles * 16 * k_rows * 2 * passes;
  out->bytes = (int64_t)pk->bytes;
  return ok();
}

hobo_status hobo_tensor_prepare(hobo_tensor* t, uint32_t fn_mask, uint32_t prec_mask) {
  g_err.clear();
  if (!t) return fail(HOBO_ERR_INVALID_ARG, "tensor is NULL");
  if (fn_mask & ~7u) return fail(HOBO_ERR_INVALID_ARG, "unknown function bits");
  if (prec_mask & ~63u) return fail(HOBO_ERR_INVALID_ARG, "unknown precision bits");
  for (int p = 0; p <= HOBO_PREC_FP16X2; ++p) {
    std::string e;
    if ((prec_mask & (1u << p)) && fn_mask && p != HOBO_PREC_FP64)
      if (int s = hobo::check_prec(&t->t, p, &e)) return fail(s, e);
  }
  if (hobo_status s = need_device()) return s;
  std::string err;
  for (int p = 0; p <= HOBO_PREC_FP16X2; ++p) {
    if (!(prec_mask & (1u << p))) continue;
    if (p == HOBO_PREC_INT8X4 && !t->t.integer) return fail(HOBO_ERR_PRECISION, "INT8X4 needs an integer tensor");
    if (p == HOBO_PREC_FP64) {
      hobo::TermsDev* td;
      if (int s = hobo::get_terms(&t->t, &td, &err)) return fail(s, err);
      continue;
    }
    hobo::Packed* pk;
    if (fn_mask & 1u)
      if (int s = hobo::get_packed(&t->t, hobo::M_ENERGY, p, &pk, &err)) return fail(s, err);
    if (fn_mask & 2u)
      if (int s = hobo::get_packed(&t->t, hobo::M_FIELDS, p, &pk, &err)) return fail(s, err);
    if (fn_mask & 4u) {
      if (int s = hobo::get_packed(&t->t, hobo::M_SLABS, p, &pk, &err)) return fail(s, err);
      if (t->t.order <= 3 && p != HOBO_PREC_INT8X4 && blocked_exact(t->t))
        if (int s = hobo::get_packed(&t->t, hobo::M_BLOCKS, p, &pk, &err)) return fail(s, err);
    }
  }
  if (fn_mask & 4u) {
    hobo::TermsDev* td;
    if (int s = hobo::get_terms(&t->t, &td, &err)) return fail(s, err);
  }
  return ok();
}

hobo_status hobo_energy(const hobo_tensor* tc, const uint64_t* x_bits, int64_t B, int32_t precision, void* e_out,
                        void* stream) {
  g_err.clear();
  if (hobo_status s = check_bits_args(tc, x_bits, B, precision)) return s;
  if (!e_out) return fail(HOBO_ERR_INVALID_ARG, "e_out is NULL");
  if (hobo_status s = need_device()) return s;
  hobo_tensor* t = const_cast<hobo_tensor*>(tc);
  std::string err;
  if (t->t.n_mono() == 0) {
    size_t bytes = (size_t)B * 8;
    return hip_status(hipMemsetAsync(e_out, 0, bytes, (hipStream_t)stream), "hipMemsetAsync");
  }
  if (precision == HOBO_PREC_FP64) {
    hobo::TermsDev* td;
    if (int s = hobo::get_terms(&t->t, &td, &err)) return fail(s, err);
    void* work = nullptr;
    if (hobo_status s = hip_status(hipMallocAsync(&work, hobo::term_workspace_bytes(&t->t, B), (hipStream_t)stream),
                                   "hipMallocAsync"))
      return s;
    hobo::TermArgs a{td, &t->t, x_bits, B, e_out, work, stream};
    int s = hobo::launch_term_energy(a, &err);
    (void)hipFreeAsync(work, (hipStream_t)stream);
    if (s) return fail(s, err);
    return ok();
  }
  hobo::Packed* pk;
  if (int s = hobo::get_packed(&t->t, hobo::M_ENERGY, precision, &pk, &err)) return fail(s, err);
  int rt, ct;
  eval_shape(t->t, precision, B, &rt, &ct, hobo::TK_ENERGY);
  size_t wb = hobo::eval_workspace_bytes(&t->t, hobo::M_ENERGY, B, ct);
  void* work = nullptr;
  if (wb) {
    if (hobo_status s = hip_status(hipMallocAsync(&work, wb, (hipStream_t)stream), "hipMallocAsync")) return s;
  }
  hobo::EvalArgs a{pk, &t->t, x_bits, B, nullptr, e_out, work, rt, ct, stream};
  int s = hobo::launch_eval(a, &err);
  if (work) (void)hipFreeAsync(work, (hipStream_t)stream);
  if (s) return fail(s, err);
  return ok();
}

hobo_status hobo_energy_noalloc(const hobo_tensor* tc, const uint64_t* x_bits, int64_t B, int32_t precision,
                                void* e_out, void* stream) {
  g_err.clear();
  if (hobo_status s = check_bits_args(tc, x_bits, B, precision)) return s;
  if (!e_out) return fail(HOBO_ERR_INVALID_ARG, "e_out is NULL");
  if (hobo_status s = need_device()) return s;
  hobo_tensor* t = const_cast<hobo_tensor*>(tc);
  std::string err;
  void* scratch = nullptr;
  if (int s = hobo::noalloc_scratch(&scratch, &err)) return fail(s, err);
  if (t->t.n_mono() == 0) {
    if (int s = hobo::launch_zero_u64(e_out, B, stream, &err)) return fail(s, err);
    return ok();
  }
  const size_t cap = hobo::kNoallocScratchBytes;
  if (precision == HOBO_PREC_FP64) {
    hobo::TermsDev* td = nullptr;
    {
      std::lock_guard<std::mutex> lock(t->t.mu);
      td = t->t.terms.get();
    }
    if (!td)
      return fail(HOBO_ERR_INVALID_ARG, "FP64 term list not on the device: call hobo_tensor_prepare(t, 1, 1 << FP64) first");
    const size_t need = hobo::term_workspace_bytes(&t->t, B);
    if (need > cap)
      return fail(HOBO_ERR_INVALID_ARG, "batch needs " + std::to_string(need) + " bytes of workspace; the no-allocation "
                  "scratch holds " + std::to_string(cap));
    hobo::TermArgs a{td, &t->t, x_bits, B, e_out, scratch, stream};
    if (int s = hobo::launch_term_energy(a, &err)) return fail(s, err);
    return ok();
  }
  hobo::Packed* pk = nullptr;
  {
    std::lock_guard<std::mutex> lock(t->t.mu);
    auto it = t->t.packed.find(hobo::M_ENERGY * 16 + precision);
    if (it != t->t.packed.end()) pk = it->second.get();
  }
  if (!pk)
    return fail(HOBO_ERR_INVALID_ARG, "energy layout of this precision not on the device: call "
                "hobo_tensor_prepare(t, 1, 1 << precision) first");
  int rt, ct;
  eval_shape(t->t, precision, B, &rt, &ct, hobo::TK_ENERGY);
  const size_t need = hobo::eval_workspace_bytes(&t->t, hobo::M_ENERGY, B, ct);
  if (need > cap)
    return fail(HOBO_ERR_INVALID_ARG, "batch needs " + std::to_string(need) + " bytes of workspace; the no-allocation "
                "scratch holds " + std::to_string(cap));
  hobo::EvalArgs a{pk, &t->t, x_bits, B, nullptr, e_out, need ? scratch : nullptr, rt, ct, stream};
  if (int s = hobo::launch_eval(a, &err)) return fail(s, err);
  return ok();
}

hobo_status hobo_local_fields(const hobo_tensor* tc, const uint64_t* x_bits, int64_t B, int32_t precision,
                              void* de_out, void* e_out, void* stream) {
  g_err.clear();
  if (hobo_status s = check_bits_args(tc, x_bits, B, precision)) return s;
  if (!de_out) return fail(HOBO_ERR_INVALID_ARG, "de_out is NULL");
  if (precision == HOBO_PREC_FP64)
    return fail(HOBO_ERR_PRECISION, "hobo_local_fields supports FP32, BF16X2, BF16X3, FP16X2 and INT8X4");
  if (hobo_status s = need_device()) return s;
  hobo_tensor* t = const_cast<hobo_tensor*>(tc);
  std::string err;
  if (t->t.n_mono() == 0) {
    size_t eb = t->t.integer ? 8 : 4;
    if (hobo_status s = hip_status(hipMemsetAsync(de_out, 0, (size_t)B * t->t.n_vars * eb, (hipStream_t)stream),
                                   "hipMemsetAsync"))
      return s;
    if (e_out) return hip_status(hipMemsetAsync(e_out, 0, (size_t)B * 8, (hipStream_t)stream), "hipMemsetAsync");
    return ok();
  }
  hobo::Packed* pk;
  if (int s = hobo::get_packed(&t->t, hobo::M_FIELDS, precision, &pk, &err)) return fail(s, err);
  int rt, ct;
  eval_shape(t->t, precision, B, &rt, &ct, hobo::TK_FIELDS);
  size_t wb = e_out ? hobo::eval_workspace_bytes(&t->t, hobo::M_FIELDS, B, ct) : 0;
  void* work = nullptr;
  if (wb) {
    if (hobo_status s = hip_status(hipMallocAsync(&work, wb, (hipStream_t)stream), "hipMallocAsync")) return s;
  }
  hobo::EvalArgs a{pk, &t->t, x_bits, B, de_out, e_out, work, rt, ct, stream};
  int s = hobo::launch_eval(a, &err);
  if (work) (void)hipFreeAsync(work, (hipStream_t)stream);
  if (s) return fail(s, err);
  return ok();
}

hobo_status hobo_anneal_batch(hobo_tensor* const* tensors, int32_t n_instances, const int64_t* replicas,
                              const hobo_anneal_params* params, uint64_t* x_inout, uint64_t* best_x_out,
                              void* best_e_out, double* trace_out, int32_t launch_mode, void* stream) {
  g_err.clear();
  if (!tensors || !replicas || !params || !x_inout || !best_x_out || !best_e_out)
    return fail(HOBO_ERR_INVALID_ARG, "NULL argument");
  if (n_instances < 1) return fail(HOBO_ERR_INVALID_ARG, "n_instances must be >= 1");
  const hobo_anneal_params& P = *params;
  if (P.sweeps < 0) return fail(HOBO_ERR_INVALID_ARG, "sweeps must be >= 0");
  const int64_t L = P.schedule_sweeps == 0 ? (int64_t)P.sweeps : (int64_t)P.schedule_sweeps;
  if (P.schedule_sweeps < 0 || P.first_sweep < 0) return fail(HOBO_ERR_INVALID_ARG, "negative sweep index");
  if (P.schedule_sweeps == 0 && P.first_sweep != 0)
    return fail(HOBO_ERR_INVALID_ARG, "first_sweep needs schedule_sweeps");
  if ((int64_t)P.first_sweep + P.sweeps > L) return fail(HOBO_ERR_INVALID_ARG, "sweeps run past the schedule");
  if (!(P.t_start > 0.0) || !(P.t_end > 0.0) || !std::isfinite(P.t_start) || !std::isfinite(P.t_end))
    return fail(HOBO_ERR_INVALID_ARG, "temperatures must be finite and > 0");
  if (P.init != HOBO_INIT_RANDOM && P.init != HOBO_INIT_GIVEN) return fail(HOBO_ERR_INVALID_ARG, "unknown init");
  if (P.continue_best != 0 && P.continue_best != 1) return fail(HOBO_ERR_INVALID_ARG, "continue_best must be 0 or 1");
  if (P.proposal != HOBO_PROPOSAL_METROPOLIS && P.proposal != HOBO_PROPOSAL_MASKED &&
      P.proposal != HOBO_PROPOSAL_LEARNED)
    return fail(HOBO_ERR_INVALID_ARG, "unknown proposal");
  if (P.proposal == HOBO_PROPOSAL_MASKED && !P.attempt)
    return fail(HOBO_ERR_INVALID_ARG, "MASKED proposal needs attempt masks");
  if (P.proposal == HOBO_PROPOSAL_LEARNED) {
    if (!P.mlp) return fail(HOBO_ERR_INVALID_ARG, "LEARNED proposal needs network weights");
    if (P.refresh < 1) return fail(HOBO_ERR_INVALID_ARG, "refresh must be >= 1");
    if (!(P.p_floor >= 0.0f && P.p_floor <= 1.0f)) return fail(HOBO_ERR_INVALID_ARG, "p_floor must be in [0, 1]");
    if (std::isnan(P.tau)) return fail(HOBO_ERR_INVALID_ARG, "tau is NaN");
  }
  if (!hobo::tiled_prec(P.precision))
    return fail(HOBO_ERR_PRECISION, "annealing precision must be FP32, BF16X2, BF16X3, FP16X2 or INT8X4");
  if (launch_mode < HOBO_LAUNCH_PER_INSTANCE || launch_mode > HOBO_LAUNCH_GRAPH)
    return fail(HOBO_ERR_INVALID_ARG, "unknown launch_mode");
  if (P.waves_per_block != 0 && P.waves_per_block != 1 && P.waves_per_block != 2 && P.waves_per_block != 4 &&
      P.waves_per_block != 8 && P.waves_per_block != 16)
    return fail(HOBO_ERR_INVALID_ARG, "waves_per_block must be 0, 1, 2, 4, 8 or 16");
  if (P.algorithm < HOBO_ANNEAL_AUTO || P.algorithm > HOBO_ANNEAL_BLOCKS)
    return fail(HOBO_ERR_INVALID_ARG, "unknown algorithm");
  bool all_int = true, any_int = false;
  int max_n = 0;
  for (int j = 0; j < n_instances; ++j) {
    if (!tensors[j]) return fail(HOBO_ERR_INVALID_ARG, "tensor is NULL");
    if (replicas[j] < 1 || replicas[j] > (int64_t)1 << 31) return fail(HOBO_ERR_INVALID_ARG, "replicas out of range");
    all_int = all_int && tensors[j]->t.integer;
    any_int = any_int || tensors[j]->t.integer;
    max_n = std::max(max_n, tensors[j]->t.n_vars);
  }
  if (any_int && !all_int) return fail(HOBO_ERR_INVALID_ARG, "instances mix integer and real coefficients");
  if (P.precision == HOBO_PREC_INT8X4 && !all_int) return fail(HOBO_ERR_PRECISION, "INT8X4 needs integer tensors");
  if (P.precision == HOBO_PREC_INT8X4 && max_n > 64)
    return fail(HOBO_ERR_UNSUPPORTED, "INT8X4 annealing supports at most 64 variables");
  for (int j = 0; j < n_instances; ++j) {
    std::string e;
    if (int s = hobo::check_prec(&tensors[j]->t, P.precision, &e)) return fail(s, e);
  }
  // kernel of each instance: blocked where it applies (and is not overridden)
  std::vector<int> blocked((size_t)n_instances);
  for (int j = 0; j < n_instances; ++j) {
    const bool can = tensors[j]->t.order <= 3 && P.precision != HOBO_PREC_INT8X4;
    if (P.algorithm == HOBO_ANNEAL_BLOCKS && !can)
      return fail(HOBO_ERR_UNSUPPORTED, "the blocked annealer covers orders up to 3 in FP32 / BF16 precisions");
    const bool exact = blocked_exact(tensors[j]->t);
    if (P.algorithm == HOBO_ANNEAL_BLOCKS && !exact)
      return fail(HOBO_ERR_RANGE, "integer tensor too large for the blocked annealer's exact FP32 fields "
                                  "(3 x the largest per-variable sum |w| must stay below 2^24)");
    blocked[(size_t)j] = P.algorithm == HOBO_ANNEAL_SLABS ? 0 : (can && exact ? 1 : 0);
  }
  if (hobo_status s = need_device()) return s;
  hipStream_t st = (hipStream_t)stream;
  std::string err;

  // device layouts (blocking on first use)
  std::vector<hobo::Packed*> pks((size_t)n_instances);
  std::vector<hobo::TermsDev*> tds((size_t)n_instances);
  for (int j = 0; j < n_instances; ++j) {
    const int mode = blocked[(size_t)j] ? hobo::M_BLOCKS : hobo::M_SLABS;
    if (int s = hobo::get_packed(&tensors[j]->t, mode, P.precision, &pks[(size_t)j], &err)) return fail(s, err);
    if (int s = hobo::get_terms(&tensors[j]->t, &tds[(size_t)j], &err)) return fail(s, err);
  }
  const int S = P.sweeps;
  // workspace layout
  int64_t totB = 0, tot_tiles = 0, max_B = 0;
  int max_W = 1;
  for (int j = 0; j < n_instances; ++j) {
    totB += replicas[j];
    tot_tiles += (replicas[j] + 15) / 16;
    max_B = std::max<int64_t>(max_B, replicas[j]);
    max_W = std::max(max_W, (tensors[j]->t.n_vars + 63) / 64);
  }
  auto align = [](size_t v) { return (v + 255) & ~(size_t)255; };
  size_t off_e = 0;
  size_t off_best = align(off_e + (size_t)totB * 8);
  size_t off_trace = align(off_best + (size_t)totB * 8);
  size_t off_beta = align(off_trace + (size_t)tot_tiles * (size_t)std::max(S, 1) * 8);
  size_t off_inst = align(off_beta + (size_t)std::max(S, 1) * 8);
  size_t off_items = align(off_inst + (size_t)n_instances * sizeof(hobo::AnnealInstDev));
  size_t off_small = align(off_items + (size_t)tot_tiles * sizeof(hobo::AnnealItem));
  size_t off_term = align(off_small + (size_t)n_instances * sizeof(hobo::InstSmall));
  size_t term_bytes = 0;
  int max_groups = 1;
  for (int j = 0; j < n_instances; ++j) {
    term_bytes += align(hobo::term_workspace_bytes(&tensors[j]->t, replicas[j]));
    max_groups = std::max(max_groups, (tds[(size_t)j]->n_mono + 4095) / 4096);
  }
  size_t off_ones = align(off_term + term_bytes);
  const bool learned = P.proposal == HOBO_PROPOSAL_LEARNED;
  size_t off_learn = align(off_ones + 256);
  size_t learn_bytes = 0;
  if (learned)
    for (int j = 0; j < n_instances; ++j) {
      const int64_t n = tensors[j]->t.n_vars;
      learn_bytes += align((size_t)replicas[j] * n * (tensors[j]->t.integer ? 8 : 4));
      learn_bytes += align((size_t)((replicas[j] + 15) / 16) * P.refresh * n);
    }
  // the blocked kernel's uniforms -log(u): one launch window at a time,
  // 2 KB per (16 replicas, sweep, block); the window is cut to keep them
  // within 1 GiB
  size_t unif_per_sweep = 0;
  for (int j = 0; j < n_instances; ++j)
    if (blocked[(size_t)j])
      unif_per_sweep += (size_t)((replicas[j] + 15) / 16) * (size_t)pks[(size_t)j]->nblocks * 2048;
  const int win_max = P.proposal != HOBO_PROPOSAL_METROPOLIS ? hobo::anneal_mask_window() : hobo::anneal_sweep_window();
  int unif_sweeps = 0;
  if (unif_per_sweep > 0) {
    const size_t cap = (size_t)1 << 30;
    unif_sweeps = (int)std::min<size_t>((size_t)std::min(win_max, std::max(S, 1)),
                                        std::max<size_t>(1, cap / unif_per_sweep));
  }
  size_t off_unif = align(off_learn + learn_bytes);
  size_t total = align(off_unif + unif_per_sweep * (size_t)unif_sweeps);
  std::vector<hobo::Packed*> fpks((size_t)n_instances, nullptr);
  std::vector<const double*> rns((size_t)n_instances, nullptr);
  if (learned)
    for (int j = 0; j < n_instances; ++j) {
      if (int s = hobo::get_packed(&tensors[j]->t, hobo::M_FIELDS, P.precision, &fpks[(size_t)j], &err))
        return fail(s, err);
      if (int s = hobo::get_row_norms(&tensors[j]->t, &rns[(size_t)j], &err)) return fail(s, err);
    }

  // inverse temperatures of this call's sweeps
  std::vector<double> beta((size_t)std::max(S, 1));
  for (int s = 0; s < S; ++s) beta[(size_t)s] = schedule_beta(P.t_start, P.t_end, P.first_sweep + s, L);
  const int init_random = P.init == HOBO_INIT_RANDOM ? 1 : 0;
  // Tuned annealer width of the call's kernel of each kind (1 blocked, 0
  // per-bit): the hobo_autotune result of its costliest instance (stored
  // tiles x replicas), 0 if that one was not tuned.  All instances of a kind
  // share one persistent launch, so the instance that dominates its time
  // decides its shape.
  auto tuned_of_kind = [&](int kind) {
    int best = -1;
    int64_t best_cost = -1;
    for (int j = 0; j < n_instances; ++j) {
      if (blocked[(size_t)j] != kind) continue;
      const int64_t c = (int64_t)pks[(size_t)j]->ntiles * replicas[j];
      if (c > best_cost) {
        best_cost = c;
        best = j;
      }
    }
    return best < 0 ? 0 : tuned_shape(tensors[best]->t, hobo::TK_ANNEAL, P.precision, replicas[best]);
  };
  const int tuned_blk = tuned_of_kind(1);
  // waves per work-group of the per-bit slab kernel: requested, tuned, or its default
  // (at most 8: a request of 16 means the widest)
  const int slab_waves = std::min(8, P.waves_per_block ? P.waves_per_block : tuned_of_kind(0));
  auto base_plan = [&]() {
    hobo::AnnealPlan pl;
    pl.sweeps = S;
    pl.s_first = P.first_sweep;
    pl.seed = P.seed;
    pl.init_random = init_random;
    pl.cont = P.continue_best;
    pl.masked = P.proposal != HOBO_PROPOSAL_METROPOLIS ? 1 : 0;
    pl.prec = P.precision;
    return pl;
  };
  // blocked kernel width (one decision wave plus streaming waves, so at
  // least 2): one 16-replica group per CU wants all sixteen waves (with a
  // staging wave), two groups per CU eight each; the three-term split keeps
  // sixteen (its eight-wave form runs short of registers)
  auto blk_waves = [&](int64_t tiles) {
    int nw = P.waves_per_block;
    if (!nw) nw = tuned_blk;
    if (!nw) nw = (tiles <= 256 || P.precision == HOBO_PREC_BF16X3) ? 16 : 8;
    return nw < 2 ? 2 : nw;
  };

  // cache lookup
  std::vector<uint64_t> key;
  key.push_back((uint64_t)launch_mode);
  key.push_back((uint64_t)n_instances);
  for (int j = 0; j < n_instances; ++j) {
    key.push_back((uint64_t)(uintptr_t)tensors[j]);
    key.push_back((uint64_t)replicas[j]);
  }
  {
    uint64_t pbits[7];
    std::memcpy(&pbits[0], &P.t_start, 8);
    std::memcpy(&pbits[1], &P.t_end, 8);
    pbits[2] = P.seed;
    pbits[3] = ((uint64_t)(uint32_t)P.sweeps << 32) | (uint32_t)P.precision;
    pbits[4] = ((uint64_t)(uint32_t)P.init << 32) | ((uint32_t)P.proposal << 8) | (uint32_t)P.waves_per_block;
    // the first sweep only sets the plans' sweep offset and the uploaded
    // inverse temperatures, which a non-captured setup takes per call (so
    // consecutive windows of one schedule reuse the setup); a captured graph
    // holds them
    const uint32_t fs_key = launch_mode == HOBO_LAUNCH_GRAPH ? (uint32_t)P.first_sweep : 0u;
    pbits[5] = ((uint64_t)fs_key << 32) | (uint32_t)L;
    pbits[6] = ((uint64_t)(uint32_t)P.continue_best << 32) | (uint32_t)P.algorithm;
    for (auto v : pbits) key.push_back(v);
  }
  key.push_back((uint64_t)(uintptr_t)P.attempt);
  key.push_back(((uint64_t)(uint32_t)slab_waves << 32) | (uint32_t)tuned_blk);  // tuned shapes in force
  if (learned) {
    uint64_t lb[2];
    uint32_t tb32, pf32;
    std::memcpy(&tb32, &P.tau, 4);
    std::memcpy(&pf32, &P.p_floor, 4);
    lb[0] = ((uint64_t)tb32 << 32) | pf32;
    lb[1] = (uint64_t)(uint32_t)P.refresh;
    key.push_back(lb[0]);
    key.push_back(lb[1]);
    key.push_back((uint64_t)(uintptr_t)P.mlp);
  }
  key.push_back((uint64_t)(uintptr_t)x_inout);
  key.push_back((uint64_t)(uintptr_t)best_x_out);
  key.push_back((uint64_t)(uintptr_t)best_e_out);
  key.push_back((uint64_t)(uintptr_t)trace_out);

  std::lock_guard<std::mutex> lock(g_anneal_mu);
  AnnealEntry* ent = nullptr;
  for (auto it = g_anneal.begin(); it != g_anneal.end(); ++it)
    if (it->key == key) {
      g_anneal.splice(g_anneal.begin(), g_anneal, it);
      ent = &g_anneal.front();
      break;
    }
  if (!ent) {
    AnnealEntry ne;
    ne.key = key;
    ne.mode = launch_mode;
    if (hobo_status hs = hip_status(hipMalloc(&ne.work, total), "hipMalloc")) return hs;
    ne.bytes = total;
    char* wb = static_cast<char*>(ne.work);
    std::vector<hobo::AnnealInstDev> inst((size_t)n_instances);
    std::vector<hobo::InstSmall> small((size_t)n_instances);
    std::vector<std::vector<hobo::AnnealItem>> items_of((size_t)n_instances);
    int64_t xoff = 0, roff = 0, toff = 0, att_off = 0;
    size_t term_off = 0, learn_off = 0, unif_off = 0;
    int max_ct = 1, max_nw = 1;
    ne.beta = beta;
    if (learned) {
      ne.refresh = P.refresh;
      ne.mlp = P.mlp;
      ne.p_floor = (double)P.p_floor;
      ne.precision = P.precision;
      const double tau = (double)P.tau;
      ne.lthr = tau <= 0.0 ? -INFINITY : (tau >= 1.0 ? INFINITY : (float)std::log(tau / (1.0 - tau)));
    }
    for (int j = 0; j < n_instances; ++j) {
      const hobo::Tensor& T = tensors[j]->t;
      const hobo::Packed* pk = pks[(size_t)j];
      const int64_t Bj = replicas[j];
      const int W = (T.n_vars + 63) / 64;
      const int nt = (int)((Bj + 15) / 16);
      hobo::AnnealInstDev& d = inst[(size_t)j];
      d.tiles = reinterpret_cast<const unsigned char*>(pk->d_tiles);
      d.chunks = pk->d_chunks;
      d.runs = reinterpret_cast<const unsigned long long*>(pk->d_runs);
      d.slabs = pk->d_slabs;
      d.blocks = pk->d_blocks;
      d.triples = pk->d_triples;
      d.nblocks = pk->nblocks;
      d.inv_scale = std::ldexp(1.0, -pk->scale_exp);
      if (blocked[(size_t)j]) {
        d.unif = reinterpret_cast<double*>(wb + off_unif + unif_off);
        unif_off += (size_t)nt * (size_t)pk->nblocks * 2048 * (size_t)unif_sweeps;
      }
      d.x = reinterpret_cast<unsigned long long*>(x_inout + xoff);
      d.best_x = reinterpret_cast<unsigned long long*>(best_x_out + xoff);
      d.e_track = reinterpret_cast<double*>(wb + off_e) + roff;
      d.best_track = reinterpret_cast<double*>(wb + off_best) + roff;
      d.trace_part = S > 0 ? reinterpret_cast<double*>(wb + off_trace) + toff * S : nullptr;
      d.attempt = P.proposal == HOBO_PROPOSAL_MASKED ? P.attempt + att_off : nullptr;
      if (learned) {
        AnnealEntry::Learn L;
        L.fields = fpks[(size_t)j];
        L.t = &T;
        L.rnorm = rns[(size_t)j];
        L.de = wb + off_learn + learn_off;
        learn_off += align((size_t)Bj * T.n_vars * (T.integer ? 8 : 4));
        L.mask = reinterpret_cast<unsigned char*>(wb + off_learn + learn_off);
        learn_off += align((size_t)nt * P.refresh * T.n_vars);
        L.x = x_inout + xoff;
        L.B = Bj;
        eval_shape(T, P.precision, Bj, &L.rt, &L.ct, hobo::TK_FIELDS);
        d.attempt = L.mask;
        ne.learn.push_back(L);
      }
      d.B = Bj;
      d.n_vars = T.n_vars;
      d.W = W;
      d.integer = T.integer ? 1 : 0;
      d.inst_id = (unsigned long long)j;
      d.n_chunks = pk->nchunks;
      d.n_tiles = (unsigned)pk->ntiles;
      hobo::InstSmall& sm = small[(size_t)j];
      sm.rec = tds[(size_t)j]->d_rec;
      sm.n_mono = tds[(size_t)j]->n_mono;
      sm.n_vars = T.n_vars;
      sm.W = W;
      sm.integer = d.integer;
      sm.B = Bj;
      sm.rep_off = roff;
      sm.x = d.x;
      sm.best_x = d.best_x;
      sm.e_track = d.e_track;
      sm.best_track = d.best_track;
      sm.best_out = all_int ? (void*)(static_cast<int64_t*>(best_e_out) + roff)
                            : (void*)(static_cast<double*>(best_e_out) + roff);
      sm.trace_part = d.trace_part;
      sm.trace_out = trace_out ? trace_out + (int64_t)j * S : nullptr;
      sm.inst_id = d.inst_id;
      sm.ntiles16 = nt;
      sm.term_part = wb + off_term + term_off;
      term_off += align(hobo::term_workspace_bytes(&T, Bj));
      for (int q = 0; q < nt; ++q) items_of[(size_t)j].push_back(hobo::AnnealItem{j, q});
      xoff += (int64_t)W * Bj;
      roff += Bj;
      toff += nt;
      att_off += (int64_t)nt * S * T.n_vars;
      if (!blocked[(size_t)j]) {
        int ctj, nwj;
        hobo::anneal_shape((T.n_vars + 15) / 16, slab_waves, &ctj, &nwj);
        max_ct = std::max(max_ct, ctj);
        max_nw = std::max(max_nw, nwj);
      }
    }
    // item list: blocked-kernel items first, then slab-kernel items; in the
    // persistent modes each part runs most expensive instances first
    std::vector<hobo::AnnealItem> items;
    auto cost = [&](int j) { return (int64_t)pks[(size_t)j]->ntiles; };
    // blocked-kernel width: set by the whole call's item count in every
    // launch mode, so that the modes run the same kernels (the width sets
    // how the FP32 partial fields are grouped, so real-valued results
    // depend on it)
    int64_t n_blk_items = 0;
    for (int j = 0; j < n_instances; ++j)
      if (blocked[(size_t)j]) n_blk_items += (int64_t)items_of[(size_t)j].size();
    const int call_nw_blk = blk_waves(n_blk_items);
    if (launch_mode == HOBO_LAUNCH_PER_INSTANCE) {
      for (int j = 0; j < n_instances; ++j) {
        hobo::AnnealPlan pl = base_plan();
        pl.item0 = (int)items.size();
        pl.inst0 = j;
        pl.ninst = 1;
        const int nt = (int)items_of[(size_t)j].size();
        if (blocked[(size_t)j]) {
          pl.n_blk = nt;
          pl.nw_blk = call_nw_blk;
        } else {
          pl.n_slab = nt;
          hobo::anneal_shape((tensors[j]->t.n_vars + 15) / 16, slab_waves, &pl.ct, &pl.nw);
        }
        items.insert(items.end(), items_of[(size_t)j].begin(), items_of[(size_t)j].end());
        ne.plans.push_back(pl);
      }
    } else {
      std::vector<int> ord((size_t)n_instances);
      for (int j = 0; j < n_instances; ++j) ord[(size_t)j] = j;
      std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return cost(a) > cost(b); });
      hobo::AnnealPlan pl = base_plan();
      pl.inst0 = 0;
      pl.ninst = n_instances;
      for (int pass = 0; pass < 2; ++pass)
        for (int j : ord)
          if (blocked[(size_t)j] == (pass == 0 ? 1 : 0)) {
            items.insert(items.end(), items_of[(size_t)j].begin(), items_of[(size_t)j].end());
            (pass == 0 ? pl.n_blk : pl.n_slab) += (int)items_of[(size_t)j].size();
          }
      pl.nw_blk = call_nw_blk;
      // slab kernel shape: widest instance decides (all share one launch)
      int maxT = 1;
      for (int j = 0; j < n_instances; ++j)
        if (!blocked[(size_t)j]) maxT = std::max(maxT, (tensors[j]->t.n_vars + 15) / 16);
      hobo::anneal_shape(maxT, slab_waves, &pl.ct, &pl.nw);
      ne.plans.push_back(pl);
    }
    (void)max_ct;
    (void)max_nw;
    // the blocked kernel's work schedule for each plan's group width
    for (const hobo::AnnealPlan& pl : ne.plans) {
      if (pl.n_blk == 0) continue;
      for (int j = pl.inst0; j < pl.inst0 + pl.ninst; ++j) {
        if (!blocked[(size_t)j]) continue;
        const hobo::BlockSchedule* bs = nullptr;
        if (int s = hobo::get_block_schedule(&tensors[j]->t, pks[(size_t)j], pl.nw_blk, pl.masked != 0, &bs, &err)) {
          (void)hipFree(ne.work);
          return fail(s, err);
        }
        inst[(size_t)j].sched = bs->d_words;
        inst[(size_t)j].sched_hdr = bs->d_hdr;
      }
    }
    ne.tb.d_inst = reinterpret_cast<hobo::AnnealInstDev*>(wb + off_inst);
    ne.tb.d_items = reinterpret_cast<hobo::AnnealItem*>(wb + off_items);
    ne.tb.d_small = reinterpret_cast<hobo::InstSmall*>(wb + off_small);
    ne.tb.d_beta = reinterpret_cast<double*>(wb + off_beta);
    ne.tb.n_items = (int)items.size();
    ne.tb.max_B = max_B;
    ne.tb.max_W = max_W;
    ne.tb.max_groups = max_groups;
    ne.tb.d_ones = reinterpret_cast<const unsigned char*>(wb + off_ones);
    ne.tb.unif_sweeps = unif_sweeps;
    hipError_t e = hipMemcpy(ne.tb.d_inst, inst.data(), inst.size() * sizeof(inst[0]), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(ne.tb.d_items, items.data(), items.size() * sizeof(items[0]), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(ne.tb.d_small, small.data(), small.size() * sizeof(small[0]), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ne.tb.d_beta, beta.data(), beta.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
      std::vector<unsigned char> ones(256, 1);
      e = hipMemcpy(wb + off_ones, ones.data(), ones.size(), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
      (void)hipFree(ne.work);
      return hip_status(e, "table upload");
    }
    if (launch_mode == HOBO_LAUNCH_GRAPH) {
      hipStream_t cap;
      if (hobo_status hs = hip_status(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "hipStreamCreate")) {
        (void)hipFree(ne.work);
        return hs;
      }
      hipGraph_t graph = nullptr;
      int s = HOBO_OK;
      e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        s = enqueue_plan(ne, ne.plans[0], (void*)cap, &err);
        hipError_t e2 = hipStreamEndCapture(cap, &graph);
        if (e == hipSuccess) e = e2;
      }
      (void)hipStreamDestroy(cap);
      if (e == hipSuccess && s == HOBO_OK) e = hipGraphInstantiate(&ne.exec, graph, nullptr, nullptr, 0);
      if (graph) (void)hipGraphDestroy(graph);
      if (e != hipSuccess || s != HOBO_OK) {
        (void)hipFree(ne.work);
        if (s) return fail(s, err);
        return hip_status(e, "graph capture");
      }
    }
    g_anneal.push_front(std::move(ne));
    ent = &g_anneal.front();
    size_t older = 0;
    for (auto it = std::next(g_anneal.begin()); it != g_anneal.end(); ++it) older += it->bytes;
    while (g_anneal.size() > 1 && (g_anneal.size() > kAnnealKeep || older > kAnnealKeepBytes)) {
      older -= g_anneal.back().bytes;
      release_entry(g_anneal.back());
      g_anneal.pop_back();
    }
  }
  int s = HOBO_OK;
  if (launch_mode == HOBO_LAUNCH_GRAPH) {
    return hip_status(hipGraphLaunch(ent->exec, st), "hipGraphLaunch");
  }
  if (!ent->plans.empty() && ent->plans[0].s_first != P.first_sweep) {
    // a setup built for another window of the schedule: this call's sweep
    // offset and inverse temperatures (uploaded in stream order, after the
    // previous call's kernels have read theirs)
    for (auto& pl : ent->plans) pl.s_first = P.first_sweep;
    ent->beta = beta;
    if (hobo_status hs = hip_status(hipMemcpyAsync(ent->tb.d_beta, beta.data(), beta.size() * 8,
                                                   hipMemcpyHostToDevice, st), "inverse temperature upload"))
      return hs;
  }
  for (size_t k = 0; k < ent->plans.size() && s == HOBO_OK; ++k) s = enqueue_plan(*ent, ent->plans[k], stream, &err);
  if (s) return fail(s, err);
  return ok();
}

// ------------------------------------------------------------ learned proposal
hobo_status hobo_mlp_forward(const float* params, const float* feats, int64_t M, float* logits_out, void* stream) {
  g_err.clear();
  if (!params || !feats || !logits_out) return fail(HOBO_ERR_INVALID_ARG, "NULL argument");
  if (M < 0 || M > (int64_t)1 << 40) return fail(HOBO_ERR_INVALID_ARG, "M out of range");
  if (hobo_status s = need_device()) return s;
  std::string err;
  if (int s = hobo::mlp_forward(params, feats, M, logits_out, (hipStream_t)stream, &err)) return fail(s, err);
  return ok();
}

hobo_status hobo_mlp_train(float* state, const float* feats, const float* labels, int64_t M,
                           const hobo_mlp_train_params* tp, float* loss_trace, void* stream) {
  g_err.clear();
  if (!state || !feats || !labels || !tp) return fail(HOBO_ERR_INVALID_ARG, "NULL argument");
  if (M < 1 || M > (int64_t)1 << 40) return fail(HOBO_ERR_INVALID_ARG, "M out of range");
  if (tp->batch < 1 || tp->batch > (1 << 24)) return fail(HOBO_ERR_INVALID_ARG, "batch out of range");
  if (tp->epochs < 0) return fail(HOBO_ERR_INVALID_ARG, "epochs must be >= 0");
  if (!(tp->lr > 0.0f) || !(tp->beta1 >= 0.0f && tp->beta1 < 1.0f) || !(tp->beta2 >= 0.0f && tp->beta2 < 1.0f) ||
      !(tp->eps > 0.0f) || tp->step0 < 0)
    return fail(HOBO_ERR_INVALID_ARG, "invalid optimiser parameters");
  if (hobo_status s = need_device()) return s;
  hipStream_t st = (hipStream_t)stream;
  std::string err;
  void* part = nullptr;
  if (hobo_status s = hip_status(hipMallocAsync(&part, hobo::mlp_train_workspace(tp->batch), st), "hipMallocAsync"))
    return s;
  int64_t step = tp->step0, k = 0;
  int rc = HOBO_OK;
  for (int e = 0; e < tp->epochs && rc == HOBO_OK; ++e)
    for (int64_t m0 = 0; m0 < M && rc == HOBO_OK; m0 += tp->batch, ++k) {
      const int mb = (int)std::min<int64_t>(tp->batch, M - m0);
      ++step;
      const float bc1 = (float)(1.0 - std::pow((double)tp->beta1, (double)step));
      const float bc2 = (float)(1.0 - std::pow((double)tp->beta2, (double)step));
      rc = hobo::mlp_train_step(state, feats, labels, m0, mb, tp->lr, tp->beta1, tp->beta2, tp->eps, bc1, bc2,
                                static_cast<float*>(part), loss_trace ? loss_trace + k : nullptr, st, &err);
    }
  (void)hipFreeAsync(part, st);
  if (rc) return fail(rc, err);
  return ok();
}

hobo_status hobo_mlp_grad(const float* params, const float* feats, const float* labels, int64_t M, float* grad_out,
                          float* loss_out, void* stream) {
  g_err.clear();
  if (!params || !feats || !labels || !grad_out) return fail(HOBO_ERR_INVALID_ARG, "NULL argument");
  if (M < 1 || M > (1 << 24)) return fail(HOBO_ERR_INVALID_ARG, "M must be in [1, 2^24]");
  if (hobo_status s = need_device()) return s;
  hipStream_t st = (hipStream_t)stream;
  std::string err;
  void* part = nullptr;
  if (hobo_status s = hip_status(hipMallocAsync(&part, hobo::mlp_train_workspace((int)M), st), "hipMallocAsync"))
    return s;
  int rc = hobo::mlp_grad(params, feats, labels, (int)M, static_cast<float*>(part), grad_out, loss_out, st, &err);
  (void)hipFreeAsync(part, st);
  if (rc) return fail(rc, err);
  return ok();
}

hobo_status hobo_proposal_features(const hobo_tensor* tc, const uint64_t* x_bits, const uint64_t* x_after, int64_t B,
                                   const void* de, double t_start, double t_end, int32_t sweep,
                                   int32_t schedule_sweeps, float* feats_out, float* labels_out, void* stream) {
  g_err.clear();
  if (!tc || !x_bits || !de || !feats_out) return fail(HOBO_ERR_INVALID_ARG, "NULL argument");
  if (labels_out && !x_after) return fail(HOBO_ERR_INVALID_ARG, "labels need x_after");
  if (B < 1 || B > (int64_t)1 << 40) return fail(HOBO_ERR_INVALID_ARG, "B out of range");
  if (!(t_start > 0.0) || !(t_end > 0.0) || !std::isfinite(t_start) || !std::isfinite(t_end))
    return fail(HOBO_ERR_INVALID_ARG, "temperatures must be finite and > 0");
  if (schedule_sweeps < 1 || sweep < 0 || sweep >= schedule_sweeps)
    return fail(HOBO_ERR_INVALID_ARG, "sweep must lie in [0, schedule_sweeps)");
  const double beta = schedule_beta(t_start, t_end, sweep, schedule_sweeps);
  if (hobo_status s = need_device()) return s;
  hobo_tensor* t = const_cast<hobo_tensor*>(tc);
  std::string err;
  const double* rn = nullptr;
  if (int s = hobo::get_row_norms(&t->t, &rn, &err)) return fail(s, err);
  if (int s = hobo::proposal_features(reinterpret_cast<const unsigned long long*>(x_bits),
                                      reinterpret_cast<const unsigned long long*>(x_after), B, t->t.n_vars, de,
                                      t->t.integer ? 1 : 0, beta, rn, feats_out, labels_out, (hipStream_t)stream,
                                      &err))
    return fail(s, err);
  return ok();
}

hobo_status hobo_record_transitions(hobo_tensor* t, int64_t B, const hobo_anneal_params* params,
                                    const int32_t* record, int32_t n_record, float* feats_out, float* labels_out,
                                    void* stream) {
  g_err.clear();
  if (!t || !params || !feats_out || !labels_out || (n_record > 0 && !record))
    return fail(HOBO_ERR_INVALID_ARG, "NULL argument");
  if (B < 1 || B > ((int64_t)1 << 31)) return fail(HOBO_ERR_INVALID_ARG, "B out of range");
  const hobo_anneal_params P = *params;
  if (P.sweeps < 1) return fail(HOBO_ERR_INVALID_ARG, "the schedule needs at least one sweep");
  if (P.proposal != HOBO_PROPOSAL_METROPOLIS) return fail(HOBO_ERR_INVALID_ARG, "transitions come from plain runs");
  for (int32_t k = 0; k < n_record; ++k)
    if (record[k] < 0 || record[k] >= P.sweeps || (k > 0 && record[k] <= record[k - 1]))
      return fail(HOBO_ERR_INVALID_ARG, "record must list increasing sweeps of the schedule");
  if (hobo_status s = need_device()) return s;
  hipStream_t st = (hipStream_t)stream;
  const int n = t->t.n_vars, W = (n + 63) / 64;
  const size_t xb = (size_t)W * (size_t)B * 8, deb = (size_t)B * (size_t)n * (t->t.integer ? 8 : 4);
  auto align = [](size_t v) { return (v + 255) & ~(size_t)255; };
  void* work = nullptr;
  if (hobo_status s = hip_status(hipMallocAsync(&work, align(xb) * 3 + align((size_t)B * 8) + align(deb), st),
                                 "hipMallocAsync"))
    return s;
  char* w = static_cast<char*>(work);
  uint64_t* x = reinterpret_cast<uint64_t*>(w);
  uint64_t* bx = reinterpret_cast<uint64_t*>(w + align(xb));
  uint64_t* xprev = reinterpret_cast<uint64_t*>(w + 2 * align(xb));
  void* be = w + 3 * align(xb);
  void* de = w + 3 * align(xb) + align((size_t)B * 8);
  hobo_anneal_params q = P;
  q.schedule_sweeps = P.sweeps;
  q.attempt = nullptr;
  hobo_tensor* ts[1] = {t};
  const int64_t reps[1] = {B};
  hobo_status rc = HOBO_OK;
  auto anneal = [&](int first, int count, int init, int cont) {
    q.first_sweep = first;
    q.sweeps = count;
    q.init = init;
    q.continue_best = cont;
    if (rc == HOBO_OK) rc = hobo_anneal_batch(ts, 1, reps, &q, x, bx, be, nullptr, HOBO_LAUNCH_PERSISTENT, stream);
  };
  // the start states (no sweep), then the schedule in calls that end before
  // each recorded sweep, which runs alone between its features and its labels
  anneal(0, 0, P.init, 0);
  int s = 0;
  const int fprec = P.precision == HOBO_PREC_INT8X4 ? HOBO_PREC_INT8X4 : P.precision;
  for (int32_t k = 0; k < n_record && rc == HOBO_OK; ++k) {
    const int r = record[k];
    if (r > s) anneal(s, r - s, HOBO_INIT_GIVEN, 1);
    if (rc == HOBO_OK) rc = hobo_local_fields(t, x, B, fprec, de, nullptr, stream);
    if (rc == HOBO_OK) rc = hip_status(hipMemcpyAsync(xprev, x, xb, hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
    anneal(r, 1, HOBO_INIT_GIVEN, 1);
    if (rc == HOBO_OK)
      rc = hobo_proposal_features(t, xprev, x, B, de, P.t_start, P.t_end, r, P.sweeps,
                                  feats_out + (size_t)k * (size_t)B * (size_t)n * 3,
                                  labels_out + (size_t)k * (size_t)B * (size_t)n, stream);
    s = r + 1;
  }
  (void)hipFreeAsync(work, st);
  return rc == HOBO_OK ? ok() : rc;
}

// ------------------------------------------------------------ gradient descent
hobo_status hobo_gd_gradient(const hobo_tensor* tc, const double* p, int64_t B, double* g_out, void* stream) {
  g_err.clear();
  if (!tc || !p || !g_out) return fail(HOBO_ERR_INVALID_ARG, "NULL argument");
  if (B < 1 || B > ((int64_t)1 << 40)) return fail(HOBO_ERR_INVALID_ARG, "B out of range");
  if (hobo_status s = need_device()) return s;
  hobo_tensor* t = const_cast<hobo_tensor*>(tc);
  std::string err;
  hobo::GDDev* gd;
  if (int s = hobo::get_gd(&t->t, &gd, &err)) return fail(s, err);
  hobo::GDArgs a{gd->d_ptr, gd->d_rec, t->t.n_vars, B, p, g_out, 0.0, 1, t->t.order, stream};
  if (int s = hobo::launch_gd_step(a, &err)) return fail(s, err);
  return ok();
}

hobo_status hobo_gd_batch(const hobo_tensor* tc, int64_t B, const hobo_gd_params* params, double* p_inout,
                          uint64_t* x_out, void* e_out, void* stream) {
  g_err.clear();
  if (!tc || !params || !p_inout || !x_out || !e_out) return fail(HOBO_ERR_INVALID_ARG, "NULL argument");
  const hobo_gd_params P = *params;
  if (B < 1 || B > ((int64_t)1 << 31)) return fail(HOBO_ERR_INVALID_ARG, "B out of range");
  if (P.iterations < 0) return fail(HOBO_ERR_INVALID_ARG, "iterations must be >= 0");
  if (!(P.eta >= 0.0) || std::isinf(P.eta)) return fail(HOBO_ERR_INVALID_ARG, "eta must be finite and >= 0");
  if (P.init != HOBO_INIT_RANDOM && P.init != HOBO_INIT_GIVEN) return fail(HOBO_ERR_INVALID_ARG, "unknown init");
  if (hobo_status s = need_device()) return s;
  hobo_tensor* t = const_cast<hobo_tensor*>(tc);
  hipStream_t st = (hipStream_t)stream;
  std::string err;
  const int n = t->t.n_vars;
  hobo::GDDev* gd;
  if (int s = hobo::get_gd(&t->t, &gd, &err)) return fail(s, err);
  hobo::TermsDev* td;
  if (int s = hobo::get_terms(&t->t, &td, &err)) return fail(s, err);
  if (P.init == HOBO_INIT_RANDOM)
    if (int s = hobo::launch_gd_init(n, B, P.seed, p_inout, stream, &err)) return fail(s, err);
  // ping-pong between the caller's buffer and a workspace; the term energies'
  // workspace shares the allocation
  const size_t pbytes = ((size_t)n * (size_t)B * 8 + 255) & ~(size_t)255;
  const size_t wbytes = pbytes + hobo::term_workspace_bytes(&t->t, B);
  void* work = nullptr;
  if (hobo_status s = hip_status(hipMallocAsync(&work, wbytes, st), "hipMallocAsync")) return s;
  double* other = static_cast<double*>(work);
  double* cur = p_inout;
  int rc = HOBO_OK;
  for (int it = 0; it < P.iterations && rc == HOBO_OK; ++it) {
    double* nxt = cur == p_inout ? other : p_inout;
    hobo::GDArgs a{gd->d_ptr, gd->d_rec, n, B, cur, nxt, P.eta, 0, t->t.order, stream};
    rc = hobo::launch_gd_step(a, &err);
    cur = nxt;
  }
  if (rc == HOBO_OK && cur != p_inout)
    rc = hip_status(hipMemcpyAsync(p_inout, cur, (size_t)n * (size_t)B * 8, hipMemcpyDeviceToDevice, st),
                    "hipMemcpyAsync");
  if (rc == HOBO_OK) rc = hobo::launch_gd_round(n, B, p_inout, x_out, stream, &err);
  if (rc == HOBO_OK) {
    hobo::TermArgs ta{td, &t->t, x_out, B, e_out, static_cast<char*>(work) + pbytes, stream};
    rc = hobo::launch_term_energy(ta, &err);
  }
  (void)hipFreeAsync(work, st);
  if (rc != HOBO_OK) return err.empty() ? rc : fail(rc, err);
  return ok();
}

// ------------------------------------------------------------ tensor train
struct hobo_tt {
  std::unique_ptr<hobo::TTDev> tt;
};

hobo_status hobo_tt_build(const hobo_tensor* t, hobo_tt** out) {
  g_err.clear();
  if (!t || !out) return fail(HOBO_ERR_INVALID_ARG, "NULL argument");
  if (t->t.n_mono() == 0) return fail(HOBO_ERR_INVALID_ARG, "the tensor has no monomials");
  std::string err;
  std::unique_ptr<hobo_tt> h(new (std::nothrow) hobo_tt());
  if (!h) return fail(HOBO_ERR_OOM, "host allocation failed");
  try {
    if (int s = hobo::tt_decompose(&t->t, &h->tt, &err)) return fail(s, err);
  } catch (const std::bad_alloc&) {
    return fail(HOBO_ERR_OOM, "host allocation failed");
  }
  *out = h.release();
  return ok();
}

hobo_status hobo_tt_free(hobo_tt* tt) {
  g_err.clear();
  delete tt;
  return ok();
}

hobo_status hobo_tt_info(const hobo_tt* tt, int32_t* order, int32_t* n_vars, int32_t* ranks, int64_t* n_params) {
  g_err.clear();
  if (!tt) return fail(HOBO_ERR_INVALID_ARG, "tt is NULL");
  const hobo::TTDev& d = *tt->tt;
  if (order) *order = d.order;
  if (n_vars) *n_vars = d.n;
  if (ranks)
    for (int k = 0; k <= d.order; ++k) ranks[k] = d.ranks[(size_t)k];
  if (n_params) *n_params = (int64_t)d.h_cores.size();
  return ok();
}

hobo_status hobo_tt_cores(const hobo_tt* tt, double* host_out, int64_t capacity) {
  g_err.clear();
  if (!tt || !host_out) return fail(HOBO_ERR_INVALID_ARG, "NULL argument");
  const auto& c = tt->tt->h_cores;
  if (capacity < (int64_t)c.size()) return fail(HOBO_ERR_INVALID_ARG, "capacity below the number of core entries");
  std::memcpy(host_out, c.data(), c.size() * sizeof(double));
  return ok();
}

hobo_status hobo_tt_energy(const hobo_tt* tt, const uint64_t* x_bits, int64_t B, double* e_out, void* stream) {
  g_err.clear();
  if (!tt || !x_bits || !e_out) return fail(HOBO_ERR_INVALID_ARG, "NULL argument");
  if (B < 1 || B > ((int64_t)1 << 40)) return fail(HOBO_ERR_INVALID_ARG, "B out of range");
  if (hobo_status s = need_device()) return s;
  std::string err;
  if (int s = hobo::tt_upload(tt->tt.get(), &err)) return fail(s, err);
  if (int s = hobo::launch_tt_energy(tt->tt.get(), x_bits, B, e_out, stream, &err)) return fail(s, err);
  return ok();
}

// ------------------------------------------------------------ results
hobo_status hobo_aggregate(int32_t n_vars, int64_t B, const uint64_t* x_bits, const void* energies,
                           int32_t is_integer, int64_t* n_unique, int64_t* rep_out, int64_t* count_out) {
  g_err.clear();
  if (n_vars < 1 || n_vars > hobo::kMaxVars) return fail(HOBO_ERR_INVALID_ARG, "n_vars out of range");
  if (B < 0) return fail(HOBO_ERR_INVALID_ARG, "B must be >= 0");
  if (B > 0 && (!x_bits || !energies || !rep_out || !count_out))
    return fail(HOBO_ERR_INVALID_ARG, "NULL argument");
  if (!n_unique) return fail(HOBO_ERR_INVALID_ARG, "n_unique is NULL");
  if (B == 0) {
    *n_unique = 0;
    return ok();
  }
  std::string err;
  try {
    if (int s = hobo::aggregate_states(n_vars, B, x_bits, energies, is_integer ? 1 : 0, n_unique, rep_out, count_out,
                                       &err))
      return fail(s, err);
  } catch (const std::bad_alloc&) {
    return fail(HOBO_ERR_OOM, "host allocation failed");
  }
  return ok();
}

// ------------------------------------------------------------ autotuning
hobo_status hobo_autotune(hobo_tensor* t, const uint64_t* x_bits, int64_t B, int32_t fn_mask, int32_t precision,
                          int32_t* shapes_out, void* stream) {
  g_err.clear();
  if (hobo_status s = check_bits_args(t, x_bits, B, precision)) return s;
  if (fn_mask < 1 || fn_mask > 7) return fail(HOBO_ERR_INVALID_ARG, "fn_mask must combine 1, 2 and 4");
  if (precision == HOBO_PREC_FP64) return fail(HOBO_ERR_PRECISION, "FP64 has no tiled kernels to tune");
  if (B > ((int64_t)1 << 24)) return fail(HOBO_ERR_INVALID_ARG, "tune with at most 2^24 states");
  if (hobo_status s = need_device()) return s;
  hipStream_t st = (hipStream_t)stream;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    return fail(HOBO_ERR_INVALID_ARG, "hobo_autotune blocks the host; it cannot run under stream capture");
  const hobo::Tensor& T = t->t;
  const int n = T.n_vars, W = (n + 63) / 64;
  std::string err;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  void *e = nullptr, *de = nullptr, *xa = nullptr, *bx = nullptr, *be = nullptr;
  int rc = HOBO_OK;
  auto H = [&](hipError_t x, const char* what) {
    if (rc == HOBO_OK && x != hipSuccess) rc = hip_status(x, what);
    return rc == HOBO_OK;
  };
  // time one candidate: a warm-up call, then the best of three timed calls
  auto time_it = [&](auto&& call) -> float {
    float best = 1e30f;
    if (call() != HOBO_OK) return -1.0f;
    for (int r = 0; r < 3 && rc == HOBO_OK; ++r) {
      if (!H(hipEventRecord(ev0, st), "hipEventRecord")) break;
      if (call() != HOBO_OK) return -1.0f;
      if (!H(hipEventRecord(ev1, st), "hipEventRecord") || !H(hipEventSynchronize(ev1), "hipEventSynchronize")) break;
      float ms = 0.0f;
      if (!H(hipEventElapsedTime(&ms, ev0, ev1), "hipEventElapsedTime")) break;
      best = std::min(best, ms);
    }
    return rc == HOBO_OK ? best : -1.0f;
  };
  int chosen[3] = {0, 0, 0};
  if (H(hipEventCreate(&ev0), "hipEventCreate") && H(hipEventCreate(&ev1), "hipEventCreate") &&
      H(hipMalloc(&e, (size_t)B * 8), "hipMalloc") && H(hipMalloc(&de, (size_t)B * n * 8), "hipMalloc")) {
    for (int f = 0; f < 2 && rc == HOBO_OK; ++f) {
      const int kernel = f == 0 ? hobo::TK_ENERGY : hobo::TK_FIELDS;
      if (!(fn_mask & (f == 0 ? 1 : 2))) continue;
      float best = 1e30f;
      int pick = 0;
      for (int rt = 1; rt <= 4 && rc == HOBO_OK; rt *= 2)
        for (int ct = 1; ct <= 8 && rc == HOBO_OK; ct *= 2) {
          if ((precision == HOBO_PREC_INT8X4 || rt == 4) && ct > 4) continue;
          {
            std::lock_guard<std::mutex> lock(t->t.mu);
            t->t.tuned[hobo::tune_key(kernel, precision, B)] = rt * 16 + ct;
          }
          float ms = time_it([&]() -> int {
            hobo_status s = f == 0 ? hobo_energy(t, x_bits, B, precision, e, stream)
                                   : hobo_local_fields(t, x_bits, B, precision, de, nullptr, stream);
            if (s != HOBO_OK && rc == HOBO_OK) rc = s;
            return s;
          });
          if (ms >= 0.0f && ms < best) {
            best = ms;
            pick = rt * 16 + ct;
          }
        }
      std::lock_guard<std::mutex> lock(t->t.mu);
      if (pick) t->t.tuned[hobo::tune_key(kernel, precision, B)] = pick;
      else t->t.tuned.erase(hobo::tune_key(kernel, precision, B));
      chosen[f] = pick;
    }
    if ((fn_mask & 4) && rc == HOBO_OK && H(hipMalloc(&xa, (size_t)W * B * 8), "hipMalloc") &&
        H(hipMalloc(&bx, (size_t)W * B * 8), "hipMalloc") && H(hipMalloc(&be, (size_t)B * 8), "hipMalloc")) {
      float best = 1e30f;
      int pick = 0;
      const int cand[5] = {1, 2, 4, 8, 16};
      for (int q = 0; q < 5 && rc == HOBO_OK; ++q) {
        hobo_anneal_params ap{};
        ap.sweeps = 8;
        ap.precision = precision;
        ap.t_start = 2.0;
        ap.t_end = 1.0;
        ap.seed = 1;
        ap.init = HOBO_INIT_GIVEN;
        ap.waves_per_block = cand[q];
        hobo_tensor* ts[1] = {t};
        const int64_t reps[1] = {B};
        float ms = time_it([&]() -> int {
          if (!H(hipMemcpyAsync(xa, x_bits, (size_t)W * B * 8, hipMemcpyDeviceToDevice, st), "hipMemcpyAsync"))
            return rc;
          hobo_status s = hobo_anneal_batch(ts, 1, reps, &ap, static_cast<uint64_t*>(xa), static_cast<uint64_t*>(bx),
                                            be, nullptr, HOBO_LAUNCH_PERSISTENT, stream);
          if (s != HOBO_OK && rc == HOBO_OK) rc = s;
          return s;
        });
        if (ms >= 0.0f && ms < best) {
          best = ms;
          pick = cand[q];
        }
      }
      std::lock_guard<std::mutex> lock(t->t.mu);
      if (pick) t->t.tuned[hobo::tune_key(hobo::TK_ANNEAL, precision, B)] = pick;
      chosen[2] = pick;
    }
  }
  (void)hipStreamSynchronize(st);
  if (e) (void)hipFree(e);
  if (de) (void)hipFree(de);
  if (xa) (void)hipFree(xa);
  if (bx) (void)hipFree(bx);
  if (be) (void)hipFree(be);
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  if (rc != HOBO_OK) return rc;
  if (shapes_out)
    for (int k = 0; k < 3; ++k) shapes_out[k] = chosen[k];
  return ok();
}

}  // extern "C"
