// Tensor-train (TT) form of the HOBO tensor (Sec. VI.E-F): the sequential
// decomposition of the dense paper-layout tensor into cores
// G_k[r_{k-1}][n][r_k] without approximation, on the host, and the device copy
// of the cores (made on first use) for the batched contraction kernel
// (tt_kernels.hip).
//
// Each step takes the SVD of the current matrix C (r_{k-1} n rows), keeps
// its left singular vectors of non-negligible singular value as core k and
// carries Sigma V^T into the next step.  The SVD is a one-sided Jacobi
// (Hestenes) iteration in double precision: plane rotations orthogonalise
// the columns of C^T (or of C when it is taller than wide) until every pair
// is orthogonal to working precision, so small singular values are resolved
// to about eps times the largest and the numerical rank is well defined.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "hobo_internal.h"
#include "../../include/hobo.h"

namespace hobo {

namespace {

// Orthogonalise the q columns (length p, column-major in m) by Jacobi
// rotations, accumulating the rotations in v (q x q, column-major).
void hestenes(int p, int q, std::vector<double>& m, std::vector<double>& v) {
  v.assign((size_t)q * q, 0.0);
  for (int j = 0; j < q; ++j) v[(size_t)j * q + j] = 1.0;
  const double eps = 2.220446049250313e-16;
  for (int sweep = 0; sweep < 80; ++sweep) {
    bool rotated = false;
    for (int a = 0; a < q - 1; ++a)
      for (int b = a + 1; b < q; ++b) {
        double* ca = &m[(size_t)a * p];
        double* cb = &m[(size_t)b * p];
        double alpha = 0.0, beta = 0.0, gamma = 0.0;
        for (int i = 0; i < p; ++i) {
          alpha += ca[i] * ca[i];
          beta += cb[i] * cb[i];
          gamma += ca[i] * cb[i];
        }
        if (gamma == 0.0 || std::fabs(gamma) <= eps * std::sqrt(alpha * beta)) continue;
        rotated = true;
        const double zeta = (beta - alpha) / (2.0 * gamma);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        for (int i = 0; i < p; ++i) {
          const double x = ca[i], y = cb[i];
          ca[i] = c * x - s * y;
          cb[i] = s * x + c * y;
        }
        double* va = &v[(size_t)a * q];
        double* vb = &v[(size_t)b * q];
        for (int i = 0; i < q; ++i) {
          const double x = va[i], y = vb[i];
          va[i] = c * x - s * y;
          vb[i] = s * x + c * y;
        }
      }
    if (!rotated) break;
  }
}

// SVD of the rows x cols matrix a (row-major) truncated to its numerical rank
// (sigma > sigma_max * max(rows, cols) * eps): u (rows x r, row-major) and
// sv = Sigma V^T (r x cols, row-major).
int svd_rank(int rows, int cols, const std::vector<double>& a, std::vector<double>& u, std::vector<double>& sv) {
  const double eps = 2.220446049250313e-16;
  std::vector<double> m, v;
  std::vector<double> sig;
  int r = 0;
  if (rows <= cols) {
    // columns of a^T (length cols) are the rows of a: a^T V = U' Sigma, a = V Sigma U'^T
    m = a;  // row i of a = column i of a^T, already contiguous
    hestenes(cols, rows, m, v);
    sig.resize((size_t)rows);
    for (int j = 0; j < rows; ++j) {
      double s = 0.0;
      for (int i = 0; i < cols; ++i) s += m[(size_t)j * cols + i] * m[(size_t)j * cols + i];
      sig[(size_t)j] = std::sqrt(s);
    }
    std::vector<int> ord((size_t)rows);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return sig[(size_t)x] > sig[(size_t)y]; });
    const double tol = (rows ? sig[(size_t)ord[0]] : 0.0) * std::max(rows, cols) * eps;
    for (int j : ord)
      if (sig[(size_t)j] > tol) ++r;
    r = std::max(r, 1);
    u.assign((size_t)rows * r, 0.0);
    sv.assign((size_t)r * cols, 0.0);
    for (int k = 0; k < r; ++k) {
      const int j = ord[(size_t)k];
      for (int i = 0; i < rows; ++i) u[(size_t)i * r + k] = v[(size_t)j * rows + i];  // left vector = column j of V
      for (int i = 0; i < cols; ++i) sv[(size_t)k * cols + i] = m[(size_t)j * cols + i];  // sigma_j u'_j^T
    }
  } else {
    // columns of a: a V = U Sigma
    m.assign((size_t)rows * cols, 0.0);
    for (int i = 0; i < rows; ++i)
      for (int j = 0; j < cols; ++j) m[(size_t)j * rows + i] = a[(size_t)i * cols + j];
    hestenes(rows, cols, m, v);
    sig.resize((size_t)cols);
    for (int j = 0; j < cols; ++j) {
      double s = 0.0;
      for (int i = 0; i < rows; ++i) s += m[(size_t)j * rows + i] * m[(size_t)j * rows + i];
      sig[(size_t)j] = std::sqrt(s);
    }
    std::vector<int> ord((size_t)cols);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return sig[(size_t)x] > sig[(size_t)y]; });
    const double tol = sig[(size_t)ord[0]] * std::max(rows, cols) * eps;
    for (int j : ord)
      if (sig[(size_t)j] > tol) ++r;
    r = std::max(r, 1);
    u.assign((size_t)rows * r, 0.0);
    sv.assign((size_t)r * cols, 0.0);
    for (int k = 0; k < r; ++k) {
      const int j = ord[(size_t)k];
      const double s = sig[(size_t)j];
      for (int i = 0; i < rows; ++i) u[(size_t)i * r + k] = s > 0.0 ? m[(size_t)j * rows + i] / s : 0.0;
      for (int i = 0; i < cols; ++i) sv[(size_t)k * cols + i] = s * v[(size_t)j * cols + i];  // sigma_j v_j^T
    }
  }
  return r;
}

}  // namespace

TTDev::~TTDev() {
  if (d_cores) (void)hipFree(d_cores);
}

int tt_decompose(const Tensor* t, std::unique_ptr<TTDev>* out, std::string* err) {
  const int n = t->n_vars, d = std::max(t->order, 1);
  double total = 1.0;
  for (int k = 0; k < d; ++k) total *= n;
  if (total > (double)kTTMaxDense) {
    *err = "N^k exceeds the dense limit of the TT decomposition (2^24 entries)";
    return HOBO_ERR_UNSUPPORTED;
  }
  const size_t full = (size_t)total;
  // dense tensor in the paper's layout: the smallest variable of a monomial
  // is repeated at the front until it has d indices
  std::vector<double> c(full, 0.0);
  for (int m = 0; m < t->n_mono(); ++m) {
    const uint8_t* s = t->mono_idx.data() + t->mono_ptr[m];
    const int len = (int)(t->mono_ptr[m + 1] - t->mono_ptr[m]);
    size_t off = 0;
    for (int k = 0; k < d; ++k) {
      const int v = k < d - len ? s[0] : s[k - (d - len)];
      off = off * (size_t)n + (size_t)v;
    }
    c[off] += t->w_f[m];
  }
  std::unique_ptr<TTDev> tt(new TTDev());
  tt->n = n;
  tt->order = d;
  tt->ranks.assign((size_t)d + 1, 1);
  std::vector<double> cores;
  size_t rest = full;
  int r_prev = 1;
  for (int k = 0; k < d - 1; ++k) {
    const int rows = r_prev * n;
    rest /= (size_t)n;
    const int cols = (int)rest;
    std::vector<double> u, sv;
    const int r = svd_rank(rows, cols, c, u, sv);
    if (r > kTTMaxRank) {
      *err = "TT rank " + std::to_string(r) + " exceeds the kernel limit of " + std::to_string(kTTMaxRank);
      return HOBO_ERR_UNSUPPORTED;
    }
    tt->core_off.push_back((int64_t)cores.size());
    cores.insert(cores.end(), u.begin(), u.end());  // [r_prev][n][r] row-major = u's layout
    tt->ranks[(size_t)k + 1] = r;
    c.swap(sv);  // r x cols: the next matrix, reshaped to (r n) x (cols / n)
    r_prev = r;
  }
  tt->core_off.push_back((int64_t)cores.size());
  cores.insert(cores.end(), c.begin(), c.end());  // last core [r_prev][n][1]
  tt->h_cores = cores;
  *out = std::move(tt);
  return HOBO_OK;
}

int tt_upload(TTDev* tt, std::string* err) {
  std::lock_guard<std::mutex> lock(tt->mu);
  if (tt->d_cores) return HOBO_OK;
  double* d = nullptr;
  // the cores, then kTTMaxRank zeros: the contraction reads every row whole
  // (up to its rank limit of columns) and reads rows past a core's rank there
  std::vector<double> padded(tt->h_cores);
  padded.resize(padded.size() + kTTMaxRank, 0.0);
  if (hipMalloc(reinterpret_cast<void**>(&d), padded.size() * 8) != hipSuccess) {
    (void)hipGetLastError();
    *err = "hipMalloc of the TT cores failed";
    return HOBO_ERR_OOM;
  }
  if (hipMemcpy(d, padded.data(), padded.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    *err = "hipMemcpy of the TT cores failed";
    return HOBO_ERR_HIP;
  }
  tt->d_cores = d;
  return HOBO_OK;
}

}  // namespace hobo
