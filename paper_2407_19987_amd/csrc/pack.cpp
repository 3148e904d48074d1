// Device layouts of a canonical HOBO instance.
//
// Every contraction in the engine is the product of a generated monomial
// matrix Y (one row per replica, one column per candidate monomial S' of the
// replica's bits) with a coefficient matrix M (one row per monomial S', one
// column per variable c), followed by a per-replica epilogue:
//
//   fields  : M[S'][c] = w_{S' u {c}}        (c not in S')    -> g_c, dE_c
//   energy  : M[S'][c] = w_{S' u {c}}        (c > max S')     -> E = sum_c x_c G_c
//   slab i  : M[S'][c] = w_{S' u {c} u {i}}  (c > max S', c,S' without i)
//             -> g_i = w_i + sum_c x_c G_c    (the annealer's field of bit i)
//
// The upper-triangular "energy" matrix is the paper's HOBO tensor (Sec. III.C)
// unfolded along its last index: each monomial S is stored once, at
// (S minus max S, max S).  A constant row S' = {} carries the linear
// coefficients.
//
// Rows are grouped in *runs*: eight monomials P u {m}, m = 8*beta..8*beta+7,
// that share a prefix P with max P < m.  A replica's eight values of a run are
// one byte of its bit vector masked by the product of its prefix bits, so the
// kernels generate Y from a run descriptor with a byte load.  Runs that are
// zero in every column are dropped, so sparse instances skip their zeros.
// Runs are ordered by degree, then block beta, then prefix: in the
// triangular layouts a run of block beta only reaches columns above 8*beta,
// so every chunk of runs has a contiguous range of non-zero column tiles.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <unordered_map>

#include "hobo_internal.h"
#include "../../include/hobo.h"

namespace hobo {

Packed::~Packed() {
  if (d_tiles) (void)hipFree(d_tiles);
  if (d_chunks) (void)hipFree(d_chunks);
  if (d_runs) (void)hipFree(d_runs);
  if (d_slabs) (void)hipFree(d_slabs);
  if (d_blocks) (void)hipFree(d_blocks);
  if (d_triples) (void)hipFree(d_triples);
}
BlockSchedule::~BlockSchedule() {
  if (d_words) (void)hipFree(d_words);
  if (d_hdr) (void)hipFree(d_hdr);
}
TermsDev::~TermsDev() {
  if (d_rec) (void)hipFree(d_rec);
}
Tensor::~Tensor() {
  packed.clear();
  terms.reset();
  if (d_row_norm) (void)hipFree(d_row_norm);
}

namespace {

// dense coefficient blocks of a run list (8 rows x n columns per run)
struct RunMat {
  int n = 0;
  bool integer = false;
  std::unordered_map<uint64_t, int> index;
  std::vector<uint64_t> desc;
  std::vector<double> cf;  // [run][8][n]
  std::vector<int64_t> ci;

  int run_of(uint64_t d) {
    auto it = index.find(d);
    if (it != index.end()) return it->second;
    int r = (int)desc.size();
    index.emplace(d, r);
    desc.push_back(d);
    cf.resize(cf.size() + 8 * (size_t)n, 0.0);
    if (integer) ci.resize(ci.size() + 8 * (size_t)n, 0);
    return r;
  }
  void add(uint64_t d, int e, int c, double wf, int64_t wi) {
    int r = run_of(d);
    size_t at = ((size_t)r * 8 + (size_t)e) * (size_t)n + (size_t)c;
    cf[at] += wf;
    if (integer) ci[at] += wi;
  }
};

inline uint64_t const_desc() { return (uint64_t)kRunConst << 8; }
inline uint64_t null_desc() { return (uint64_t)kRunNull << 8; }
// descriptor of the run holding monomial P u {m} (P sorted, all < m)
inline uint64_t run_desc(const uint8_t* p, int np, int m) {
  uint64_t d = (uint64_t)(m >> 3) | ((uint64_t)np << 8);
  for (int j = 0; j < np; ++j) d |= (uint64_t)p[j] << (16 + 8 * j);
  return d;
}
inline int desc_degree(uint64_t d) {
  uint32_t np = (uint32_t)(d >> 8) & 0xFF;
  if (np == kRunConst) return 0;
  if (np == kRunNull) return 99;
  return (int)np + 1;
}

// Scatter monomial S' u {c} with weight w into row S' (a run element) and
// column c.  `rest` = S' sorted (may be empty).
inline void scatter(RunMat& rm, const uint8_t* rest, int nrest, int c, double wf, int64_t wi) {
  if (nrest == 0) {
    rm.add(const_desc(), 0, c, wf, wi);
  } else {
    int m = rest[nrest - 1];
    rm.add(run_desc(rest, nrest - 1, m), m & 7, c, wf, wi);
  }
}

// Sorted permutation of the runs: degree, beta, prefix.
std::vector<int> run_order(const RunMat& rm) {
  std::vector<int> ord(rm.desc.size());
  for (size_t r = 0; r < ord.size(); ++r) ord[r] = (int)r;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) {
    uint64_t da = rm.desc[a], db = rm.desc[b];
    int ga = desc_degree(da), gb = desc_degree(db);
    if (ga != gb) return ga < gb;
    uint32_t ba = (uint32_t)(da & 0xFF), bb = (uint32_t)(db & 0xFF);
    if (ba != bb) return ba < bb;
    for (int j = 0; j < 6; ++j) {
      uint32_t pa = (uint32_t)(da >> (16 + 8 * j)) & 0xFF, pb = (uint32_t)(db >> (16 + 8 * j)) & 0xFF;
      if (pa != pb) return pa < pb;
    }
    return false;
  });
  return ord;
}

inline uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
inline float bf16_to_f(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// balanced base-256 digits d_q in [-128, 127], v = sum_q 256^q d_q
inline bool int8_limbs(int64_t v, int8_t d[4]) {
  for (int q = 0; q < 4; ++q) {
    int64_t r = ((v % 256) + 256) % 256;  // 0..255
    int64_t dq = r >= 128 ? r - 256 : r;
    d[q] = (int8_t)dq;
    v = (v - dq) / 256;
  }
  return v == 0;
}

struct PackOut {
  std::vector<uint8_t> tiles;
  std::vector<ChunkMeta> chunks;
  std::vector<uint64_t> runs;
};

// Append the runs of `rm` (already ordered by `ord`) to `po` as chunks of
// tiles in precision `prec`.  When `segments` is set the runs of each degree
// start a new chunk and the chunk that closes a degree carries seg_end.
int pack_runs(const RunMat& rm, const std::vector<int>& ord, int prec, bool segments, int n_col_tiles,
              PackOut* po, std::string* err, bool all_tiles = false, int scale_exp = 0) {
  const int rpc = runs_per_chunk(prec);
  const int n = rm.n;
  // padded run sequence (-1 = null run) and per-run order of its degree
  std::vector<int> seq;
  std::vector<int> seg_after;  // order completed after this position (0 = none)
  for (size_t p = 0; p < ord.size(); ++p) {
    seq.push_back(ord[p]);
    int deg = desc_degree(rm.desc[ord[p]]);
    bool last_of_deg = p + 1 == ord.size() || desc_degree(rm.desc[ord[p + 1]]) != deg;
    if (segments && last_of_deg) {
      while (seq.size() % rpc) seq.push_back(-1);
      seg_after.resize(seq.size(), 0);
      seg_after.back() = deg + 1;  // runs of degree d are monomials of order d+1
    }
  }
  while (seq.size() % rpc) seq.push_back(-1);
  seg_after.resize(seq.size(), 0);
  const int nchunk = (int)(seq.size() / rpc);
  const int tb = tile_bytes(prec);
  auto coef_f = [&](int run, int e, int c) -> double {
    return run < 0 || c >= n ? 0.0 : rm.cf[((size_t)run * 8 + (size_t)e) * (size_t)n + (size_t)c];
  };
  auto coef_i = [&](int run, int e, int c) -> int64_t {
    return run < 0 || c >= n ? 0 : rm.ci[((size_t)run * 8 + (size_t)e) * (size_t)n + (size_t)c];
  };
  for (int c = 0; c < nchunk; ++c) {
    // non-zero column tiles of this chunk
    int t_lo = n_col_tiles, t_hi = 0;
    for (int t = 0; t < n_col_tiles; ++t) {
      bool nz = false;
      for (int k = 0; k < rpc && !nz; ++k) {
        int run = seq[(size_t)c * rpc + k];
        if (run < 0) continue;
        for (int e = 0; e < 8 && !nz; ++e)
          for (int j = 0; j < kTileCols && !nz; ++j) nz = coef_f(run, e, 16 * t + j) != 0.0;
      }
      if (nz) {
        t_lo = std::min(t_lo, t);
        t_hi = std::max(t_hi, t + 1);
      }
    }
    if (t_hi <= t_lo) t_lo = t_hi = 0;
    if (all_tiles) {  // store every column tile, zero ones included
      t_lo = 0;
      t_hi = n_col_tiles;
    }
    ChunkMeta cm{};
    cm.tile_off = (uint32_t)(po->tiles.size() / (size_t)tb);
    cm.t_lo = (uint8_t)t_lo;
    cm.t_hi = (uint8_t)t_hi;
    cm.seg_end = (uint8_t)seg_after[(size_t)(c + 1) * rpc - 1];
    po->chunks.push_back(cm);
    for (int k = 0; k < rpc; ++k) {
      int run = seq[(size_t)c * rpc + k];
      po->runs.push_back(run < 0 ? null_desc() : rm.desc[run]);
    }
    for (int t = t_lo; t < t_hi; ++t) {
      size_t base = po->tiles.size();
      po->tiles.resize(base + (size_t)tb, 0);
      uint8_t* tile = po->tiles.data() + base;
      for (int l = 0; l < 64; ++l) {
        int g = l >> 4, j = l & 15, col = 16 * t + j;
        if (prec == P_FP32) {
          float* dst = reinterpret_cast<float*>(tile + l * 32);
          int run = seq[(size_t)c * rpc + g];
          for (int e = 0; e < 8; ++e) {
            double w = rm.integer ? (double)coef_i(run, e, col) : coef_f(run, e, col);
            dst[e] = (float)w;
          }
        } else if (prec == P_BF16X2 || prec == P_BF16X3) {
          int np = prec == P_BF16X2 ? 2 : 3;
          int run = seq[(size_t)c * rpc + g];
          for (int e = 0; e < 8; ++e) {
            double w = rm.integer ? (double)coef_i(run, e, col) : coef_f(run, e, col);
            float f = (float)w;
            uint16_t h[3];
            h[0] = bf16_rne(f);
            float r1 = f - bf16_to_f(h[0]);
            h[1] = bf16_rne(r1);
            float r2 = r1 - bf16_to_f(h[1]);
            h[2] = bf16_rne(r2);
            if (rm.integer) {
              double back = (double)bf16_to_f(h[0]) + (double)bf16_to_f(h[1]) + (np == 3 ? (double)bf16_to_f(h[2]) : 0.0);
              if (back != w) {
                *err = "integer coefficient " + std::to_string((long long)w) + " is not exact in the BF16 split";
                return HOBO_ERR_RANGE;
              }
            }
            for (int q = 0; q < np; ++q) {
              uint16_t* dst = reinterpret_cast<uint16_t*>(tile + q * 1024 + l * 16);
              dst[e] = h[q];
            }
          }
        } else if (prec == P_FP16X2) {
          // c 2^scale_exp as hi = fp16(c'), lo = fp16(c' - hi); c' - hi is
          // exact in FP32, so the pair carries 22 significant bits
          int run = seq[(size_t)c * rpc + g];
          for (int e = 0; e < 8; ++e) {
            double w = rm.integer ? (double)coef_i(run, e, col) : coef_f(run, e, col);
            const float f = std::ldexp((float)w, scale_exp);
            const _Float16 h0 = (_Float16)f;
            const _Float16 h1 = (_Float16)(f - (float)h0);
            if (rm.integer && std::ldexp((double)h0 + (double)h1, -scale_exp) != w) {
              *err = "integer coefficient " + std::to_string((long long)w) + " is not exact in the FP16 split";
              return HOBO_ERR_RANGE;
            }
            uint16_t b0, b1;
            std::memcpy(&b0, &h0, 2);
            std::memcpy(&b1, &h1, 2);
            reinterpret_cast<uint16_t*>(tile + l * 16)[e] = b0;
            reinterpret_cast<uint16_t*>(tile + 1024 + l * 16)[e] = b1;
          }
        } else {  // INT8X4
          for (int e = 0; e < 16; ++e) {
            int run = seq[(size_t)c * rpc + 2 * g + (e >> 3)];
            int64_t w = coef_i(run, e & 7, col);
            int8_t d[4];
            if (!int8_limbs(w, d)) {
              *err = "integer coefficient " + std::to_string((long long)w) + " exceeds four INT8 digits";
              return HOBO_ERR_RANGE;
            }
            for (int q = 0; q < 4; ++q) tile[q * 1024 + l * 16 + e] = (uint8_t)d[q];
          }
        }
      }
    }
  }
  return HOBO_OK;
}

template <class T>
int upload(const std::vector<T>& v, T** dst, size_t* bytes, std::string* err) {
  size_t nb = std::max<size_t>(v.size() * sizeof(T), 16);
  if (hipMalloc(reinterpret_cast<void**>(dst), nb) != hipSuccess) {
    (void)hipGetLastError();
    *err = "hipMalloc of " + std::to_string(nb) + " bytes failed";
    return HOBO_ERR_OOM;
  }
  if (!v.empty() && hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
    *err = "hipMemcpy to device failed";
    return HOBO_ERR_HIP;
  }
  *bytes += nb;
  return HOBO_OK;
}

// FP16X2 scale: the largest |w| times 2^e lies in [2^14, 2^15), well inside
// FP16's range (65504) with hi rounding included
int fp16_scale_exp(const Tensor* t) {
  double mx = 0.0;
  for (double w : t->w_f) mx = std::max(mx, std::fabs((double)(float)w));
  if (!(mx > 0.0)) return 0;
  int ex;
  (void)std::frexp(mx, &ex);  // mx = f 2^ex, f in [0.5, 1)
  return 15 - ex;
}

}  // namespace

int check_prec(const Tensor* t, int prec, std::string* err) {
  if (prec == P_INT8X4 && !t->integer) {
    *err = "INT8X4 precision needs an integer tensor";
    return HOBO_ERR_PRECISION;
  }
  if (prec == P_INT8X4) {
    // four balanced base-256 digits hold -128 * 0x01010101 .. 127 * 0x01010101
    constexpr int64_t kDigitsLo = -128LL * 0x01010101LL, kDigitsHi = 127LL * 0x01010101LL;
    if (t->w_lo < kDigitsLo || t->w_hi > kDigitsHi) {
      *err = "INT8X4: an integer coefficient exceeds four INT8 digits";
      return HOBO_ERR_RANGE;
    }
    // Each digit pass sums 0/1 products of digits in [-128, 127] over at most
    // every monomial of the instance into an int32 lane: 128 * n_mono must
    // stay below 2^31.  The fields kernel's energy carries the per-order sums
    // scaled by lcm(1..7) = 420 with up to `order` fields per monomial, in
    // int64: 420 * order * sum |w| must stay below 2^63 (which also keeps the
    // annealer's tracked energies exact in double).
    if ((int64_t)t->n_mono() >= ((int64_t)1 << 24)) {
      *err = "INT8X4: more than 2^24 monomials would overflow the int32 digit sums";
      return HOBO_ERR_RANGE;
    }
    const unsigned __int128 lim = ((unsigned __int128)1 << 63) / (unsigned __int128)(420 * std::max(t->order, 1));
    if (t->abs_sum >= lim) {
      *err = "INT8X4: 420 * order * sum |w| would overflow the int64 energy sums";
      return HOBO_ERR_RANGE;
    }
  }
  if (t->integer && (prec == P_FP32 || prec == P_BF16X2 || prec == P_BF16X3 || prec == P_FP16X2)) {
    // every partial sum of an FP32 accumulation must be an exact integer
    if (t->abs_sum >= ((unsigned __int128)1 << 24)) {
      *err = "integer tensor with sum |w| >= 2^24 cannot be exact in FP32 accumulation; use INT8X4";
      return HOBO_ERR_RANGE;
    }
  }
  return HOBO_OK;
}

int get_packed(Tensor* t, int mode, int prec, Packed** out, std::string* err) {
  std::lock_guard<std::mutex> lock(t->mu);
  int key = mode * 16 + prec;
  auto it = t->packed.find(key);
  if (it != t->packed.end()) {
    *out = it->second.get();
    return HOBO_OK;
  }
  int st = check_prec(t, prec, err);
  if (st) return st;
  const int n = t->n_vars;
  const int n_col_tiles = (n + kTileCols - 1) / kTileCols;
  const int nm = t->n_mono();
  std::unique_ptr<Packed> pk(new Packed());
  pk->mode = mode;
  pk->prec = prec;
  pk->n_col_tiles = n_col_tiles;
  if (prec == P_FP16X2) pk->scale_exp = fp16_scale_exp(t);
  const int sx = pk->scale_exp;
  PackOut po;
  // tile 0 is all zeros: the kernels load it in place of absent tiles so that
  // every chunk issues the same number of loads
  po.tiles.assign((size_t)tile_bytes(prec), 0);
  uint8_t rest[kMaxOrder];
  if (mode == M_FIELDS || mode == M_ENERGY) {
    RunMat rm;
    rm.n = n;
    rm.integer = t->integer;
    for (int m = 0; m < nm; ++m) {
      const uint8_t* s = t->mono_idx.data() + t->mono_ptr[m];
      int len = (int)(t->mono_ptr[m + 1] - t->mono_ptr[m]);
      double wf = t->w_f[m];
      int64_t wi = t->integer ? t->w_i[m] : 0;
      if (mode == M_FIELDS) {
        for (int a = 0; a < len; ++a) {  // column c = s[a], row S minus c
          int nr = 0;
          for (int b = 0; b < len; ++b)
            if (b != a) rest[nr++] = s[b];
          scatter(rm, rest, nr, s[a], wf, wi);
        }
      } else {  // column c = max S
        scatter(rm, s, len - 1, s[len - 1], wf, wi);
      }
    }
    st = pack_runs(rm, run_order(rm), prec, mode == M_FIELDS, n_col_tiles, &po, err, false, sx);
    if (st) return st;
    pk->nchunks = (int)po.chunks.size();
  } else if (mode == M_BLOCKS) {
    if (t->order > 3) {
      *err = "the blocked annealing layout covers orders up to 3";
      return HOBO_ERR_UNSUPPORTED;
    }
    if (prec == P_INT8X4) {
      *err = "the blocked annealing layout has no INT8X4 form";
      return HOBO_ERR_UNSUPPORTED;
    }
    const int nb = (n + kBlockBits - 1) / kBlockBits;
    std::vector<std::vector<int>> touch((size_t)nb);  // monomials with a variable in each block
    for (int m = 0; m < nm; ++m) {
      int last = -1;
      for (int64_t p = t->mono_ptr[m]; p < t->mono_ptr[m + 1]; ++p) {
        int q = t->mono_idx[p] / kBlockBits;
        if (q != last) touch[(size_t)q].push_back(m);
        last = q;
      }
    }
    std::vector<BlockMeta> bm((size_t)nb);
    std::vector<float> tri((size_t)nb * 4096, 0.0f);
    for (int q = 0; q < nb; ++q) {
      const int j0 = q * kBlockBits;
      const int nbits = std::min(kBlockBits, n - j0);
      const int npairs = nbits * (nbits - 1) / 2;
      const int npt = (npairs + kTileCols - 1) / kTileCols;
      RunMat rg;
      rg.n = kTileCols;
      rg.integer = t->integer;
      std::vector<RunMat> rh((size_t)kPairTiles);
      for (auto& r : rh) {
        r.n = kTileCols;
        r.integer = t->integer;
      }
      for (int m : touch[(size_t)q]) {
        const uint8_t* s = t->mono_idx.data() + t->mono_ptr[m];
        const int len = (int)(t->mono_ptr[m + 1] - t->mono_ptr[m]);
        const double wf = t->w_f[m];
        const int64_t wi = t->integer ? t->w_i[m] : 0;
        int in[kMaxOrder], nin = 0;  // positions of s inside the block
        for (int a = 0; a < len; ++a)
          if (s[a] >= j0 && s[a] < j0 + kBlockBits) in[nin++] = a;
        // field of variable s[in[u]]: row S minus it.  A row with exactly one
        // other variable b of the block is left out: the kernel adds
        // sum_b x_b H_ab(x0), which holds those terms, and counts every row
        // with two (a triple inside the block) twice, so that row is stored
        // with its sign reversed.  Rows with no variable of the block are
        // stored as they are.
        if (nin == 1 || nin == 3)
          for (int u = 0; u < nin; ++u) {
            int nr = 0;
            for (int b = 0; b < len; ++b)
              if (b != in[u]) rest[nr++] = s[b];
            const double sg = nin == 3 ? -1.0 : 1.0;
            scatter(rg, rest, nr, s[in[u]] - j0, sg * wf, nin == 3 ? -wi : wi);
          }
        for (int u = 0; u < nin; ++u)
          for (int v = u + 1; v < nin; ++v) {  // coupling of the pair: row S minus both
            int nr = 0;
            for (int b = 0; b < len; ++b)
              if (b != in[u] && b != in[v]) rest[nr++] = s[b];
            const int pc = pair_col(s[in[u]] - j0, s[in[v]] - j0);
            scatter(rh[(size_t)(pc / kTileCols)], rest, nr, pc % kTileCols, wf, wi);
          }
        if (len == 3 && nin == 3) {  // triple inside the block, stored at every ordering
          const int v3[3] = {s[0] - j0, s[1] - j0, s[2] - j0};
          const int pm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
          for (auto& o : pm)
            tri[(size_t)q * 4096 + (size_t)v3[o[0]] * 256 + (size_t)v3[o[1]] * 16 + (size_t)v3[o[2]]] =
                std::ldexp((float)wf, sx);
        }
      }
      BlockMeta& b = bm[(size_t)q];
      b.nbits = (uint32_t)nbits;
      b.npt = (uint32_t)npt;
      // The field list's runs that read no bit of the previous block of the
      // sweep come first: the kernel computes them while that block's
      // decisions are still being taken.
      const int p0 = ((q + nb - 1) % nb) * kBlockBits;
      auto reads_prev = [&](uint64_t d) {
        const uint32_t np = (uint32_t)(d >> 8) & 0xFFu;
        if (np == kRunConst || np == kRunNull) return false;
        const int lo = (int)(d & 0xFFu) * 8;  // the run's eight variables lo .. lo+7
        if (lo + 8 > p0 && lo < p0 + kBlockBits) return true;
        for (uint32_t j = 0; j < np; ++j) {
          const int v = (int)((d >> (16 + 8 * j)) & 0xFFu);
          if (v >= p0 && v < p0 + kBlockBits) return true;
        }
        return false;
      };
      for (int li = 0; li < kBlockLists; ++li) {
        b.chunk0[li] = (uint32_t)po.chunks.size();
        if (li == 0) {
          std::vector<int> early, late;
          for (int r : run_order(rg)) (reads_prev(rg.desc[(size_t)r]) ? late : early).push_back(r);
          if (!early.empty()) {
            st = pack_runs(rg, early, prec, false, 1, &po, err, true, sx);
            if (st) return st;
          }
          b.nearly = (uint32_t)po.chunks.size() - b.chunk0[0];
          if (!late.empty()) {
            st = pack_runs(rg, late, prec, false, 1, &po, err, true, sx);
            if (st) return st;
          }
        } else if (li - 1 < npt) {
          RunMat& r = rh[(size_t)(li - 1)];
          st = pack_runs(r, run_order(r), prec, false, 1, &po, err, true, sx);
          if (st) return st;
        }
        b.nchunks[li] = (uint32_t)po.chunks.size() - b.chunk0[li];
      }
    }
    pk->nchunks = (int)po.chunks.size();
    pk->nblocks = nb;
    pk->h_blocks = bm;
    st = upload(bm, &pk->d_blocks, &pk->bytes, err);
    if (st) return st;
    st = upload(tri, &pk->d_triples, &pk->bytes, err);
    if (st) return st;
  } else {  // M_SLABS: one triangular matrix per variable i
    // monomials containing each variable
    std::vector<std::vector<int>> inc((size_t)n);
    for (int m = 0; m < nm; ++m)
      for (int64_t p = t->mono_ptr[m]; p < t->mono_ptr[m + 1]; ++p) inc[t->mono_idx[p]].push_back(m);
    std::vector<SlabMeta> slabs((size_t)n);
    for (int i = 0; i < n; ++i) {
      RunMat rm;
      rm.n = n;
      rm.integer = t->integer;
      SlabMeta sm{};
      for (int m : inc[(size_t)i]) {
        const uint8_t* s = t->mono_idx.data() + t->mono_ptr[m];
        int len = (int)(t->mono_ptr[m + 1] - t->mono_ptr[m]);
        double wf = t->w_f[m];
        int64_t wi = t->integer ? t->w_i[m] : 0;
        if (len == 1) {
          sm.a_f += wf;
          sm.a_i += wi;
          continue;
        }
        int nr = 0;
        uint8_t tt[kMaxOrder];
        for (int b = 0; b < len; ++b)
          if (s[b] != i) tt[nr++] = s[b];
        // slab monomial T = S minus i; column c = max T, row T minus c
        scatter(rm, tt, nr - 1, tt[nr - 1], wf, wi);
      }
      sm.chunk0 = (uint32_t)po.chunks.size();
      sm.run0 = (uint32_t)po.runs.size();
      st = pack_runs(rm, run_order(rm), prec, false, n_col_tiles, &po, err, false, sx);
      if (st) return st;
      sm.nchunks = (uint32_t)po.chunks.size() - sm.chunk0;
      if (sm.nchunks == 0) {  // the annealer visits every slab through at least one chunk
        ChunkMeta cm{};
        cm.tile_off = (uint32_t)(po.tiles.size() / (size_t)tile_bytes(prec));
        po.chunks.push_back(cm);
        for (int k = 0; k < runs_per_chunk(prec); ++k) po.runs.push_back(null_desc());
        sm.nchunks = 1;
      }
      for (uint32_t c = sm.chunk0; c < sm.chunk0 + sm.nchunks; ++c) {
        po.chunks[c].bit = (uint8_t)i;
        po.chunks[c].seg_end = c + 1 == sm.chunk0 + sm.nchunks ? 1 : 0;
      }
      slabs[(size_t)i] = sm;
    }
    pk->nchunks = (int)po.chunks.size();
    st = upload(slabs, &pk->d_slabs, &pk->bytes, err);
    if (st) return st;
  }
  pk->ntiles = (int)(po.tiles.size() / (size_t)tile_bytes(prec));
  pk->h_chunks = po.chunks;
  uint8_t* dt = nullptr;
  st = upload(po.tiles, &dt, &pk->bytes, err);
  pk->d_tiles = dt;
  if (st) return st;
  st = upload(po.chunks, &pk->d_chunks, &pk->bytes, err);
  if (st) return st;
  st = upload(po.runs, &pk->d_runs, &pk->bytes, err);
  if (st) return st;
  *out = pk.get();
  t->packed.emplace(key, std::move(pk));
  return HOBO_OK;
}

int get_block_schedule(Tensor* t, Packed* pk, int nw, bool masked, const BlockSchedule** out, std::string* err) {
  std::lock_guard<std::mutex> lock(t->mu);
  const int key = nw * 2 + (masked ? 1 : 0);
  auto it = pk->sched.find(key);
  if (it != pk->sched.end()) {
    *out = it->second.get();
    return HOBO_OK;
  }
  const int ns = block_streamers(nw);
  if (ns < 1 || pk->h_blocks.empty()) {
    *err = "no blocked layout for this work-group width";
    return HOBO_ERR_INVALID_ARG;
  }
  if ((int64_t)pk->nchunks + 1 >= (int64_t)1 << 20) {
    *err = "blocked schedule: more chunks than a slot word holds";
    return HOBO_ERR_RANGE;
  }
  std::vector<uint32_t> words, hdr;
  build_block_schedule(pk->h_blocks, ns, masked, &words, &hdr);
  for (uint32_t w : words)
    if ((w & 0xFFFFFu) >= (uint32_t)pk->ntiles) {
      *err = "blocked schedule: tile index out of range";
      return HOBO_ERR_RANGE;
    }
  std::unique_ptr<BlockSchedule> bs(new BlockSchedule());
  size_t bytes = 0;
  int st = upload(words, &bs->d_words, &bytes, err);
  if (st) return st;
  st = upload(hdr, &bs->d_hdr, &bytes, err);
  if (st) return st;
  pk->bytes += bytes;
  *out = bs.get();
  pk->sched.emplace(key, std::move(bs));
  return HOBO_OK;
}

int get_row_norms(Tensor* t, const double** out, std::string* err) {
  std::lock_guard<std::mutex> lock(t->mu);
  if (!t->d_row_norm) {
    size_t bytes = 0;
    double* d = nullptr;
    int st = upload(t->row_norm, &d, &bytes, err);
    if (st) {
      if (d) (void)hipFree(d);
      return st;
    }
    t->d_row_norm = d;
  }
  *out = t->d_row_norm;
  return HOBO_OK;
}

int get_terms(Tensor* t, TermsDev** out, std::string* err) {
  std::lock_guard<std::mutex> lock(t->mu);
  if (t->terms) {
    *out = t->terms.get();
    return HOBO_OK;
  }
  std::unique_ptr<TermsDev> td(new TermsDev());
  const int nm = t->n_mono();
  std::vector<TermRec> rec((size_t)nm);
  for (int m = 0; m < nm; ++m) {
    TermRec r{};
    int len = (int)(t->mono_ptr[m + 1] - t->mono_ptr[m]);
    const uint8_t* s = t->mono_idx.data() + t->mono_ptr[m];
    for (int j = 0; j < 7; ++j) r.idx[j] = j < len ? s[j] : s[0];
    r.len = (uint8_t)len;
    if (t->integer)
      r.w.i = t->w_i[m];
    else
      r.w.f = t->w_f[m];
    rec[(size_t)m] = r;
  }
  td->n_mono = nm;
  int st = upload(rec, &td->d_rec, &td->bytes, err);
  if (st) return st;
  *out = td.get();
  t->terms = std::move(td);
  return HOBO_OK;
}

}  // namespace hobo
