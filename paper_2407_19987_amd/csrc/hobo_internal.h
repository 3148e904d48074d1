// Internal declarations shared by the host-side C++ files and the HIP kernels
// of the HOBO engine.  Nothing here is part of the public C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

namespace hobo {

// ------------------------------------------------------------------ limits
constexpr int kMaxVars = 256;      // bits of one replica fit in 32 bytes
constexpr int kMaxOrder = 7;       // a monomial record holds at most 7 variables
constexpr int kRunWidth = 8;       // variables per run (one byte of bits)
constexpr int kTileCols = 16;      // MFMA 16x16 output tile width

// precision modes (values match the public header)
enum Prec : int { P_FP32 = 0, P_BF16X2 = 1, P_BF16X3 = 2, P_INT8X4 = 3, P_FP64 = 4, P_FP16X2 = 5 };
// the precisions with tiled matrix-core layouts
inline bool tiled_prec(int p) { return (p >= P_FP32 && p <= P_INT8X4) || p == P_FP16X2; }

// layouts a coefficient matrix can be packed for
enum Mode : int { M_FIELDS = 0, M_ENERGY = 1, M_SLABS = 2, M_BLOCKS = 3 };

// runs per chunk: one MFMA K-step covers 4 runs (32 rows) for FP32/BF16 and
// 8 runs (64 rows) for INT8
inline int runs_per_chunk(int prec) { return prec == P_INT8X4 ? 8 : 4; }
// bytes of one 16-column tile of one chunk, all passes / limbs included
inline int tile_bytes(int prec) {
  switch (prec) {
    case P_FP32: return 64 * 8 * 4;
    case P_BF16X2: return 2 * 64 * 8 * 2;
    case P_BF16X3: return 3 * 64 * 8 * 2;
    case P_FP16X2: return 2 * 64 * 8 * 2;
    case P_INT8X4: return 4 * 64 * 16;
    default: return 0;
  }
}

// A run is eight consecutive candidate monomials P u {m}, m = 8*beta .. 8*beta+7,
// sharing a prefix P (sorted, all < m).  Descriptor bit fields (uint64):
//   byte 0      beta (block of eight variables)
//   byte 1      number of prefix variables, or kRunConst / kRunNull
//   bytes 2..7  prefix variables
constexpr uint32_t kRunConst = 0xFE;  // constant monomial: only element 0 is 1
constexpr uint32_t kRunNull = 0xFF;   // padding: every element is 0

struct ChunkMeta {   // one K-step worth of runs (4 or 8)
  uint32_t tile_off; // offset of the chunk's first tile, in tiles
  uint8_t t_lo;      // first 16-column tile with a non-zero coefficient
  uint8_t t_hi;      // one past the last such tile
  uint8_t seg_end;   // fields layout: all monomials of order <= seg_end are done after this chunk;
                     // slab layout: 1 on the last chunk of a variable's slab
  uint8_t bit;       // slab layout: the variable whose slab holds this chunk
};

struct SlabMeta {     // annealer: per-variable slab of the local field
  uint32_t chunk0;    // first chunk of this variable's slab
  uint32_t nchunks;
  uint32_t run0;      // first run descriptor (chunk c of the slab uses runs run0 + rpc*c ...)
  uint32_t pad;
  double a_f;         // linear coefficient w_{i}
  int64_t a_i;
};

// Blocked annealer: variables in blocks of 16.  For block q (variables
// J = 16q .. 16q+15) list 0 is the field matrix of the block's 16 columns
// (rows: monomials of order <= k-1 with no variable of J, and the pairs
// inside J with the entry negated; the kernel adds sum_b x_b H_ab for the
// rest), lists 1..8 are the pair matrices of the
// 120 pairs (a, b) of J, 16 pairs per list (rows: monomials of order <= k-2,
// entry w_{row u {a, b}}), and the block's 16x16x16 table holds the order-3
// coefficients w_{abc} of triples inside J.  Every chunk of these lists has
// exactly one tile: chunk c's tile is tile 1 + c of the tile buffer.
constexpr int kBlockBits = 16;
constexpr int kBlockLists = 9;
constexpr int kPairTiles = 8;
struct BlockMeta {
  uint32_t chunk0[kBlockLists];   // first chunk of each list
  uint32_t nchunks[kBlockLists];  // chunks of each list
  uint32_t nbits;                 // variables in the block (16, fewer in the last)
  uint32_t npt;                   // pair lists in use (ceil(C(nbits,2) / 16))
  uint32_t nearly;                // leading chunks of the field list that read no bit of the
                                  // block before it in a sweep (block q-1, or the last for q = 0)
};
// Blocked annealer work schedule.  For a work-group of nw waves (wave 0
// decides; with 16 waves wave 1 stages; the other NS stream) each block's
// chunks are dealt to the NS streaming waves as whole rounds of kBlockRing
// slots: first the early part (field chunks that read no bit of the block
// before), then the late part (the other field chunks, then the wave's pair
// tiles).  One 32-bit word per slot: tile index (chunk + 1, 0 = the zero
// tile) in bits 0..19, kind in bits 20..21 (0 chunk, 1 chunk that closes
// its list, 2 padding, 3 past the last block), target list in bits 22..25
// (0 fields, 1 + t pair tile t).  Header per (block, wave): word offset of
// its slots, then (early slots << 16) | slots.
constexpr int kBlockRing = 8;
constexpr uint32_t kSlotPad = 2u << 20, kSlotEnd = 3u << 20;
inline int block_streamers(int nw) { return nw - 1 - (nw == 16 ? 1 : 0); }
struct BlockSchedule {
  uint32_t* d_words = nullptr;
  uint32_t* d_hdr = nullptr;  // [nblocks][NS][2]
  ~BlockSchedule();
};

// pair (a, b), a < b < 16, of a block -> its column among the 120 pair columns
__host__ __device__ inline int pair_col(int a, int b) { return b * (b - 1) / 2 + a; }

// Device-resident packed matrix for one (mode, precision).
struct Packed {
  int mode = 0, prec = 0;
  int nchunks = 0;          // fields/energy: number of chunks
  int ntiles = 0;           // tiles stored
  int n_col_tiles = 0;
  void* d_tiles = nullptr;  // tile_bytes(prec) * ntiles
  ChunkMeta* d_chunks = nullptr;
  uint64_t* d_runs = nullptr;
  SlabMeta* d_slabs = nullptr;  // slabs mode only, [n_vars]
  BlockMeta* d_blocks = nullptr;  // blocks mode only, [nblocks]
  float* d_triples = nullptr;     // blocks mode only, [nblocks][16][16][16] w_{abc} at [c][a][b]
  int nblocks = 0;
  // FP16X2: the tiles (and the blocked layout's order-3 table) hold every
  // coefficient times 2^scale_exp, so that the largest one sits just below
  // 2^15 and the FP16 pair keeps 22 significant bits over the whole range;
  // the kernels multiply their sums by 2^-scale_exp (exact).  0 otherwise.
  int scale_exp = 0;
  std::vector<BlockMeta> h_blocks;  // blocks mode only
  std::map<int, std::unique_ptr<BlockSchedule>> sched;  // blocks mode: key = nw * 2 + masked
  std::vector<ChunkMeta> h_chunks;
  size_t bytes = 0;
  ~Packed();
};

// Flat monomial list for the FP64 / int64 term-loop kernels.
struct TermRec {          // one canonical monomial for the term-loop kernels
  uint8_t idx[7];         // variables (unused slots repeat idx[0])
  uint8_t len;
  union { double f; int64_t i; } w;
};
struct TermsDev {
  int n_mono = 0;
  TermRec* d_rec = nullptr;
  size_t bytes = 0;
  ~TermsDev();
};

struct Tensor {
  int n_vars = 0;
  int order = 0;
  bool integer = false;
  int device = 0;
  // canonical monomials: sorted distinct variables, non-zero weight
  std::vector<int64_t> mono_ptr;  // [n_mono+1]
  std::vector<uint8_t> mono_idx;
  std::vector<int64_t> w_i;  // integer weights (integer instances)
  std::vector<double> w_f;   // weights as double (both kinds)
  int64_t offset_i = 0;
  double offset_f = 0.0;
  std::vector<int64_t> n_per_order;  // [order+1]
  unsigned __int128 abs_sum = 0;     // integer tensors: sum |w| (exact)
  unsigned __int128 var_abs_max = 0; // integer tensors: max over variables i of sum |w| over monomials with i
  int64_t w_lo = 0, w_hi = 0;        // integer tensors: smallest and largest weight
  double row_norm_max = 0.0;
  std::vector<double> row_norm;  // ||H_i||_2 over monomials containing i

  std::mutex mu;
  std::map<int, std::unique_ptr<Packed>> packed;  // key = mode*16 + prec
  std::unique_ptr<TermsDev> terms;
  std::unique_ptr<struct GDDev> gd;  // gradient-descent records (built on first use)
  double* d_row_norm = nullptr;  // device copy of row_norm (uploaded on first use)
  // autotuned launch shapes (hobo_autotune): key = (kernel << 16) | (prec << 8) | ceil(log2 B)
  std::map<uint32_t, int> tuned;
  ~Tensor();
  int n_mono() const { return (int)(mono_ptr.size() - 1); }
};

// kernels with tuned shapes
enum TuneKernel : int { TK_FIELDS = 1, TK_ENERGY = 2, TK_ANNEAL = 3 };
inline uint32_t tune_key(int kernel, int prec, int64_t B) {
  int bc = 0;
  while (bc < 62 && ((int64_t)1 << bc) < B) ++bc;
  return ((uint32_t)kernel << 16) | ((uint32_t)prec << 8) | (uint32_t)bc;
}

// ------------------------------------------------------------------ status
struct Error {
  int code;
  std::string msg;
};

// canon.cpp
int canonicalize(int n_vars, int max_order, int64_t n_terms, const int64_t* term_ptr,
                 const int32_t* term_idx, const void* coeff, int coeff_type, Tensor* t,
                 std::string* err);

// tt.cpp / tt_kernels.hip -- tensor-train form of the HOBO tensor: cores
// G_k [r_{k-1}][n][r_k] (row-major, concatenated), r_0 = r_d = 1
constexpr int kTTMaxRank = 32;
constexpr size_t kTTMaxDense = (size_t)1 << 24;  // entries of the dense tensor it is built from
struct TTDev {
  int n = 0, order = 0;
  std::vector<int> ranks;         // [order + 1]
  std::vector<int64_t> core_off;  // [order] offsets (in doubles) of the cores
  std::vector<double> h_cores;
  double* d_cores = nullptr;       // device copy, made on first use
  std::mutex mu;
  ~TTDev();
};
int tt_decompose(const Tensor* t, std::unique_ptr<TTDev>* out, std::string* err);
int tt_upload(TTDev* tt, std::string* err);
int launch_tt_energy(const TTDev* tt, const uint64_t* bits, int64_t B, double* e_out, void* stream,
                     std::string* err);

// gd.cpp / gd_kernels.hip -- projected gradient descent on the multilinear
// extension.  Per variable i, one record per monomial S containing i: its
// weight and the other variables of S (ascending), in monomial order.
struct GDRec {
  double w;
  uint8_t n;       // other variables (|S| - 1)
  uint8_t o[7];
};
struct GDDev {
  int n_vars = 0;
  int32_t* d_ptr = nullptr;  // [n_vars + 1] record offsets per variable
  GDRec* d_rec = nullptr;
  size_t bytes = 0;
  ~GDDev();
};
int get_gd(Tensor* t, GDDev** out, std::string* err);
struct GDArgs {
  const int32_t* ptr;   // device copies of the GDDev arrays
  const GDRec* rec;
  int n_vars;
  int64_t B;
  const double* p_in;   // [N][B]
  double* p_out;        // [N][B]: the projected step (mode 0) or the gradient (mode 1)
  double eta;
  int mode;
  int max_order;        // largest monomial order of the tensor
  void* stream;
};
int launch_gd_step(const GDArgs& a, std::string* err);
int launch_gd_init(int n_vars, int64_t B, uint64_t seed, double* p, void* stream, std::string* err);
int launch_gd_round(int n_vars, int64_t B, const double* p, uint64_t* x, void* stream, std::string* err);

// results.cpp -- unique states of a batch (host buffers), ordered by energy
// then by the bit sequence x_0, x_1, ...; per unique state the first replica
// holding it and its number of replicas
int aggregate_states(int n_vars, int64_t B, const uint64_t* x_bits, const void* energies, int is_integer,
                     int64_t* n_unique, int64_t* rep_out, int64_t* count_out, std::string* err);

// pack.cpp -- whether a precision can represent the tensor exactly enough
// (host-only checks: INT8X4 needs an integer tensor whose digit and energy
// sums fit; FP32 / BF16 on an integer tensor need sum |w| < 2^24)
int check_prec(const Tensor* t, int prec, std::string* err);
// pack.cpp -- build (once) the packed layout; returns a status code
int get_packed(Tensor* t, int mode, int prec, Packed** out, std::string* err);
// the blocked annealer's schedule for nw-wave work-groups (built on first use)
int get_block_schedule(Tensor* t, Packed* pk, int nw, bool masked, const BlockSchedule** out, std::string* err);
// the schedule's slot words and per-(block, wave) headers for NS streaming
// waves (host only; get_block_schedule uploads them)
void build_block_schedule(const std::vector<BlockMeta>& blocks, int ns, bool masked, std::vector<uint32_t>* words,
                          std::vector<uint32_t>* hdr);
int get_terms(Tensor* t, TermsDev** out, std::string* err);
int get_row_norms(Tensor* t, const double** out, std::string* err);

// mlp_kernels.hip -- the learned flip proposal
int mlp_forward(const float* params, const float* feats, long long M, float* logits, hipStream_t st,
                std::string* err);
size_t mlp_train_workspace(int batch);
int mlp_train_step(float* state, const float* feats, const float* labels, long long m0, int mb, float lr,
                   float beta1, float beta2, float eps, float bc1, float bc2, float* part, float* loss_out,
                   hipStream_t st, std::string* err);
int mlp_grad(const float* params, const float* feats, const float* labels, int mb, float* part, float* grad,
             float* loss_out, hipStream_t st, std::string* err);
int proposal_features(const unsigned long long* x, const unsigned long long* xa, long long B, int N, const void* de,
                      int de_int, double beta, const double* rnorm, float* feats, float* labels, hipStream_t st,
                      std::string* err);
int proposal_masks(const float* params, const unsigned long long* x, long long B, int N, const void* de, int de_int,
                   double beta, const double* rnorm, float lthr, double p_floor, unsigned long long seed,
                   unsigned long long inst, int s0, int nsw, unsigned char* mask, hipStream_t st, std::string* err);

// kernels.hip -- launchers (return hipError_t as int)
struct EvalArgs {
  const Packed* pk;
  const Tensor* t;
  const uint64_t* bits;
  int64_t B;
  void* de_out;   // fields: [B][N] float or int64 (may be null)
  void* e_out;    // double[B] or int64[B] (may be null)
  void* work;     // partial sums [ncg][order][B] (double or int64)
  int rt, ct;     // tile shape
  void* stream;
};
int launch_eval(const EvalArgs& a, std::string* err);
size_t eval_workspace_bytes(const Tensor* t, int mode, int64_t B, int ct);

// no-allocation entry point: size of the per-GPU scratch array, its device
// address on the current device (resolved once per device), and a zero fill
// kernel (no hipMemsetAsync, so that callers may capture the call)
constexpr size_t kNoallocScratchBytes = (size_t)32 << 20;
int noalloc_scratch(void** out, std::string* err);
int launch_zero_u64(void* p, long long n, void* stream, std::string* err);

struct TermArgs {
  const TermsDev* td;
  const Tensor* t;
  const uint64_t* bits;
  int64_t B;
  void* e_out;  // double or int64
  void* work;   // term_workspace_bytes
  void* stream;
};
int launch_term_energy(const TermArgs& a, std::string* err);
size_t term_workspace_bytes(const Tensor* t, int64_t B);

// ---------------------------------------------------------------- annealer
struct AnnealInstDev {       // per-instance view of the annealing kernel
  const unsigned char* tiles;
  const ChunkMeta* chunks;
  const unsigned long long* runs;
  const SlabMeta* slabs;
  unsigned long long* x;       // [W][B] current states (in/out)
  unsigned long long* best_x;  // [W][B] best states (out)
  double* e_track;             // [B] tracked energy (in: start energy, out: final)
  double* best_track;          // [B] tracked best energy
  double* trace_part;          // [ntiles16][S] per-tile minima, or null
  const unsigned char* attempt;  // [ntiles16][S][N] attempt masks, or null
  long long B;
  int n_vars, W;
  int integer;
  int n_chunks;                // chunks of all slabs (one sweep)
  unsigned long long inst_id;
  unsigned n_tiles;            // tiles stored in the packed buffer
  unsigned pad2;
  double inv_scale;            // 2^-scale_exp of the packed layout (1 unless FP16X2)
  const BlockMeta* blocks;     // blocked layout: [nblocks]
  const float* triples;        // blocked layout: [nblocks][16][16][16]
  const uint32_t* sched;       // blocked layout: slot words of the launch's group width
  const uint32_t* sched_hdr;   // and their headers [nblocks][NS][2]
  double* unif;                // blocked layout: -log(u) of a launch window,
                               // [ntiles16][window sweeps][nblocks][16 replicas][16 bits]
  int nblocks;
  int pad3;
};
struct AnnealItem { int inst; int tile16; };  // 16 replicas of one instance

struct InstSmall {            // per-instance view for the setup / finish kernels
  const TermRec* rec;
  int n_mono;
  int n_vars;
  int W;
  int integer;
  long long B;
  long long rep_off;
  unsigned long long* x;
  unsigned long long* best_x;
  double* e_track;
  double* best_track;
  void* best_out;             // double* or long long*, already offset
  const double* trace_part;   // [ntiles16][S]
  double* trace_out;          // [S] or null
  unsigned long long inst_id;
  int ntiles16;
  int pad;
  void* term_part;            // [term groups][B] partial sums of the term-loop energies
};

struct AnnealTables {         // device tables of one anneal call
  AnnealInstDev* d_inst = nullptr;
  AnnealItem* d_items = nullptr;
  InstSmall* d_small = nullptr;
  double* d_beta = nullptr;
  const unsigned char* d_ones = nullptr;  // one byte equal to 1
  int n_items = 0;
  long long max_B = 0;
  int max_W = 0;
  int max_groups = 1;         // term-loop groups of the largest instance
  int unif_sweeps = 0;        // sweeps of one blocked launch window the uniform buffers hold
};

// (column tiles per wave, waves per work-group) of the annealer for T column tiles
void anneal_shape(int T, int cs_req, int* ctw, int* cs);
// sweeps per blocked-kernel launch with attempt masks / without
int anneal_mask_window();
int anneal_sweep_window();

// launch timing (kernels: 0 = annealer, 1 = fields, 2 = energy)
void timing_enable(int on);
int timing_read(int kernel, double* total_ms, int64_t* launches);
// One launch sequence of hobo_anneal_batch: items [item0, item0 + n_blk) run
// the blocked kernel, the next n_slab items the per-bit slab kernel.
struct AnnealPlan {
  int sweeps = 0;       // sweeps of the call
  int s_first = 0;      // global index of its first sweep
  uint64_t seed = 0;
  int init_random = 0;
  int cont = 0;         // best state continues from best_x (rescored at the start)
  int masked = 0;       // attempt masks present
  int prec = 0;
  int ct = 1, nw = 1;   // slab kernel: column tiles per wave, waves per work-group
  int nw_blk = 4;       // blocked kernel: waves per work-group
  int item0 = 0, n_blk = 0, n_slab = 0;
  int inst0 = 0, ninst = 0;
};
int enqueue_anneal_seq(const AnnealTables& tb, const AnnealPlan& pl, void* stream, std::string* err);
int enqueue_anneal_setup(const AnnealTables& tb, const AnnealPlan& pl, void* stream, std::string* err);
int enqueue_anneal_sweeps(const AnnealTables& tb, const AnnealPlan& pl, int s_begin, int s_end, int mask_s0,
                          int mask_rows, int cont, void* stream, std::string* err);
int enqueue_anneal_finish(const AnnealTables& tb, const AnnealPlan& pl, void* stream, std::string* err);

}  // namespace hobo
