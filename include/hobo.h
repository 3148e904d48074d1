/*
 * hobo.h -- C-ABI of the MI355X (gfx950) HOBO engine.
 *
 * The engine evaluates higher-order binary optimisation (HOBO) objectives
 *     f(x) = offset + sum_S w_S prod_{i in S} x_i,   x in {0,1}^N,
 * (HOBOTAN, arXiv 2407.19987, Sec. II.B: the QUBO form with terms a_i x_i and
 * b_ij x_i x_j, extended by c_ijk x_i x_j x_k and higher orders) for large
 * batches of candidate bit vectors, and searches them with batched
 * single-flip Metropolis annealing (Sec. II.D.1).  The paper stores the
 * coefficients as an order-k tensor whose lower-order terms repeat their
 * smallest index (Sec. III.C, IV.A) and contracts it with a matrix of many
 * candidate vectors at once (Sec. IV.C, the "tensor batch system");
 * hobo_energy computes exactly that contraction, row by row.
 *
 * Conventions
 * -----------
 * - Every function returns a hobo_status (0 = HOBO_OK).  No exception or
 *   signal crosses the ABI.  hobo_last_error() returns a thread-local
 *   description of the last failure on the calling thread.
 * - All argument checks happen before any HIP call, so invalid arguments
 *   never reach the GPU.
 * - Bit vectors are uint64 words in [W][B] order, W = ceil(N/64): variable i
 *   of row b is bit (i & 63) of word x_bits[(i >> 6) * B + b].  Bits at or
 *   above N in the last word must be zero.
 * - Device buffers (x_bits, outputs) are allocated by the caller and must be
 *   device memory of the current HIP device.  All device work is enqueued on
 *   the caller's stream (a hipStream_t passed as void*, NULL = default
 *   stream); results are valid once the caller synchronises that stream.
 * - A hobo_tensor is owned by the library until hobo_free_tensor.  It is
 *   immutable once built, except that device layouts are created on first use
 *   of a (function, precision) pair; that first use blocks the host and must
 *   not happen during stream capture -- call hobo_tensor_prepare first.
 * - Energies exclude the constant offset (the paper prints the energy
 *   without it); the offset is returned by hobo_build_tensor.
 * - Limits: 1 <= N <= 256 variables, order <= 7, B >= 1.
 */
#ifndef HOBO_H
#define HOBO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hobo_status;
enum {
  HOBO_OK = 0,
  HOBO_ERR_INVALID_ARG = 1, /* null pointer, bad size, index out of range */
  HOBO_ERR_ORDER = 2,       /* order above max_order or above the engine limit */
  HOBO_ERR_RANGE = 3,       /* integer instance not exactly representable */
  HOBO_ERR_PRECISION = 4,   /* precision not valid for this tensor / function */
  HOBO_ERR_NO_DEVICE = 5,   /* no HIP device */
  HOBO_ERR_OOM = 6,         /* device allocation failed */
  HOBO_ERR_HIP = 7,         /* a HIP runtime call failed */
  HOBO_ERR_UNSUPPORTED = 8  /* valid request the engine does not implement */
};

/* coefficient types */
enum { HOBO_COEFF_INT64 = 0, HOBO_COEFF_F64 = 1 };

/* arithmetic of the contraction kernels
 *  FP32   : FP32 coefficients, FP32 matrix-core products and sums
 *  BF16X2 : coefficient c (rounded to FP32) split as hi = bf16(c),
 *           lo = bf16(c - hi); two BF16 matrix-core passes, FP32 sums
 *  BF16X3 : three-way split hi + mid + lo (exact for normal FP32 values)
 *  INT8X4 : integer coefficients as four balanced base-256 digits in
 *           [-128, 127]; INT8 matrix-core products, int32 per-digit sums,
 *           recombined exactly in int64.  Integer tensors only.
 *  FP64   : double-precision term-by-term sums (hobo_energy only; used to
 *           rescore states)
 *  FP16X2 : coefficient c (rounded to FP32) times a per-tensor power of two
 *           2^e (the largest |c| 2^e in [2^14, 2^15)) split as
 *           hi = fp16(c 2^e), lo = fp16(c 2^e - hi); two FP16 matrix-core
 *           passes at the BF16 rate, FP32 sums multiplied by 2^-e (exact).
 *           About 22 significant bits per coefficient (error at most
 *           2^-22 |c|), against 16 for BF16X2, for every |c| above 2^-17
 *           times the largest |c|; smaller coefficients keep an absolute
 *           error below 2^-39 times the largest.  Same tile size and speed
 *           as BF16X2. */
enum {
  HOBO_PREC_FP32 = 0,
  HOBO_PREC_BF16X2 = 1,
  HOBO_PREC_BF16X3 = 2,
  HOBO_PREC_INT8X4 = 3,
  HOBO_PREC_FP64 = 4,
  HOBO_PREC_FP16X2 = 5
};

typedef struct hobo_tensor hobo_tensor;

typedef struct {
  int32_t n_vars;
  int32_t order;
  int32_t is_integer;
  int32_t reserved;
  int64_t n_monomials;
  int64_t n_per_order[8]; /* monomials of each order 0..7 (order 0 always 0) */
  int64_t offset_i64;     /* offset of an integer tensor */
  double offset_f64;      /* offset as double (both kinds) */
  int64_t device_bytes;   /* device memory held by the tensor's layouts */
} hobo_tensor_info;

/* Build a tensor from a raw term list (HOBOTAN Sec. III.C / IV.A compile step).
 *  n_vars     : N, 1..256; variables are 0..N-1 (drop unused variables first,
 *               Sec. IV.D)
 *  max_order  : 0 = infer; otherwise HOBO_ERR_ORDER if the instance is larger
 *  n_terms    : number of terms (>= 0)
 *  term_ptr   : host int64[n_terms+1], CSR offsets into term_idx, term_ptr[0] = 0
 *  term_idx   : host int32 variable indices; repeats inside a term collapse
 *               (x*x = x); an empty term is a constant and goes to the offset
 *  coeff      : host int64[n_terms] (HOBO_COEFF_INT64) or double[n_terms]
 *               (HOBO_COEFF_F64); duplicate monomials are summed, zero sums
 *               dropped
 *  out        : receives the new handle (unchanged on error)
 *  offset_out : host int64* (integer) or double* (real), may be NULL
 * Integer sums that overflow int64 give HOBO_ERR_RANGE. */
hobo_status hobo_build_tensor(int32_t n_vars, int32_t max_order, int64_t n_terms,
                              const int64_t* term_ptr, const int32_t* term_idx, const void* coeff,
                              int32_t coeff_type, hobo_tensor** out, void* offset_out);

/* Release a tensor and all its device memory (NULL is accepted). */
hobo_status hobo_free_tensor(hobo_tensor* t);

/* Host-side description of a tensor. */
hobo_status hobo_tensor_info_get(const hobo_tensor* t, hobo_tensor_info* info);

/* Copy the canonical monomials to the host: mono_ptr int64[n_monomials+1],
 * mono_idx int32[mono_ptr[n]], weights int64 (integer) or double (real).
 * Each array may be NULL to skip it; capacities are checked. */
hobo_status hobo_tensor_monomials(const hobo_tensor* t, int64_t* mono_ptr, int64_t ptr_cap,
                                  int32_t* mono_idx, int64_t idx_cap, void* weights,
                                  int64_t w_cap);

/* Dense N^k tensor in the paper's layout (Sec. III.C): a monomial of size
 * r < k is stored at the index tuple that repeats its smallest variable
 * k - r + 1 times followed by its other variables in increasing order; all
 * other entries are 0.  host_out: int64 or double [N^k], row-major, with
 * N^k <= capacity and N^k <= 2^26. */
hobo_status hobo_tensor_export_dense(const hobo_tensor* t, void* host_out, int64_t capacity);

/* Matrix-core work of one device layout, for measurement: the layout that
 * hobo_energy (fn 1), hobo_local_fields (fn 2) or hobo_anneal_batch (fn 4,
 * the blocked layout where it applies, else the per-bit one) uses for
 * `precision`, created on first use (blocks the host).  issued_flops counts
 * every 16-column coefficient tile the kernels multiply for one replica
 * (one evaluation, or one annealing sweep): tiles x 16 columns x K rows
 * (32, or 64 for INT8X4) x 2 x passes (1 FP32, 2 BF16X2 / FP16X2,
 * 3 BF16X3, 4 INT8X4 digits); zero entries inside stored tiles count, absent
 * tiles do not. */
typedef struct {
  int64_t chunks;       /* K steps of the layout */
  int64_t tiles;        /* stored coefficient tiles (the shared zero tile excluded) */
  int64_t issued_flops; /* matrix-core flops (or int ops) issued per replica */
  int64_t bytes;        /* device bytes of the layout */
} hobo_layout_info;
hobo_status hobo_tensor_layout_info(hobo_tensor* t, int32_t fn, int32_t precision, hobo_layout_info* out);

/* Create the device layouts of `t` for the functions in `fn_mask`
 * (1 = hobo_energy, 2 = hobo_local_fields, 4 = hobo_anneal_batch) and the
 * precisions in `prec_mask` (bit p = precision p).  Blocks the host. */
hobo_status hobo_tensor_prepare(hobo_tensor* t, uint32_t fn_mask, uint32_t prec_mask);

/* Batched energies E_b = sum_S w_S prod_{i in S} x_{b,i} (offset excluded),
 * the paper's batch contraction (Sec. IV.C) of its HOBO tensor (Sec. II.C).
 *  x_bits    : device uint64 [W][B]
 *  B         : rows, >= 1
 *  precision : FP32 | BF16X2 | BF16X3 | FP16X2 | INT8X4 (integer tensors) | FP64
 *  e_out     : device int64[B] for integer tensors, double[B] for real ones
 *  stream    : hipStream_t */
hobo_status hobo_energy(const hobo_tensor* t, const uint64_t* x_bits, int64_t B,
                        int32_t precision, void* e_out, void* stream);

/* hobo_energy without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and kernels as hobo_energy.
 * Its workspace is a per-GPU scratch array of 32 MiB inside the library,
 * held until the process ends; the batch is refused (HOBO_ERR_INVALID_ARG)
 * when it needs more (tiled precisions: 8 B x max(16-column tiles, column
 * groups) x B, e.g. B <= 524288 at N = 128; FP64: 8 B x ceil(monomials /
 * 4096) x B plus the replica masks).  The tensor's layout for the precision
 * must already be on the device (hobo_tensor_prepare with fn 1 and the
 * precision's bit), else HOBO_ERR_INVALID_ARG.  Every call on a GPU shares
 * that GPU's scratch: calls that overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller.  No hipMemsetAsync
 * is issued, so the call may be captured into a graph (with
 * hobo_timing_enable off). */
hobo_status hobo_energy_noalloc(const hobo_tensor* t, const uint64_t* x_bits, int64_t B, int32_t precision,
                                void* e_out, void* stream);

/* Batched single-flip energy changes dE_{b,i} = f(x_b xor e_i) - f(x_b)
 * = (1 - 2 x_{b,i}) g_{b,i}, with the local field
 * g_{b,i} = sum_{S containing i} w_S prod_{j in S, j != i} x_{b,j},
 * the quantity the Metropolis search (Sec. II.D.1) needs for every bit.
 *  precision : FP32 | BF16X2 | BF16X3 | FP16X2 | INT8X4 (integer tensors)
 *  de_out    : device [B][N] row-major: int64 for integer tensors, float
 *              otherwise
 *  e_out     : optional device energies (as in hobo_energy), computed from
 *              the per-order fields with Euler's identity
 *              sum_i x_i g_i^(r) = r E^(r). */
hobo_status hobo_local_fields(const hobo_tensor* t, const uint64_t* x_bits, int64_t B,
                              int32_t precision, void* de_out, void* e_out, void* stream);

/* ------------------------------------------------------------- annealing */
enum { HOBO_INIT_RANDOM = 0, HOBO_INIT_GIVEN = 1 };
enum { HOBO_PROPOSAL_METROPOLIS = 0, HOBO_PROPOSAL_MASKED = 1, HOBO_PROPOSAL_LEARNED = 2 };
enum { HOBO_LAUNCH_PER_INSTANCE = 0, HOBO_LAUNCH_PERSISTENT = 1, HOBO_LAUNCH_GRAPH = 2 };
/* annealing kernels: AUTO picks BLOCKS where it applies (order <= 3, FP32 /
 * BF16X2 / BF16X3 / FP16X2, and for integer tensors 3 x the largest sum |w|
 * over the monomials of one variable below 2^24, so that its FP32 fields stay
 * exact), else SLABS.  Both run the same chain.  BLOCKS asked for where it
 * does not apply: HOBO_ERR_UNSUPPORTED (order, precision) or HOBO_ERR_RANGE
 * (the integer bound). */
enum { HOBO_ANNEAL_AUTO = 0, HOBO_ANNEAL_SLABS = 1, HOBO_ANNEAL_BLOCKS = 2 };

typedef struct {
  int32_t sweeps;      /* sweeps of this call, >= 0 */
  int32_t precision;   /* FP32 | BF16X2 | BF16X3 | FP16X2 | INT8X4 */
  double t_start;      /* T_0 > 0 */
  double t_end;        /* T_{L-1} > 0; T_s = T_0 (T_end/T_0)^(s/(L-1)), L = schedule length */
  uint64_t seed;
  int32_t init;        /* HOBO_INIT_RANDOM or HOBO_INIT_GIVEN */
  int32_t proposal;    /* METROPOLIS, MASKED (attempt masks) or LEARNED (network) */
  const uint8_t* attempt; /* MASKED: device uint8 [ceil(B/16)][sweeps][N] per instance,
                             concatenated; 1 = the 16-replica group visits the bit */
  int32_t waves_per_block; /* waves sharing 16 replicas (1, 2, 4, 8, 16); 0 = default
                              (the autotuned width, else 16 up to 256 groups of 16
                              replicas in the call, 8 above).  The per-bit kernel uses
                              at most 8, the blocked one at least 2.  Integer results
                              do not depend on it; for real coefficients the blocked
                              kernel's width sets how its FP32 partial fields are
                              grouped, so decisions within rounding of a tie may
                              differ between widths. */
  int32_t algorithm;   /* HOBO_ANNEAL_AUTO | SLABS | BLOCKS */
  int32_t first_sweep; /* this call runs sweeps first_sweep .. first_sweep+sweeps-1;
                          consecutive windows of one schedule with the same
                          buffers reuse one setup (PER_INSTANCE / PERSISTENT),
                          so such calls must be ordered, as their shared
                          buffers already require */
  int32_t schedule_sweeps; /* L, length of the whole schedule; 0 = sweeps (first_sweep
                              must then be 0) */
  int32_t continue_best; /* 1: the best states start from best_x_out (their energies
                            are recomputed) instead of the start states */
  int32_t refresh;     /* LEARNED: sweeps per proposal segment, >= 1 */
  const float* mlp;    /* LEARNED: device FP32 parameter vector (hobo_mlp_forward) */
  float tau;           /* LEARNED: a tile attempts bit i iff some replica has p_i >= tau */
  float p_floor;       /* LEARNED: ... or a floor draw u < p_floor (p_floor = 1: plain) */
} hobo_anneal_params;

/* Batched single-flip Metropolis simulated annealing (Sec. II.D.1) over one
 * or several instances.  Replica b of instance j:
 *   - initial state: x_inout (GIVEN) or bit i = top bit of Philox4x64-10 word
 *     i%4 at counter (b, 0, i/4, 1), key (seed, j) (RANDOM);
 *   - sweep s visits variables 0..N-1 in order (skipping the bits a replica's
 *     16-replica group does not attempt in MASKED / LEARNED mode); at
 *     variable i it draws u = (r >> 11) 2^-53 from word i%4 of Philox4x64-10
 *     at counter (b, s, i/4, 0), key (seed, j), computes dE_i in the tensor
 *     precision, and accepts iff dE_i <= 0 or dE_i * beta_s < -ln(u) in
 *     double (the test u < exp(-dE_i beta_s)), with beta_s = 1 / T_s; on
 *     acceptance x_i flips and E += dE_i (double);
 *   - the best state is the initial one (or best_x_out with continue_best),
 *     then after each sweep the current one if its tracked energy is lower.
 * LEARNED: every `refresh` sweeps the library computes each replica's flip
 * changes at its current state, evaluates the network on the features
 * [x_i, beta_s dE_i, beta_s ||H_i||] (hobo_proposal_features) and lets a
 * group attempt bit i during the segment iff some replica's logit is at least
 * logit(tau) or u < p_floor, with u from Philox4x64-10 word i%4 at counter
 * (group, s, i/4, 2), key (seed, j); attempted bits get the exact Metropolis
 * test above.
 *  tensors     : host array of n_instances handles
 *  replicas    : host int64[n_instances], B_j >= 1
 *  x_inout     : device uint64, instance j's [W_j][B_j] block after those of
 *                instances < j; in: initial states (GIVEN), out: final states
 *  best_x_out  : device uint64, same layout: best states
 *  best_e_out  : device, one value per replica (instances concatenated):
 *                exact int64 energies of the best states when every instance
 *                is integer, else double energies recomputed in FP64
 *  trace_out   : optional device double [n_instances][sweeps]: minimum over the
 *                instance's replicas of the tracked best energy after each sweep
 *  launch_mode : PER_INSTANCE (one launch sequence per instance),
 *                PERSISTENT (one persistent launch over all instances), or
 *                GRAPH (the persistent sequence captured once in a hipGraph
 *                and launched from it) -- the same kernels and widths in all
 *                three, so identical results
 * The library keeps the device setup of recent calls (tables, a workspace of
 * up to about 1 GiB of Metropolis uniforms per call, the captured graph), keyed
 * by every argument including the buffer pointers, so a repeated call only
 * launches.  It keeps at most 16 setups, the older ones holding at most 4 GiB;
 * hobo_free_tensor releases the setups that name its tensor. */
hobo_status hobo_anneal_batch(hobo_tensor* const* tensors, int32_t n_instances,
                              const int64_t* replicas, const hobo_anneal_params* params,
                              uint64_t* x_inout, uint64_t* best_x_out, void* best_e_out,
                              double* trace_out, int32_t launch_mode, void* stream);

/* ------------------------------------------------------------- gradient descent */
/* Gradient-descent search (Sec. II.D.2) on the multilinear extension of the
 * energy, E(p) = sum_S w_S prod_{i in S} p_i for p in [0, 1]^N (equal to the
 * energy at binary points), with
 *   g_i(p) = dE/dp_i = sum_{S containing i} w_S prod_{j in S, j != i} p_j
 * (the local field at binary points).  Each replica runs projected
 * full-gradient steps p <- min(1, max(0, p - eta g(p))); the answer is the
 * rounded state x_i = [p_i > 1/2] with its exact energy.  FP64, products
 * and sums rounded separately, contributions summed in monomial order.
 * Continuous points are device double [N][B] (variable-major: p_i of
 * replica b at i * B + b). */
typedef struct {
  int32_t iterations;  /* steps, >= 0 */
  int32_t init;        /* HOBO_INIT_RANDOM: p_i from Philox4x64-10 word i%4 at
                          counter (b, 0, i/4, 3), key (seed, 0), as (r >> 11) 2^-53;
                          HOBO_INIT_GIVEN: p_inout as passed */
  double eta;          /* step size, finite, >= 0 */
  uint64_t seed;
} hobo_gd_params;

/* g_out [N][B] = the gradient at p [N][B] (both device double). */
hobo_status hobo_gd_gradient(const hobo_tensor* t, const double* p, int64_t B, double* g_out, void* stream);

/* Run the steps on B replicas: p_inout (device double [N][B]) ends as the
 * last point, x_out (device uint64 [W][B]) the rounded states, e_out (device
 * int64[B] for integer tensors, double[B] otherwise) their exact energies
 * (offset excluded).  Allocates a workspace of 8 N B bytes plus the energy
 * pass's (stream-ordered). */
hobo_status hobo_gd_batch(const hobo_tensor* t, int64_t B, const hobo_gd_params* params, double* p_inout,
                          uint64_t* x_out, void* e_out, void* stream);

/* ------------------------------------------------------------- tensor train */
/* The tensor-train (TT) form of the HOBO tensor (Sec. VI.E-F): the dense
 * order-k tensor in the paper's layout, H[i_1..i_k] (a monomial of size r < k
 * repeats its smallest variable, Sec. III.C), decomposed without
 * approximation into cores G_j of shape (r_{j-1}, N, r_j), r_0 = r_k = 1, by
 * the paper's sequence of SVDs (reshape, SVD, keep the left factor, carry
 * Sigma V* on); singular values at or below sigma_max * max(rows, cols) *
 * 2^-52 are dropped (the numerical rank).  Energies through the cores,
 * E(x) = prod_j (sum_i x_i G_j[:, i, :]), cost O(k N r^2) per state instead
 * of the dense contraction's O(N^k). */
typedef struct hobo_tt hobo_tt;

/* Decompose t (host work, N^k <= 2^24 entries, every rank <= 32, else
 * HOBO_ERR_UNSUPPORTED; no device needed).  The cores are copied to the
 * current device on the first hobo_tt_energy (which then blocks the host).
 * The handle is the caller's until hobo_tt_free; t may be freed after. */
hobo_status hobo_tt_build(const hobo_tensor* t, hobo_tt** out);
hobo_status hobo_tt_free(hobo_tt* tt);
/* order k, N, ranks [k + 1] (r_0 .. r_k) and the number of core entries;
 * each pointer may be NULL. */
hobo_status hobo_tt_info(const hobo_tt* tt, int32_t* order, int32_t* n_vars, int32_t* ranks, int64_t* n_params);
/* The cores concatenated, G_j row-major [r_{j-1}][N][r_j], host double[n_params]. */
hobo_status hobo_tt_cores(const hobo_tt* tt, double* host_out, int64_t capacity);
/* Energies of B states through the cores (FP64):
 *  x_bits : device uint64 [W][B];  e_out : device double[B] (offset excluded). */
hobo_status hobo_tt_energy(const hobo_tt* tt, const uint64_t* x_bits, int64_t B, double* e_out, void* stream);

/* ------------------------------------------------------------- results */
/* The result list of a sampling run (the paper's Sec. V result blocks: each
 * distinct state found among the `shots` samples, with its energy and number
 * of occurrences, best first).  Host-side, no device work.
 *  n_vars     : N, 1..256
 *  B          : samples (>= 0)
 *  x_bits     : host uint64 [W][B] (the layout of hobo_anneal_batch's outputs)
 *  energies   : host int64[B] (is_integer) or double[B] (no NaN), e.g. the
 *               exact energies hobo_anneal_batch returns for best_x
 *  n_unique   : receives U, the number of distinct states
 *  rep_out    : host int64[B]; rep_out[u] = the first sample holding state u
 *  count_out  : host int64[B]; count_out[u] = the samples holding state u
 * States are ordered by energy (ascending), then by the bit sequence
 * x_0, x_1, ... (lexicographic; the paper leaves the order of equal
 * energies open); samples with equal bits and equal energies are one state. */
hobo_status hobo_aggregate(int32_t n_vars, int64_t B, const uint64_t* x_bits, const void* energies,
                           int32_t is_integer, int64_t* n_unique, int64_t* rep_out, int64_t* count_out);

/* ------------------------------------------------------------- learned proposal */
/* The flip-proposal network: a two-layer perceptron 3 -> 256 -> 1 mapping a
 * bit's features [x_i, beta dE_i, beta ||H_i||] to a flip logit,
 *   h = relu(W1^T f + b1),   logit = W2 . h + b2.
 * The paper's search (Sec. II.D.1) has no learned part; this is the
 * engine's addition, judged by the exact energy.  Parameters are one FP32
 * vector of HOBO_MLP_PARAMS values: W1[f][u] at f*256+u, b1 at 768, W2 at
 * 1024, b2 at 1280.  The forward pass uses W1 and W2 rounded to BF16 (nearest
 * even) and FP32 biases, activations and sums. */
#define HOBO_MLP_PARAMS 1281
#define HOBO_MLP_ROW 1284
#define HOBO_MLP_STATE (3 * HOBO_MLP_ROW) /* params | Adam m | Adam v, rows of 1284 */

/* logits_out[m] for feats [M][3] (device FP32; params device FP32). */
hobo_status hobo_mlp_forward(const float* params, const float* feats, int64_t M, float* logits_out, void* stream);

/* Gradient of the mean binary cross-entropy over all M samples (one
 * minibatch; 1 <= M <= 2^24) with respect to the parameters, evaluated through
 * the BF16-rounded weights: grad_out device FP32 [HOBO_MLP_PARAMS], loss_out
 * optional device FP32 scalar.  The same kernels and summation order as one
 * step of hobo_mlp_train. */
hobo_status hobo_mlp_grad(const float* params, const float* feats, const float* labels, int64_t M, float* grad_out,
                          float* loss_out, void* stream);

typedef struct {
  int32_t batch;   /* samples per minibatch (the last one of an epoch may be shorter) */
  int32_t epochs;
  float lr, beta1, beta2, eps; /* Adam */
  int64_t step0;   /* Adam steps already taken on this state (bias correction) */
} hobo_mlp_train_params;

/* Minibatch training on feats [M][3] and labels [M] (device FP32, labels 0/1)
 * in sample order, one Adam step per minibatch: mean binary cross-entropy
 * softplus(l) - y l, its gradient through the BF16-rounded weights applied
 * to the FP32 master weights (Kingma & Ba bias-corrected Adam), gradient
 * sums in a fixed order (deterministic).  state: device FP32
 * [HOBO_MLP_STATE] = params | m | v, updated in place.  loss_trace: optional
 * device FP32 [epochs * ceil(M / batch)], the minibatch loss before each step. */
hobo_status hobo_mlp_train(float* state, const float* feats, const float* labels, int64_t M,
                           const hobo_mlp_train_params* tp, float* loss_trace, void* stream);

/* Features of every bit of B states before sweep `sweep` of an annealing
 * schedule: feats_out [B][N][3] FP32 = (x_i, beta dE_i, beta ||H_i||) with
 * beta = 1 / T_sweep of the geometric schedule t_start -> t_end over
 * schedule_sweeps sweeps (the schedule hobo_anneal_batch uses), dE from
 * hobo_local_fields (de: device [B][N], int64 for integer tensors, else
 * FP32) and ||H_i|| the Euclidean norm of the coefficients of all monomials
 * containing i.  With x_after (device [W][B]) and labels_out (device FP32
 * [B][N]) also the transition labels [x_i != x_after_i]. */
hobo_status hobo_proposal_features(const hobo_tensor* t, const uint64_t* x_bits, const uint64_t* x_after, int64_t B,
                                   const void* de, double t_start, double t_end, int32_t sweep,
                                   int32_t schedule_sweeps, float* feats_out, float* labels_out, void* stream);

/* Training transitions for the proposal network from a plain annealing run
 * of B replicas (params: the whole schedule in `sweeps`, its temperatures,
 * seed, precision and init; proposal METROPOLIS).  For each sweep r in
 * `record` (host int32, increasing, within the schedule): the features of
 * every (replica, bit) at the start of sweep r, as hobo_proposal_features
 * gives them, into feats_out (device FP32 [n_record][B][N][3]), and the label
 * "the bit changed during sweep r" into labels_out (device FP32
 * [n_record][B][N]).  The chain is the one hobo_anneal_batch runs for the
 * same arguments.  Allocates its state buffers (stream-ordered). */
hobo_status hobo_record_transitions(hobo_tensor* t, int64_t B, const hobo_anneal_params* params,
                                    const int32_t* record, int32_t n_record, float* feats_out, float* labels_out,
                                    void* stream);

/* ------------------------------------------------------------- autotuning */
/* Times every launch shape of the kernels in fn_mask (1 energy: 16*rt
 * replicas x 16*ct columns per wave; 2 fields: same; 4 annealing: waves per
 * 16-replica work-group) for this tensor, precision and batch size on the
 * caller's stream, with x_bits (device [W][B]) as input, and keeps the
 * fastest for later calls with the same kernel, precision and
 * ceil(log2 B).  Results never depend on the shape; only the time does.
 * Blocks the host; not allowed under stream capture.  B <= 2^24.
 * shapes_out: optional host int32[3], the chosen shapes (rt*16+ct, rt*16+ct,
 * waves; 0 = not tuned). */
hobo_status hobo_autotune(hobo_tensor* t, const uint64_t* x_bits, int64_t B, int32_t fn_mask, int32_t precision,
                          int32_t* shapes_out, void* stream);

/* ------------------------------------------------------------- timing */
/* Kernel timing for measurement tools.  While enabled, each launch of the
 * annealing kernel (id 0), the fields kernel (id 1) and the energy kernel
 * (id 2) is bracketed by two HIP events recorded on the caller's stream
 * (not during stream capture).  hobo_timing_read waits for the recorded
 * launches of one kernel, returns their summed duration in milliseconds and
 * their count, and releases them. */
hobo_status hobo_timing_enable(int32_t enable);
hobo_status hobo_timing_read(int32_t kernel, double* total_ms, int64_t* launches);

/* Description of the last error on the calling thread ("" if none). */
const char* hobo_last_error(void);

/* Library version string. */
const char* hobo_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HOBO_H */
