/*
 * qaia.h -- C ABI of libqaia, simulated-bifurcation sampling of
 * multi-objective MaxCut on AMD Instinct MI355X (gfx950).
 *
 * Method: "Multi-Objective Optimization by Quantum-Annealing-Inspired
 * Algorithms" (arXiv 2604.26477).  Each entry point names the passage of the
 * paper that defines what it computes.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every call returns an int32 status (QAIA_OK = 0 or one of the codes
 *    below).  Argument errors are detected on the host before any device
 *    work is enqueued.  qaia_last_error() returns a human-readable detail of
 *    the calling thread's most recent failure.  No C++ exception crosses the
 *    ABI.
 *  - "HOST" pointers are ordinary CPU memory; "DEVICE" pointers are device
 *    memory of the problem's device (for example torch tensors'
 *    data_ptr()).  All buffers are owned by the caller unless stated.
 *  - hip_stream is a hipStream_t (NULL = the legacy default stream).  Device
 *    work is enqueued asynchronously on it; results are valid after the
 *    caller synchronises that stream.  The library allocates no device
 *    memory in qaia_sample, qaia_evaluate or qaia_pareto_filter: their
 *    scratch space is the caller's workspace.
 *  - Edge weights are int32 fixed point: the real weight is
 *    W * 2^(-frac_bits).  Cut values are exact int64 in the same units.
 *  - Spin vectors are packed: uint64 words[ceil(n/64)] per sample, bit i of
 *    word i/64 set  <=>  s_i = -1.
 */
#ifndef QAIA_H
#define QAIA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QAIA_ABI_VERSION 2

/* status codes */
#define QAIA_OK 0
#define QAIA_INVALID_ARGUMENT 1
#define QAIA_UNSUPPORTED 2
#define QAIA_OUT_OF_MEMORY 3
#define QAIA_DEVICE_ERROR 4        /* a HIP call failed */
#define QAIA_OVERFLOW 5            /* an exact integer range bound was exceeded */
#define QAIA_WORKSPACE_TOO_SMALL 6

/* SB variants, section "Simulated Bifurcation with Gaussian noise":
 * phi(x) = x (ballistic) or sgn(x) (discrete). */
#define QAIA_BSB 0
#define QAIA_DSB 1

/* arithmetic of the coupling product J.phi(x) */
#define QAIA_FP32 0 /* float32 everywhere */
#define QAIA_BF16 1 /* discrete SB, dense path: bf16 J (per-objective scaled) x exact +-1, fp32 accumulate */
#define QAIA_FP8 2  /* discrete SB, dense path: fp8 e4m3 J (per-objective scaled) x exact +-1, fp32 accumulate */
/* ballistic or discrete SB on the generated sparse kernel (QAIA_PATH_SPARSE_REG)
 * in IEEE binary16, the half precision of the paper's GPU sampling runs
 * (section "Sampling time advantage"): x, y, the step coefficient, dt a0,
 * dt alpha and the folded edge coefficients are the float32 values of the
 * FP32 form rounded to binary16 (x0 and y0: the float32 draws rounded), every
 * update is a binary16 fused multiply-add in the FP32 form's order, two
 * replicas per lane as packed pairs; read-out and cut evaluation are exact.
 * Built on first use of each variant. */
#define QAIA_FP16 3

/* kernel family; AUTO lets the planner decide.  Each family has size limits;
 * a request for a family past its limit returns QAIA_UNSUPPORTED before
 * anything is queued.  AUTO takes the first that applies: DENSE_STAGED for
 * a BF16/FP8 field, SPARSE_REG, SPARSE_LDS, DENSE_STAGED. */
#define QAIA_PATH_AUTO 0
/* per-graph generated kernel, one replica per lane, state in registers:
 * 2n + num_edges <= 232, FP32 */
#define QAIA_PATH_SPARSE_REG 1
/* generic kernel, one spin per lane, state and adjacency in LDS:
 * n <= 4096, every degree <= 32, FP32 */
#define QAIA_PATH_SPARSE_LDS 2
/* stacked per-objective matrix product on the matrix cores, 64 x 128 tiles:
 * m <= 4 and dense images of at most 4 GiB (m * Np^2 * 7 bytes, Np = n
 * rounded up to a multiple of 128) */
#define QAIA_PATH_DENSE 3
/* as QAIA_PATH_DENSE with 128 x 128 tiles staged through LDS; same limits */
#define QAIA_PATH_DENSE_STAGED 4

typedef struct qaia_problem qaia_problem;

/* Integration schedule of Eq. (9) / Eq. (10).  The update per step t is
 *   y <- y + dt * ( -(a0 - a_t) x - c0 J(c) phi(x) + noise_alpha * eta )
 *   x <- x + dt * a0 * y
 *   |x_i| > 1  ->  x_i = sgn(x_i), y_i = 0           (inelastic wall)
 * with a_t = a0 * t / (steps - 1), J(c) = sum_k c_k J^(k) (Eq. 7) and
 * c0 = 1 / max_i |sum_j J(c)_ij|.  x and y start ~ U(-init_amp, init_amp)
 * from the counter-based stream (seed, replica index + replica_offset).
 * eta_i at step t of global replica g (= row + replica_offset) is a standard
 * normal made by Box-Muller from draw (g * steps + t) * n + i of the same
 * counter generator keyed with seed ^ 0xd1b54a32d192ed03; every path
 * (generated, generic sparse, dense) draws this one stream. */
typedef struct qaia_schedule {
    int32_t variant;     /* QAIA_BSB or QAIA_DSB */
    int32_t precision;   /* QAIA_FP32, QAIA_BF16, QAIA_FP8 */
    int32_t steps;       /* T >= 1 */
    int32_t path;        /* QAIA_PATH_* */
    float dt;            /* > 0 */
    float a0;            /* > 0 */
    float init_amp;      /* >= 0 */
    float noise_alpha;   /* >= 0; 0 = plain SB, > 0 = noise-injected SB (Eq. 10) */
    uint64_t seed;
    uint64_t replica_offset;
} qaia_schedule;

/* ---------------------------------------------------------------- basics */

int32_t qaia_abi_version(void);
const char *qaia_status_string(int32_t status);
/* Detail of the calling thread's last failure ("" if none).  The pointer
 * stays valid until the thread's next qaia_* call. */
const char *qaia_last_error(void);

/* ---------------------------------------------------------------- problem */

/* Build a multi-objective MaxCut instance: graph G = (V, E) with n nodes and
 * m >= 1 edge-weight sets J^(k) (section "Hamiltonian formulation of
 * multi-objective MaxCut", Eq. 1-3).
 *   edge_u, edge_v : HOST int32[num_edges], 0 <= u < v < n, no repeated pair.
 *   weights        : HOST int32[m][num_edges], fixed point.
 *   frac_bits      : 0..30, fraction bits of the fixed point (informational;
 *                    all arithmetic is scale-free or exact).
 *   device         : HIP device ordinal on which the images live.
 * The inputs are copied; the problem owns its device images and is
 * immutable afterwards, so it may be used from several streams at once.
 * Errors: INVALID_ARGUMENT (sizes, ranges, duplicates), OUT_OF_MEMORY,
 * DEVICE_ERROR; *out is set only on success. */
int32_t qaia_problem_create(int32_t n, int32_t m, int64_t num_edges, const int32_t *edge_u,
                            const int32_t *edge_v, const int32_t *weights, int32_t frac_bits,
                            int32_t device, qaia_problem **out);
int32_t qaia_problem_destroy(qaia_problem *p);

/* Sizes and properties of a problem: n, m, num_edges, and the per-objective
 * totals T_k = sum_E W_k (HOST int64[m], may be NULL). */
int32_t qaia_problem_info(const qaia_problem *p, int32_t *n, int32_t *m, int64_t *num_edges,
                          int64_t *total_weight);

/* ---------------------------------------------------------------- sampling */

/* Bytes of device workspace qaia_sample needs for W weight vectors and R
 * replicas each under schedule s. */
int32_t qaia_sample_workspace_bytes(const qaia_problem *p, int64_t W, int32_t R,
                                    const qaia_schedule *s, size_t *bytes);

/* Simulated bifurcation for every (weight vector, replica), then the
 * read-out s_i = sgn(x_i) (sgn 0 = +1) and the exact cut vector of every
 * sample (Eq. 9, 10 and 1; weighted-sum scalarisation, Eq. 7-8).
 *   weights : DEVICE float32[W][m], every row c_k >= 0, finite, sum > 0.
 *             Rows are not renormalised (the dynamics are invariant to a
 *             positive scale of c).
 *   s       : HOST schedule.
 *   spins   : DEVICE uint64[W*R][ceil(n/64)], row = w*R + r.
 *   obj     : DEVICE int64[W*R][m], C_k of each row's spins.
 *   workspace, ws_bytes : DEVICE scratch of at least
 *             qaia_sample_workspace_bytes(); its contents are overwritten.
 * Errors returned synchronously: INVALID_ARGUMENT, UNSUPPORTED (for example
 * a reduced precision with ballistic SB), WORKSPACE_TOO_SMALL,
 * DEVICE_ERROR.  Rows of `weights` that are negative, non-finite or
 * all-zero cannot be checked on the host: the device marks them in the
 * workspace, leaves their spins and cut values zero, and
 * qaia_workspace_status() reports them after the stream is synchronised. */
int32_t qaia_sample(const qaia_problem *p, const float *weights, int64_t W, int32_t R,
                    const qaia_schedule *s, uint64_t *spins, int64_t *obj, void *workspace,
                    size_t ws_bytes, void *hip_stream);

/* Same as qaia_sample and additionally writes x after each of the first
 * trace_steps steps: DEVICE float32[W*R][trace_steps][n].  Test hook for
 * trajectory parity; any path that supports tracing may be forced with
 * s->path. */
int32_t qaia_sample_trace(const qaia_problem *p, const float *weights, int64_t W, int32_t R,
                          const qaia_schedule *s, uint64_t *spins, int64_t *obj, void *workspace,
                          size_t ws_bytes, float *x_trace, int32_t trace_steps, void *hip_stream);

/* Bytes of the static scratch array behind qaia_sample_noalloc (16 MiB). */
#define QAIA_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): qaia_sample
 * with its workspace in a static device array of QAIA_NOALLOC_SCRATCH_BYTES
 * that the library holds on each GPU it runs on until the process ends.  The
 * call allocates nothing (no hipMalloc, no allocating library routine); the
 * caller still passes weights, spins and obj as for qaia_sample, with the
 * same layouts and results.
 *   bad_row : DEVICE int64[1] or NULL.  Once the stream has passed this
 *             call it holds the smallest weight row that is negative,
 *             non-finite or all-zero (whose spins and cuts are left zero),
 *             or -1 if every row was valid.
 * Errors returned synchronously, before anything is queued: those of
 * qaia_sample; WORKSPACE_TOO_SMALL when the call needs more scratch than
 * QAIA_NOALLOC_SCRATCH_BYTES (qaia_sample_workspace_bytes gives the need);
 * UNSUPPORTED when the chosen path would generate a kernel variant on first
 * use (the noise-injected generated kernel is built by the first qaia_sample
 * call with a nonzero noise_alpha; call that once first).
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind: calls that overlap on one GPU (on different streams, or from
 * different threads) race and give undefined results. */
int32_t qaia_sample_noalloc(const qaia_problem *p, const float *weights, int64_t W, int32_t R,
                            const qaia_schedule *s, uint64_t *spins, int64_t *obj, int64_t *bad_row,
                            void *hip_stream);

/* After synchronising the stream of a qaia_sample call: QAIA_OK if every
 * weight row was valid, else QAIA_INVALID_ARGUMENT with *bad_row = the
 * smallest offending row (HOST int64, may be NULL).  workspace is the
 * DEVICE workspace of that call; this call synchronises on it. */
int32_t qaia_workspace_status(const void *workspace, int64_t *bad_row);

/* Exact cut values, Eq. (1): obj[i][k] = sum over edges with s_u != s_v of
 * W_k.  spins DEVICE uint64[count][ceil(n/64)], obj DEVICE int64[count][m]. */
int32_t qaia_evaluate(const qaia_problem *p, const uint64_t *spins, int64_t count, int64_t *obj,
                      void *hip_stream);

/* Exact cut values of consecutive spin configurations, Eq. (1), for fronts
 * by exhaustive enumeration (the brute-force reference fronts of section
 * "Comparison to evolutionary algorithm-based heuristics").  Row r
 * (0 <= r < count) is the configuration whose packed spin word (bit i set
 * <=> s_i = -1) equals first + r; obj DEVICE int64[count][m].  Since
 * C_k(s) = C_k(-s), codes 0 .. 2^(n-1) - 1 (spin n-1 fixed to +1) cover
 * every cut once.  Needs n <= 63 and first + count <= 2^n, else
 * QAIA_UNSUPPORTED / QAIA_INVALID_ARGUMENT. */
int32_t qaia_enumerate_cuts(const qaia_problem *p, uint64_t first, int64_t count, int64_t *obj,
                            void *hip_stream);

/* Uniformly random spin configurations (the random-sampling baseline of the
 * same section): row r gets n independent fair spins drawn from the
 * counter-based stream keyed with seed ^ 0x6a09e667f3bcc909, draw
 * (r + offset) * ceil(n/64) + word; bits >= n are zero.  spins DEVICE
 * uint64[count][ceil(n/64)]. */
int32_t qaia_random_spins(int32_t n, int64_t count, uint64_t seed, uint64_t offset, uint64_t *spins,
                          void *hip_stream);

/* Weight vectors uniform on the simplex (Dirichlet(1, ..., 1); section
 * "Scalarization via the weighted sum method"): row r is the normalised
 * vector of m i.i.d. Exp(1) values -log(u), u from 24 bits of draw
 * (r + offset) * m + k of the counter stream keyed seed ^ 0xbb67ae8584caa73b.
 * weights DEVICE float[count][m], 1 <= m <= 8. */
int32_t qaia_dirichlet_weights(int32_t m, int64_t count, uint64_t seed, uint64_t offset, float *weights,
                               void *hip_stream);

/* ---------------------------------------------------------------- precision form */

/* Bytes of DEVICE workspace qaia_dense_field needs for `count` columns. */
int32_t qaia_dense_field_workspace_bytes(const qaia_problem *p, int32_t precision, int64_t count,
                                         size_t *bytes);

/* The per-objective coupling products that the dense SB path computes every
 * step (the force sum_j J^(k)_ij phi(x_j) of Eq. 9, per objective k of the
 * scalarisation of Eq. 7), for given phi, in the requested arithmetic:
 *   QAIA_FP32: fp32 J x fp32 phi; QAIA_BF16 / QAIA_FP8: J stored per objective
 *   as bf16 / e4m3 of W * 2^-e_k, phi rounded to +-1 (entries 0 stay 0),
 *   fp32 accumulation, result multiplied back by 2^e_k.
 *   phi   : DEVICE float32[count][n].
 *   field : DEVICE float32[count][m][n], in weight units (fixed point).
 *   workspace : DEVICE scratch of qaia_dense_field_workspace_bytes().
 * Test and reporting hook for the field error of reduced precision.  Errors:
 * INVALID_ARGUMENT, UNSUPPORTED (no dense images or m > 4),
 * WORKSPACE_TOO_SMALL, DEVICE_ERROR. */
int32_t qaia_dense_field(const qaia_problem *p, int32_t precision, const float *phi, int64_t count,
                         float *field, void *workspace, size_t ws_bytes, void *hip_stream);

/* ---------------------------------------------------------------- filtering */

int32_t qaia_pareto_filter_workspace_bytes(int64_t M, int32_t m, size_t *bytes);

/* Non-dominated filtering of a sample pool, section "Pareto filtering":
 * in cut (maximisation) space y' dominates y iff y'_k >= y_k for all k and
 * y' != y (Eq. 4).  Equal objective vectors are merged and represented by
 * their smallest sample index.
 *   obj      : DEVICE int64[M][m], 1 <= m <= 8.
 *   keep_idx : DEVICE int64[M] (capacity M), receives the representatives in
 *              ascending order.
 *   num_keep : DEVICE int64[1], receives their count.
 *   workspace: DEVICE scratch of qaia_pareto_filter_workspace_bytes(M, m). */
int32_t qaia_pareto_filter(const int64_t *obj, int64_t M, int32_t m, int64_t *keep_idx,
                           int64_t *num_keep, void *workspace, size_t ws_bytes, void *hip_stream);

/* Per-objective minimum of a pool, the reference point of the hypervolume
 * comparisons in section "Comparison to evolutionary algorithm-based
 * heuristics" (the worst value of each objective over all sampled or
 * enumerated solutions):
 *   obj : DEVICE int64[M][m], 1 <= m <= 8, M >= 0.
 *   lo  : DEVICE int64[m]; accumulate = 0: lo[k] = min_r obj[r][k] (INT64_MAX
 *         when M = 0); accumulate = 1: lo[k] = min(lo[k], min_r obj[r][k]),
 *         so that successive pools fold into one minimum.
 * Asynchronous on hip_stream; allocates nothing.  Errors: INVALID_ARGUMENT. */
int32_t qaia_objective_min(const int64_t *obj, int64_t M, int32_t m, int64_t *lo, int32_t accumulate,
                           void *hip_stream);

/* Non-dominated ranks of all M rows (non-dominated sorting of the sample
 * pool; the fronts behind section "Pareto filtering"): rank[i] = 0 for rows
 * whose vector no other row dominates (Eq. 4), and r for rows that become
 * non-dominated once the rows of ranks < r are removed; equal rows share a
 * rank.  Ranks >= max_rank are reported as max_rank.
 *   obj:       DEVICE int64[M][m], 1 <= m <= 8, M < 2^31
 *   rank:      DEVICE int32[M]
 *   num_ranks: HOST; number of ranks peeled (at most max_rank; rows left
 *              over when it equals max_rank carry rank max_rank)
 *   workspace: DEVICE scratch of qaia_pareto_ranks_workspace_bytes(M, m).
 * Synchronises hip_stream once per rank (the number of fronts decides the
 * work), so it cannot be captured in a graph. */
int32_t qaia_pareto_ranks_workspace_bytes(int64_t M, int32_t m, size_t *bytes);
int32_t qaia_pareto_ranks(const int64_t *obj, int64_t M, int32_t m, int32_t max_rank, int32_t *rank,
                          int32_t *num_ranks, void *workspace, size_t ws_bytes, void *hip_stream);

/* ---------------------------------------------------------------- hypervolume */

/* Exact hypervolume, Eq. (6) and Appendix A: the m-dimensional Lebesgue
 * measure of the union of boxes [ref, y] over the points.  Points with some
 * y_k <= ref_k add nothing (their box is clipped to zero width); dominated
 * and repeated points are allowed.
 *   pts : HOST int64[P][m], ref : HOST int64[m].
 *   hv  : HOST uint64[4], the exact value as a 256-bit little-endian integer
 *         in units of the product of the coordinate units.
 *   hv_approx : HOST double, may be NULL.
 * Errors: INVALID_ARGUMENT, OVERFLOW if the sum over objectives of the bit
 * lengths of (max_k y_k - ref_k) exceeds 256.
 * Synchronous host computation; for m >= 3 it runs on as many threads as
 * the calling process's CPU affinity mask allows (QAIA_HV_THREADS in the
 * environment overrides the count).  Thread-safe: calls share no state. */
int32_t qaia_hypervolume(const int64_t *pts, int64_t P, int32_t m, const int64_t *ref,
                         uint64_t hv[4], double *hv_approx);

/* ---------------------------------------------------------------- batching form */
/* A ragged batch: items of different problems (n, m, density), weight sets
 * and replica counts sampled under one schedule.  Each item is sampled
 * exactly as qaia_sample would sample it on the same path (same arithmetic,
 * same counter streams), so the outputs are bit-identical to per-item calls. */
typedef struct qaia_batch_item {
    const qaia_problem *problem;
    const float *weights; /* DEVICE [W][m] */
    int64_t W;
    int32_t R;
    int32_t path;         /* QAIA_PATH_*; AUTO = the planner's default */
    uint64_t *spins;      /* DEVICE [W*R][ceil(n/64)] */
    int64_t *obj;         /* DEVICE [W*R][m] */
    int32_t tile;         /* kernel tile knob; 0 = the family's default.  QAIA_PATH_SPARSE_LDS:
                           * replicas per 256-lane block (their spins must fit 16 per lane,
                           * replicas * n <= 4096); other families: must be 0 */
    int32_t reserved;     /* 0 */
} qaia_batch_item;

int32_t qaia_sample_batch_workspace_bytes(const qaia_batch_item *items, int32_t count,
                                          const qaia_schedule *s, size_t *bytes);
/* Samples every item with one graph launch: per-item weight preparation; for
 * the items on the generic sparse kernel one persistent launch per kernel
 * shape whose blocks take (item, replica tile) work units from a device queue
 * (items in decreasing cost per tile, each unit's whole step loop on chip);
 * each item on a generated kernel as its own launch; for the dense items one
 * grouped step launch per step over all their tiles, the step loop captured
 * in the graph.  items: HOST array, buffers DEVICE, all on one device.
 * Errors as qaia_sample; the call synchronises the host with the caller's
 * stream once (descriptor upload). */
int32_t qaia_sample_batch(const qaia_batch_item *items, int32_t count, const qaia_schedule *s,
                          void *workspace, size_t ws_bytes, void *hip_stream);

int32_t qaia_plan_autotune_workspace_bytes(const qaia_batch_item *items, int32_t count,
                                           const qaia_schedule *s, int32_t probe_steps, size_t *bytes);
/* Autotuner: for every item, times each kernel family and tile available to
 * it (generated one-replica-per-lane kernel; generic one-spin-per-lane kernel
 * with 1x, 2x and 4x its default replicas per block; 64 x 128 register and
 * 128 x 128 LDS-staged matrix-core tiles) on probe_steps steps of its real
 * shape, and writes the fastest into items[i].path and items[i].tile (HOST,
 * in place); est_seconds (HOST [count], may be NULL) receives the probe time
 * scaled to s->steps.  The items' outputs are overwritten.  Synchronises the
 * host with hip_stream. */
int32_t qaia_plan_autotune(qaia_batch_item *items, int32_t count, const qaia_schedule *s,
                           int32_t probe_steps, double *est_seconds, void *workspace, size_t ws_bytes,
                           void *hip_stream);

/* ---------------------------------------------------------------- learned form */
/* The paper scalarises with fixed weight vectors (Das-Dennis or Dirichlet,
 * section "Scalarization via the weighted sum method"); the learned form
 * proposes them instead: a multilayer perceptron in_dim -> 128 -> 128 -> 1
 * (exact-erf GELU, bf16 weights, fp32 activations and accumulation) scores
 * candidate vectors c from c and eight features of the current
 * non-dominated archive, and is trained online by Adam on the mean binary
 * cross-entropy of "c produced a new non-dominated point".
 * Parameters (flat, in this order): W1 [128][in_dim], b1 [128], W2 [128][128],
 * b2 [128], w3 [128], b3 [1]; in_dim in [1, 16].  All buffers DEVICE unless
 * stated; calls are asynchronous on hip_stream. */

int32_t qaia_mlp_param_count(int32_t in_dim, int64_t *count); /* count: HOST */
int32_t qaia_mlp_forward_workspace_bytes(int64_t N, size_t *bytes);
/* logits[N] of inputs X [N][in_dim]; params: bf16 bit patterns. */
int32_t qaia_mlp_forward(const uint16_t *params, int32_t in_dim, const float *X, int64_t N,
                         float *logits, void *workspace, size_t ws_bytes, void *hip_stream);
int32_t qaia_mlp_backward_workspace_bytes(int32_t in_dim, int64_t B, size_t *bytes);
/* grad [param count] of the mean binary cross-entropy of the logits of X
 * [B][in_dim] against labels [B] (0 or 1); logits [B] written if not NULL. */
int32_t qaia_mlp_backward(const uint16_t *params, int32_t in_dim, const float *X, const float *labels,
                          int64_t B, float *grad, float *logits, void *workspace, size_t ws_bytes,
                          void *hip_stream);
/* One Adam step (step counts from 1) on fp32 master weights and moments;
 * refreshes the bf16 params (round to nearest even). */
int32_t qaia_mlp_adam(float *master, uint16_t *params, float *moment1, float *moment2,
                      const float *grad, int64_t count, int32_t step, float lr, float beta1,
                      float beta2, float eps, void *hip_stream);

int32_t qaia_mlp_train_workspace_bytes(int32_t in_dim, int64_t n, int32_t batch, size_t *bytes);
/* The proposer's training loop of one round: `steps` Adam steps (beta1 0.9,
 * beta2 0.999, eps 1e-8, step counter from first_step >= 1) of the mean
 * binary cross-entropy on minibatches of B = min(batch, n) rows of
 * X [n][in_dim] / labels [n].  Minibatch t is window t mod floor(n / B) of a
 * random permutation of the rows, drawn at the start of every pass as the
 * top-n of n equal scores with Gumbel noise (qaia_topk, temperature 1, seed
 * seed + 104729 * (first_step + t)).  master / moment1 / moment2: DEVICE
 * fp32 [param count], params: DEVICE bf16 bits, updated in place.  All work
 * is queued on the stream without host waits. */
int32_t qaia_mlp_train(float *master, uint16_t *params, float *moment1, float *moment2, int32_t in_dim,
                       const float *X, const float *labels, int64_t n, int32_t batch, int32_t steps,
                       int32_t first_step, float lr, uint64_t seed, void *workspace, size_t ws_bytes,
                       void *hip_stream);

int32_t qaia_front_features_workspace_bytes(int64_t P, int32_t m, size_t *bytes);
/* MLP input rows feat [N][m + 8] = (c, f1..f8): c followed by eight
 * features of candidate c against the archive front
 * (int64 [P][m], normalised per objective to [0,1] by its minimum and
 * maximum; zero range maps to 1), with v_j = c . y^_j: max v; max minus the
 * second; max minus the eighth (the smallest when P < 8); distance from the
 * maximising point to its nearest other front point; fraction of the front
 * within 0.05 of it; smallest angle to the `hits` rows [n_hits][m] and to the
 * `misses` rows [n_misses][m] (pi/2 when empty); max_k |c_k - 1/m|. */
int32_t qaia_front_features(const int64_t *front, int64_t P, int32_t m, const float *cands, int64_t N,
                            const float *hits, int64_t n_hits, const float *misses, int64_t n_misses,
                            float *feat, void *workspace, size_t ws_bytes, void *hip_stream);

int32_t qaia_topk_workspace_bytes(int64_t N, size_t *bytes);
/* Indices (int64 [k]) of the k largest keys among N, largest first; equal
 * keys keep increasing index order.  temperature = 0: the keys are the
 * scores (deterministic top-k).  temperature > 0: the keys are
 * score / temperature plus a standard Gumbel draw from the counter stream
 * `seed`, i.e. k items sampled without replacement with probabilities
 * proportional to exp(score / temperature). */
int32_t qaia_topk(const float *scores, int64_t N, int64_t k, float temperature, uint64_t seed,
                  int64_t *idx, void *workspace, size_t ws_bytes, void *hip_stream);

/* labels [W] = 1 where weight row w has a sample among the kept rows of a
 * qaia_pareto_filter over [archive rows ; W*R new samples], else 0.  Because
 * duplicates are represented by their smallest index, a kept new sample is a
 * vector absent from the archive. */
int32_t qaia_new_point_labels(const int64_t *keep_idx, const int64_t *num_keep, int64_t archive_rows,
                              int32_t R, int64_t W, float *labels, void *hip_stream);

/* Row gather: dst[r][:] = src[idx[r]][:] for r < min(*count, cap), rows of
 * `width` 32-bit words (an int64 row of m values is 2m words). */
int32_t qaia_gather_rows(const void *src, int32_t width, const int64_t *idx, const int64_t *count,
                         int64_t cap, void *dst, void *hip_stream);

/* ---------------------------------------------------------------------------
 * Measurement kernels.  Not part of the method: they measure this GPU's own
 * ceilings (VALU FMA issue, matrix-core rate per operand format, HBM copy)
 * so that a kernel's roofline fraction can be stated against a measured peak
 * as well as the datasheet one.  Each result has a closed form (checked by
 * the tests); time the launch with events on `hip_stream`.  Asynchronous;
 * argument errors return before anything is enqueued.
 */

/* blocks x 256 lanes, each running eight independent fp32 FMA chains
 * x <- x * a + b for `iters` iterations from x0 = (t + c) mod 8 (lane t,
 * chain c); out[t] (DEVICE float [blocks * 256]) = sum of the eight final
 * values.  Work: blocks * 256 * iters * 8 FMAs = 16 flop per lane-iteration.
 * blocks in [1, 2^31), iters >= 1. */
int32_t qaia_peak_fma(int64_t blocks, int32_t iters, float a, float b, float *out, void *hip_stream);

/* blocks x 4 waves, each wave issuing `iters` rounds of four independent
 * 32x32 MFMAs with every operand 1.0: precision QAIA_FP32 (32x32x2),
 * QAIA_BF16 (32x32x16) or QAIA_FP8 (e4m3, 32x32x64).  out[t] (DEVICE float
 * [blocks * 256]) = 4 * K * iters with K = 2, 16, 64.  Work per launch:
 * blocks * 4 * iters * 4 * 2 * 32 * 32 * K flop.  blocks in [1, 2^31),
 * iters >= 1 and 4 * K * iters < 2^24 (exact accumulation). */
int32_t qaia_peak_mfma(int32_t precision, int64_t blocks, int32_t iters, float *out, void *hip_stream);

/* blocks x 256 lanes running the sparse SB update's instruction mix: per
 * iteration 14 soft spins per lane take 60 FMAs (y_i += k x_i, k x of its two
 * ring neighbours, k x_(i+7) for i < 4; x_i += k y_i) and 42 wall operations
 * (|x_i| > 1 compare, y select, x clamp to [-1, 1]), the 10 : 7 ratio of the
 * generated kernel's 180 FMAs to 126 wall operations per replica-step on the
 * 42-node, 48-edge graph (section "Simulated Bifurcation with Gaussian
 * noise", Eq. 9).  With k = 0 the state stays at its start values
 * x_i = ((t + i) mod 8) / 8 - 1/2, y_i = ((t + 3i) mod 4) / 4 (lane t), so
 * out[t] (DEVICE float [blocks * 256]) = sum_i (x_i + y_i) exactly.  Work:
 * blocks * 256 * iters * 102 lane instructions.  blocks in [1, 2^31),
 * iters >= 1, k finite. */
int32_t qaia_peak_valu(int64_t blocks, int32_t iters, float k, float *out, void *hip_stream);

/* dst = src, `bytes` (a multiple of 16) between two DEVICE buffers that are
 * 16-byte aligned and do not overlap; 2 * bytes of HBM traffic. */
int32_t qaia_peak_copy(const void *src, void *dst, size_t bytes, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* QAIA_H */
