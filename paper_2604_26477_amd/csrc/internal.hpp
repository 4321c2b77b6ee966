// Internal declarations of libqaia (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/qaia.h"

namespace qaia {

// ----------------------------------------------------------------- errors
struct Error {
    int32_t status;
    std::string msg;
};

void set_error(const std::string &msg);
void clear_error();
int32_t fail(int32_t status, const std::string &msg);  // records msg, returns status

#define QAIA_HIP(call)                                                                      \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            throw ::qaia::Error{QAIA_DEVICE_ERROR, std::string(#call) + ": " +              \
                                                       hipGetErrorString(e_)};              \
    } while (0)

#define QAIA_CHECK(cond, status, msg)                           \
    do {                                                        \
        if (!(cond)) throw ::qaia::Error{(status), (msg)};      \
    } while (0)

// Scoped device switch.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
};

// ----------------------------------------------------------------- problem
struct JitKernel;  // generated per-graph kernel (jit.cpp)

// Dense per-objective images of J for the matrix-core path, zero padded to
// Np = ceil64(n); bf16 / e4m3 copies hold W * 2^-e_k (value = stored * scale).
struct DenseImages {
    bool ok = false;
    std::string why;  // reason when not built
    int32_t Np = 0;
    float *J32 = nullptr;     // [m][Np][Np]
    uint16_t *J16 = nullptr;  // bf16 bits
    uint8_t *J8 = nullptr;    // e4m3 bits
    float scale16[8] = {}, scale8[8] = {};
    float *scales = nullptr;  // device [3][8]: per precision, per objective
};

struct Problem {
    int32_t n = 0, m = 0, frac_bits = 0, device = 0;
    int64_t E = 0;
    int32_t words = 0;  // ceil(n / 64)
    std::vector<int32_t> eu, ev, W;      // host copies, W is [m][E]
    std::vector<int32_t> rowptr, col, eid;  // CSR over nodes (both directions)
    std::vector<int64_t> total;          // T_k = sum_E W_k
    int32_t max_degree = 0;
    // device images
    int32_t *d_eu = nullptr, *d_ev = nullptr, *d_W = nullptr;
    int32_t *d_rowptr = nullptr, *d_col = nullptr, *d_eid = nullptr;
    int64_t *d_rho = nullptr;  // [m][n] row sums sum_j W_k,ij (exact)
    // generated register-resident kernels, index = variant (bSB, dSB)
    JitKernel *jit[2] = {nullptr, nullptr};
    JitKernel *jit_trace[2] = {nullptr, nullptr};  // tracing variants, built on first use
    JitKernel *jit_noise[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [variant][trace], noise-injected, built on first use
    JitKernel *jit16[2][2][2] = {};  // [variant][trace][noise], binary16 form, built on first use
    std::string jit_error;
    DenseImages dense;
    std::mutex mu;
    ~Problem();
};

// ----------------------------------------------------------------- sampling workspace
// Layout of the caller's workspace for qaia_sample (all offsets 256-aligned):
//   header   : WsHeader
//   kt       : float[T]          per-step coefficient -dt (a0 - a_t)
//   c0s      : double[W]         c0 per weight row (weight units); negative marks an invalid row
//   jcp      : float[W][E]       folded edge coefficients -dt c0 J(c)_e (sparse paths)
// and for the dense path: x (two buffers for ballistic SB), y, Phi (two
// buffers for discrete SB) and per-column coefficients.
struct WsHeader {
    uint64_t magic;
    int64_t bad_row;  // smallest invalid weight row, INT64_MAX if none
    int64_t W;
    int64_t reserved;
};
constexpr uint64_t kWsMagic = 0x7161696177733031ull;  // "qaiaws01"

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct WsLayout {
    size_t header = 0, kt = 0, c0s = 0, jcp = 0, total = 0;
    bool has_jcp = false;  // per-edge coefficients reserved (sparse paths)
    // dense path
    int64_t colsP = 0;
    size_t xa = 0, xb = 0, y = 0, pa = 0, pb = 0, coef = 0;
};
// edge_coefs: reserve the folded per-edge coefficients (sparse paths only)
WsLayout sample_ws_layout(const Problem &p, int64_t W, int32_t R, const qaia_schedule &s, bool edge_coefs);
void dense_ws_extend(const Problem &p, int64_t W, int32_t R, const qaia_schedule &s, WsLayout &L);

// Allocation-free sampling (noalloc.hip): this device's static scratch array
// (its address from hipGetSymbolAddress, taken once per device), its size,
// and a copy of the invalid-row flag from the scratch header (the workspace
// header sits at offset 0) into a caller-owned device word.
void *noalloc_scratch(int device);
size_t noalloc_scratch_bytes();
void launch_noalloc_bad_row(const void *scratch, int64_t *bad_row, hipStream_t st);
// Whether the generated register kernel for this schedule kind exists already
// (the tracing and noise variants are generated on first use).
bool sparse_reg_ready(const Problem &p, int variant, bool trace, bool noise, bool half = false);

// One problem's rows for the generic sparse kernel (passed by value, or as a
// device array for a ragged batch).
struct SparseJob {
    int n, m, words, R, T, rpb;
    int64_t E, rows;
    const int32_t *rowptr, *col, *eid, *Wt, *eu, *ev;
    const float *jcp;
    const double *c0s;
    const float *kt_tab;
    float dta0, dt_alpha, amp;
    uint64_t seed, offset;
    uint64_t *spins;
    int64_t *obj;
    float *trace;
    int trace_steps;
};
// One problem's dense SB state (both buffers of each double-buffered pair;
// the step parity selects them).
struct DenseJob {
    const void *J;
    float *xa, *xb, *y;
    void *pa, *pb;
    const float *coef;
    const float *kt_tab;
    float dta0;
    int Np, N, m, cols, tiles_x, tiles_y;
    float *trace;
    int trace_steps;
    int staged;  // 0: 64 x 128 tiles from global loads; 1: 128 x 128 tiles staged through LDS
    // noise injection (Eq. 10): y += dt alpha eta, eta from the keyed counter stream; off when 0
    float dt_alpha;
    int steps;
    uint64_t seed, offset;
};
struct SparseShape {
    int rpb = 1, npt = 1, maxdeg = 4;
    int64_t blocks = 0;
    size_t shmem = 0;
};

// ----------------------------------------------------------------- kernels (host launchers)
void launch_prep(const Problem &p, const float *weights, int64_t W, const qaia_schedule &s,
                 void *ws, const WsLayout &L, hipStream_t st);
void launch_sparse_lds(const Problem &p, int64_t W, int32_t R, const qaia_schedule &s, void *ws,
                       const WsLayout &L, uint64_t *spins, int64_t *obj, float *trace,
                       int32_t trace_steps, hipStream_t st, int rpb = 0);
bool sparse_lds_supported(const Problem &p, std::string *why);
// rpb: replicas per block, 0 = the default floor(256 / n) (UNSUPPORTED past 16 spins per lane)
int sparse_lds_default_rpb(const Problem &p);
SparseShape sparse_lds_shape(const Problem &p, int64_t rows, int rpb = 0);
SparseJob sparse_job(const Problem &p, int64_t W, int32_t R, const qaia_schedule &s, void *ws,
                     const WsLayout &L, uint64_t *spins, int64_t *obj, float *trace, int32_t trace_steps,
                     int rpb = 0);
// persistent launch over `count` device jobs whose work units are numbered by
// the prefix `starts` (units in total); `queue` is a device counter it resets
void launch_sparse_lds_queue(const SparseJob *jobs, int count, const int64_t *starts, int64_t units, int maxdeg,
                             int npt, size_t shmem, bool dsb, unsigned long long *queue, hipStream_t st);
// single: one job by value; otherwise `count` device jobs with block prefix `starts`
void launch_sparse_lds_jobs(const SparseJob *single, const SparseJob *jobs, int count, const int64_t *starts,
                            int64_t blocks, int maxdeg, int npt, size_t shmem, bool dsb, hipStream_t st);
void launch_enumerate(const Problem &p, uint64_t first, int64_t count, int64_t *obj, hipStream_t st);
void launch_random_spins(int n, int64_t count, uint64_t seed, uint64_t offset, uint64_t *spins, hipStream_t st);
void launch_dirichlet(int m, int64_t count, uint64_t seed, uint64_t offset, float *out, hipStream_t st);
void launch_evaluate(const Problem &p, const uint64_t *spins, int64_t count, int64_t *obj,
                     hipStream_t st);

// generated kernels (jit.cpp)
bool jit_eligible(const Problem &p, std::string *why);
void jit_prepare(Problem &p);  // compiles both variants if eligible; records failures
void launch_sparse_reg(const Problem &p, int variant, int64_t W, int32_t R, const qaia_schedule &s,
                       void *ws, const WsLayout &L, uint64_t *spins, int64_t *obj, float *trace,
                       int32_t trace_steps, hipStream_t st);
void jit_release(JitKernel *k);

// dense path (dense.hip)
void dense_build(Problem &p);
void dense_release(Problem &p);
bool dense_supported(const Problem &p, std::string *why);
void launch_dense(const Problem &p, const float *weights, int64_t W, int32_t R,
                  const qaia_schedule &s, void *ws, const WsLayout &L, uint64_t *spins, int64_t *obj,
                  float *trace, int32_t trace_steps, bool staged, hipStream_t st);
DenseJob dense_job(const Problem &p, int64_t W, int32_t R, const qaia_schedule &s, void *ws, const WsLayout &L,
                   float *trace, int32_t trace_steps, bool staged);
void launch_dense_setup(const Problem &p, const float *weights, int32_t R, const qaia_schedule &s, void *ws,
                        const WsLayout &L, const DenseJob &j, hipStream_t st);
void launch_dense_finish(const Problem &p, int32_t R, const qaia_schedule &s, void *ws, const WsLayout &L,
                         const DenseJob &j, uint64_t *spins, int64_t *obj, hipStream_t st);
// grouped step over dense jobs; staged groups share m = mt and have 8-aligned block starts
void launch_dense_batch_step(int prec, bool dsb, bool staged, int mt, const DenseJob *jobs, int count,
                             const int64_t *starts, int64_t blocks, int t, hipStream_t st);
inline bool is_dense_path(int path) { return path == QAIA_PATH_DENSE || path == QAIA_PATH_DENSE_STAGED; }
size_t dense_field_ws_bytes(const Problem &p, int prec, int64_t count);
void launch_dense_field(const Problem &p, int prec, const float *phi, int64_t count, float *field,
                        void *ws, size_t ws_bytes, hipStream_t st);

// learned proposer (mlp.hip)
int64_t mlp_param_count(int D);
size_t mlp_forward_ws_bytes(int64_t N);
size_t mlp_backward_ws_bytes(int D, int64_t B);
void launch_mlp_forward(const uint16_t *P, int D, const float *X, int64_t N, float *logits, void *ws,
                        hipStream_t st);
void launch_mlp_backward(const uint16_t *P, int D, const float *X, const float *y, int64_t B,
                         float *grad, float *logits, void *ws, hipStream_t st);
size_t mlp_train_ws_bytes(int D, int64_t n, int64_t batch);
void launch_mlp_train(float *master, uint16_t *P, float *m1, float *m2, int D, const float *X, const float *y,
                      int64_t n, int64_t batch, int steps, int first_step, float lr, uint64_t seed, void *ws,
                      size_t ws_bytes, hipStream_t st);
void launch_adam(float *master, uint16_t *P, float *m, float *v, const float *g, int64_t n, int step,
                 float lr, float b1, float b2, float eps, hipStream_t st);
size_t features_ws_bytes(int64_t Pn, int m);
void launch_features(const int64_t *front, int64_t Pn, int m, const float *cands, int64_t N,
                     const float *hits, int64_t Hn, const float *misses, int64_t Mn, float *feat,
                     void *ws, size_t ws_bytes, hipStream_t st);
size_t topk_ws_bytes(int64_t N);
void launch_topk(const float *scores, int64_t N, int64_t k, float temperature, uint64_t seed, int64_t *idx_out,
                 void *ws, size_t ws_bytes, hipStream_t st);
void launch_labels(const int64_t *keep, const int64_t *num_keep, int64_t archive, int R, int64_t W,
                   float *labels, hipStream_t st);
void launch_gather_rows(const uint32_t *src, int width, const int64_t *idx, const int64_t *count,
                        int64_t cap, uint32_t *dst, hipStream_t st);
// measurement kernels (peaks.hip)
void launch_peak_fma(int64_t blocks, int32_t iters, float a, float b, float *out, hipStream_t st);
void launch_peak_mfma(int32_t precision, int64_t blocks, int32_t iters, float *out, hipStream_t st);
void launch_peak_copy(const void *src, void *dst, size_t bytes, hipStream_t st);
void launch_peak_valu(int64_t blocks, int32_t iters, float k, float *out, hipStream_t st);

// batching form (batch.cpp)
size_t batch_ws_bytes(const qaia_batch_item *items, int32_t count, const qaia_schedule &s);
void sample_batch(const qaia_batch_item *items, int32_t count, const qaia_schedule &s, void *ws, size_t ws_bytes,
                  hipStream_t caller);
void autotune(qaia_batch_item *items, int32_t count, const qaia_schedule &s, int32_t probe_steps,
              double *est_seconds, void *ws, size_t ws_bytes, hipStream_t st);
size_t autotune_ws_bytes(const qaia_batch_item *items, int32_t count, const qaia_schedule &s, int32_t probe_steps);

// pareto filter (pareto.hip)
size_t pareto_ranks_ws_bytes(int64_t M, int32_t m);
int32_t launch_pareto_ranks(const int64_t *obj, int64_t M, int32_t m, int32_t max_rank, int32_t *rank, void *ws,
                            size_t ws_bytes, hipStream_t st);
size_t pareto_ws_bytes(int64_t M, int32_t m);
void launch_objective_min(const int64_t *obj, int64_t M, int32_t m, int64_t *lo, bool accumulate,
                          hipStream_t st);
void launch_pareto(const int64_t *obj, int64_t M, int32_t m, int64_t *keep, int64_t *num_keep,
                   void *ws, size_t ws_bytes, hipStream_t st);

// hypervolume (hypervolume.cpp)
int32_t hypervolume_exact(const int64_t *pts, int64_t P, int32_t m, const int64_t *ref,
                          uint64_t hv[4], double *approx);

}  // namespace qaia
