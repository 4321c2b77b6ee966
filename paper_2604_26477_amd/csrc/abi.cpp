// extern "C" entry points of libqaia: argument validation, path planning and
// dispatch.  No C++ exception crosses this boundary.
#include <cmath>
#include <cstring>

#include "internal.hpp"

namespace qaia {
Problem *build_problem(int32_t n, int32_t m, int64_t E, const int32_t *eu, const int32_t *ev,
                       const int32_t *W, int32_t frac_bits, int32_t device);
const char *last_error_cstr();

namespace {

template <typename F>
int32_t guarded(F &&f) {
    clear_error();
    try {
        return f();
    } catch (const Error &e) {
        return fail(e.status, e.msg);
    } catch (const std::bad_alloc &) {
        return fail(QAIA_OUT_OF_MEMORY, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(QAIA_DEVICE_ERROR, e.what());
    } catch (...) {
        return fail(QAIA_DEVICE_ERROR, "unknown error");
    }
}

void check_schedule(const Problem &p, const qaia_schedule *s) {
    QAIA_CHECK(s != nullptr, QAIA_INVALID_ARGUMENT, "null schedule");
    QAIA_CHECK(s->variant == QAIA_BSB || s->variant == QAIA_DSB, QAIA_INVALID_ARGUMENT,
               "variant must be QAIA_BSB or QAIA_DSB");
    QAIA_CHECK(s->precision == QAIA_FP32 || s->precision == QAIA_BF16 || s->precision == QAIA_FP8 ||
                   s->precision == QAIA_FP16,
               QAIA_INVALID_ARGUMENT, "unknown precision");
    QAIA_CHECK(s->steps >= 1, QAIA_INVALID_ARGUMENT, "steps must be >= 1");
    QAIA_CHECK(std::isfinite(s->dt) && s->dt > 0.0f, QAIA_INVALID_ARGUMENT, "dt must be finite and > 0");
    QAIA_CHECK(std::isfinite(s->a0) && s->a0 > 0.0f, QAIA_INVALID_ARGUMENT, "a0 must be finite and > 0");
    QAIA_CHECK(std::isfinite(s->init_amp) && s->init_amp >= 0.0f, QAIA_INVALID_ARGUMENT,
               "init_amp must be finite and >= 0");
    QAIA_CHECK(std::isfinite(s->noise_alpha) && s->noise_alpha >= 0.0f, QAIA_INVALID_ARGUMENT,
               "noise_alpha must be finite and >= 0");
    QAIA_CHECK(s->path >= QAIA_PATH_AUTO && s->path <= QAIA_PATH_DENSE_STAGED, QAIA_INVALID_ARGUMENT,
               "unknown path");
    if (s->precision == QAIA_FP16) {
        QAIA_CHECK(s->path == QAIA_PATH_AUTO || s->path == QAIA_PATH_SPARSE_REG, QAIA_UNSUPPORTED,
                   "binary16 runs on the generated sparse kernel only");
        QAIA_CHECK(p.jit[s->variant] != nullptr, QAIA_UNSUPPORTED,
                   "binary16 needs the generated sparse kernel: " +
                       (p.jit_error.empty() ? std::string("not built") : p.jit_error));
    } else if (s->precision != QAIA_FP32) {
        QAIA_CHECK(s->variant == QAIA_DSB, QAIA_UNSUPPORTED,
                   "reduced precision needs discrete SB (its phi(x) = sgn(x) is exact)");
        QAIA_CHECK(s->path == QAIA_PATH_AUTO || is_dense_path(s->path), QAIA_UNSUPPORTED,
                   "reduced precision runs on the dense path only");
    }
}

// Picks the kernel family for a sampling call.
int plan_path(const Problem &p, const qaia_schedule &s, bool tracing) {
    (void)tracing;
    if (s.path != QAIA_PATH_AUTO) return s.path;
    if (s.precision == QAIA_FP16) return QAIA_PATH_SPARSE_REG;
    if (s.precision != QAIA_FP32) return QAIA_PATH_DENSE_STAGED;
    if (p.jit[s.variant] != nullptr) return QAIA_PATH_SPARSE_REG;
    if (sparse_lds_supported(p, nullptr)) return QAIA_PATH_SPARSE_LDS;
    return QAIA_PATH_DENSE_STAGED;
}

WsLayout full_layout(const Problem &p, int64_t W, int32_t R, const qaia_schedule &s, int path) {
    WsLayout L = sample_ws_layout(p, W, R, s, !is_dense_path(path));
    if (is_dense_path(path)) {
        std::string why;
        QAIA_CHECK(dense_supported(p, &why), QAIA_UNSUPPORTED, "dense path: " + why);
        dense_ws_extend(p, W, R, s, L);
    }
    return L;
}

// no_alloc: the workspace is the library's static scratch array; a call that
// would build a generated kernel variant on first use (and so allocate code
// memory) is refused instead, and a too-small scratch is reported as such.
int32_t sample_impl(const qaia_problem *pp, const float *weights, int64_t W, int32_t R,
                    const qaia_schedule *s, uint64_t *spins, int64_t *obj, void *ws, size_t ws_bytes,
                    float *trace, int32_t trace_steps, void *stream, bool no_alloc = false) {
    QAIA_CHECK(pp != nullptr, QAIA_INVALID_ARGUMENT, "null problem");
    const Problem &p = *reinterpret_cast<const Problem *>(pp);
    check_schedule(p, s);
    QAIA_CHECK(W >= 0, QAIA_INVALID_ARGUMENT, "W must be >= 0");
    QAIA_CHECK(R >= 1, QAIA_INVALID_ARGUMENT, "R must be >= 1");
    QAIA_CHECK(W <= (int64_t(1) << 40) / R, QAIA_INVALID_ARGUMENT, "W * R too large");
    const int64_t rows = W * (int64_t)R;
    QAIA_CHECK(rows == 0 || (weights && spins && obj), QAIA_INVALID_ARGUMENT, "null weights, spins or obj");
    QAIA_CHECK(trace_steps >= 0, QAIA_INVALID_ARGUMENT, "trace_steps must be >= 0");
    QAIA_CHECK(trace_steps == 0 || trace != nullptr, QAIA_INVALID_ARGUMENT, "null trace buffer");
    const int path = plan_path(p, *s, trace_steps > 0);
    const WsLayout L = full_layout(p, W, R, *s, path);
    QAIA_CHECK(ws != nullptr, QAIA_INVALID_ARGUMENT, "null workspace");
    if (no_alloc) {
        QAIA_CHECK(L.total <= ws_bytes, QAIA_WORKSPACE_TOO_SMALL,
                   "this call needs " + std::to_string(L.total) +
                       " bytes of scratch; the allocation-free entry point holds at most " +
                       std::to_string(ws_bytes));
        QAIA_CHECK(path != QAIA_PATH_SPARSE_REG ||
                       sparse_reg_ready(p, s->variant, trace_steps > 0, s->dt * s->noise_alpha != 0.0f,
                                        s->precision == QAIA_FP16),
                   QAIA_UNSUPPORTED,
                   "the generated kernel for this schedule is built on first use, which allocates; "
                   "run qaia_sample once with the same schedule kind first, or choose another path");
    }
    QAIA_CHECK(ws_bytes >= L.total, QAIA_WORKSPACE_TOO_SMALL,
               "sample workspace needs " + std::to_string(L.total) + " bytes");
    hipStream_t st = (hipStream_t)stream;
    DeviceGuard g(p.device);
    launch_prep(p, weights, W, *s, ws, L, st);
    if (rows == 0) return QAIA_OK;
    if (is_dense_path(path))
        launch_dense(p, weights, W, R, *s, ws, L, spins, obj, trace_steps ? trace : nullptr,
                     trace_steps, path == QAIA_PATH_DENSE_STAGED, st);
    else if (path == QAIA_PATH_SPARSE_REG)
        launch_sparse_reg(p, s->variant, W, R, *s, ws, L, spins, obj, trace_steps ? trace : nullptr,
                          trace_steps, st);
    else
        launch_sparse_lds(p, W, R, *s, ws, L, spins, obj, trace_steps ? trace : nullptr,
                          trace_steps, st);
    return QAIA_OK;
}

}  // namespace
}  // namespace qaia

using namespace qaia;

extern "C" {

int32_t qaia_abi_version(void) { return QAIA_ABI_VERSION; }

const char *qaia_status_string(int32_t status) {
    switch (status) {
        case QAIA_OK: return "ok";
        case QAIA_INVALID_ARGUMENT: return "invalid argument";
        case QAIA_UNSUPPORTED: return "unsupported";
        case QAIA_OUT_OF_MEMORY: return "out of memory";
        case QAIA_DEVICE_ERROR: return "device error";
        case QAIA_OVERFLOW: return "overflow";
        case QAIA_WORKSPACE_TOO_SMALL: return "workspace too small";
        default: return "unknown status";
    }
}

const char *qaia_last_error(void) { return last_error_cstr(); }

int32_t qaia_problem_create(int32_t n, int32_t m, int64_t num_edges, const int32_t *edge_u,
                            const int32_t *edge_v, const int32_t *weights, int32_t frac_bits,
                            int32_t device, qaia_problem **out) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(out != nullptr, QAIA_INVALID_ARGUMENT, "null output pointer");
        Problem *p = build_problem(n, m, num_edges, edge_u, edge_v, weights, frac_bits, device);
        *out = reinterpret_cast<qaia_problem *>(p);
        return QAIA_OK;
    });
}

int32_t qaia_problem_destroy(qaia_problem *p) {
    return guarded([&]() -> int32_t {
        delete reinterpret_cast<Problem *>(p);
        return QAIA_OK;
    });
}

int32_t qaia_problem_info(const qaia_problem *pp, int32_t *n, int32_t *m, int64_t *num_edges,
                          int64_t *total_weight) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(pp != nullptr, QAIA_INVALID_ARGUMENT, "null problem");
        const Problem &p = *reinterpret_cast<const Problem *>(pp);
        if (n) *n = p.n;
        if (m) *m = p.m;
        if (num_edges) *num_edges = p.E;
        if (total_weight) std::memcpy(total_weight, p.total.data(), sizeof(int64_t) * p.m);
        return QAIA_OK;
    });
}

int32_t qaia_sample_workspace_bytes(const qaia_problem *pp, int64_t W, int32_t R,
                                    const qaia_schedule *s, size_t *bytes) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(pp != nullptr && bytes != nullptr, QAIA_INVALID_ARGUMENT, "null argument");
        const Problem &p = *reinterpret_cast<const Problem *>(pp);
        check_schedule(p, s);
        QAIA_CHECK(W >= 0 && R >= 1, QAIA_INVALID_ARGUMENT, "W must be >= 0 and R >= 1");
        *bytes = full_layout(p, W, R, *s, plan_path(p, *s, false)).total;
        return QAIA_OK;
    });
}

int32_t qaia_sample(const qaia_problem *p, const float *weights, int64_t W, int32_t R,
                    const qaia_schedule *s, uint64_t *spins, int64_t *obj, void *workspace,
                    size_t ws_bytes, void *hip_stream) {
    return guarded([&]() {
        return sample_impl(p, weights, W, R, s, spins, obj, workspace, ws_bytes, nullptr, 0,
                           hip_stream);
    });
}

int32_t qaia_sample_trace(const qaia_problem *p, const float *weights, int64_t W, int32_t R,
                          const qaia_schedule *s, uint64_t *spins, int64_t *obj, void *workspace,
                          size_t ws_bytes, float *x_trace, int32_t trace_steps, void *hip_stream) {
    return guarded([&]() {
        return sample_impl(p, weights, W, R, s, spins, obj, workspace, ws_bytes, x_trace,
                           trace_steps, hip_stream);
    });
}

int32_t qaia_sample_noalloc(const qaia_problem *pp, const float *weights, int64_t W, int32_t R,
                            const qaia_schedule *s, uint64_t *spins, int64_t *obj, int64_t *bad_row,
                            void *hip_stream) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(pp != nullptr, QAIA_INVALID_ARGUMENT, "null problem");
        const Problem &p = *reinterpret_cast<const Problem *>(pp);
        void *scratch = noalloc_scratch(p.device);
        const int32_t rc = sample_impl(pp, weights, W, R, s, spins, obj, scratch, noalloc_scratch_bytes(),
                                       nullptr, 0, hip_stream, true);
        if (rc == QAIA_OK && bad_row != nullptr) {
            DeviceGuard g(p.device);
            launch_noalloc_bad_row(scratch, bad_row, (hipStream_t)hip_stream);
        }
        return rc;
    });
}

int32_t qaia_workspace_status(const void *workspace, int64_t *bad_row) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(workspace != nullptr, QAIA_INVALID_ARGUMENT, "null workspace");
        WsHeader h;
        QAIA_HIP(hipMemcpy(&h, workspace, sizeof(h), hipMemcpyDeviceToHost));
        QAIA_CHECK(h.magic == kWsMagic, QAIA_INVALID_ARGUMENT, "not a sampling workspace");
        if (bad_row) *bad_row = h.bad_row == INT64_MAX ? -1 : h.bad_row;
        if (h.bad_row != INT64_MAX)
            return fail(QAIA_INVALID_ARGUMENT,
                        "weight row " + std::to_string(h.bad_row) + " is negative, non-finite or all zero");
        return QAIA_OK;
    });
}

int32_t qaia_evaluate(const qaia_problem *pp, const uint64_t *spins, int64_t count, int64_t *obj,
                      void *hip_stream) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(pp != nullptr, QAIA_INVALID_ARGUMENT, "null problem");
        QAIA_CHECK(count >= 0, QAIA_INVALID_ARGUMENT, "count must be >= 0");
        QAIA_CHECK(count == 0 || (spins && obj), QAIA_INVALID_ARGUMENT, "null spins or obj");
        const Problem &p = *reinterpret_cast<const Problem *>(pp);
        DeviceGuard g(p.device);
        launch_evaluate(p, spins, count, obj, (hipStream_t)hip_stream);
        return QAIA_OK;
    });
}

int32_t qaia_enumerate_cuts(const qaia_problem *pp, uint64_t first, int64_t count, int64_t *obj,
                            void *hip_stream) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(pp != nullptr, QAIA_INVALID_ARGUMENT, "null problem");
        QAIA_CHECK(count >= 0, QAIA_INVALID_ARGUMENT, "count must be >= 0");
        QAIA_CHECK(count == 0 || obj != nullptr, QAIA_INVALID_ARGUMENT, "null obj");
        const Problem &p = *reinterpret_cast<const Problem *>(pp);
        QAIA_CHECK(p.n <= 63, QAIA_UNSUPPORTED, "enumeration needs n <= 63");
        const uint64_t limit = 1ull << p.n;
        QAIA_CHECK(first <= limit && (uint64_t)count <= limit - first, QAIA_INVALID_ARGUMENT,
                   "first + count exceeds 2^n");
        DeviceGuard g(p.device);
        launch_enumerate(p, first, count, obj, (hipStream_t)hip_stream);
        return QAIA_OK;
    });
}

int32_t qaia_random_spins(int32_t n, int64_t count, uint64_t seed, uint64_t offset, uint64_t *spins,
                          void *hip_stream) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(n >= 1, QAIA_INVALID_ARGUMENT, "n must be >= 1");
        QAIA_CHECK(count >= 0, QAIA_INVALID_ARGUMENT, "count must be >= 0");
        QAIA_CHECK(count == 0 || spins != nullptr, QAIA_INVALID_ARGUMENT, "null spins");
        launch_random_spins(n, count, seed, offset, spins, (hipStream_t)hip_stream);
        return QAIA_OK;
    });
}

int32_t qaia_dirichlet_weights(int32_t m, int64_t count, uint64_t seed, uint64_t offset, float *weights,
                               void *hip_stream) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(m >= 1 && m <= 8, QAIA_INVALID_ARGUMENT, "m must be in [1, 8]");
        QAIA_CHECK(count >= 0, QAIA_INVALID_ARGUMENT, "count must be >= 0");
        QAIA_CHECK(count == 0 || weights != nullptr, QAIA_INVALID_ARGUMENT, "null weights");
        launch_dirichlet(m, count, seed, offset, weights, (hipStream_t)hip_stream);
        return QAIA_OK;
    });
}

int32_t qaia_dense_field_workspace_bytes(const qaia_problem *pp, int32_t precision, int64_t count,
                                         size_t *bytes) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(pp != nullptr && bytes != nullptr, QAIA_INVALID_ARGUMENT, "null argument");
        QAIA_CHECK(precision >= QAIA_FP32 && precision <= QAIA_FP8, QAIA_INVALID_ARGUMENT, "unknown precision");
        QAIA_CHECK(count >= 0, QAIA_INVALID_ARGUMENT, "count must be >= 0");
        const Problem &p = *reinterpret_cast<const Problem *>(pp);
        std::string why;
        QAIA_CHECK(dense_supported(p, &why), QAIA_UNSUPPORTED, "dense path: " + why);
        *bytes = dense_field_ws_bytes(p, precision, count);
        return QAIA_OK;
    });
}

int32_t qaia_dense_field(const qaia_problem *pp, int32_t precision, const float *phi, int64_t count,
                         float *field, void *workspace, size_t ws_bytes, void *hip_stream) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(pp != nullptr, QAIA_INVALID_ARGUMENT, "null problem");
        QAIA_CHECK(precision >= QAIA_FP32 && precision <= QAIA_FP8, QAIA_INVALID_ARGUMENT, "unknown precision");
        QAIA_CHECK(count >= 0 && count <= (int64_t(1) << 30), QAIA_INVALID_ARGUMENT, "count out of range");
        QAIA_CHECK(count == 0 || (phi && field && workspace), QAIA_INVALID_ARGUMENT, "null buffer");
        const Problem &p = *reinterpret_cast<const Problem *>(pp);
        DeviceGuard g(p.device);
        launch_dense_field(p, precision, phi, count, field, workspace, ws_bytes, (hipStream_t)hip_stream);
        return QAIA_OK;
    });
}

int32_t qaia_pareto_filter_workspace_bytes(int64_t M, int32_t m, size_t *bytes) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(bytes != nullptr, QAIA_INVALID_ARGUMENT, "null argument");
        QAIA_CHECK(M >= 0 && M < (int64_t(1) << 31), QAIA_INVALID_ARGUMENT, "M must be in [0, 2^31)");
        QAIA_CHECK(m >= 1 && m <= 8, QAIA_INVALID_ARGUMENT, "m must be in [1, 8]");
        *bytes = pareto_ws_bytes(M, m);
        return QAIA_OK;
    });
}

int32_t qaia_pareto_filter(const int64_t *obj, int64_t M, int32_t m, int64_t *keep_idx,
                           int64_t *num_keep, void *workspace, size_t ws_bytes, void *hip_stream) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(M >= 0 && M < (int64_t(1) << 31), QAIA_INVALID_ARGUMENT, "M must be in [0, 2^31)");
        QAIA_CHECK(m >= 1 && m <= 8, QAIA_INVALID_ARGUMENT, "m must be in [1, 8]");
        QAIA_CHECK(num_keep != nullptr, QAIA_INVALID_ARGUMENT, "null num_keep");
        QAIA_CHECK(M == 0 || (obj && keep_idx && workspace), QAIA_INVALID_ARGUMENT,
                   "null obj, keep_idx or workspace");
        launch_pareto(obj, M, m, keep_idx, num_keep, workspace, ws_bytes, (hipStream_t)hip_stream);
        return QAIA_OK;
    });
}

int32_t qaia_objective_min(const int64_t *obj, int64_t M, int32_t m, int64_t *lo, int32_t accumulate,
                           void *hip_stream) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(M >= 0, QAIA_INVALID_ARGUMENT, "M must be >= 0");
        QAIA_CHECK(m >= 1 && m <= 8, QAIA_INVALID_ARGUMENT, "m must be in [1, 8]");
        QAIA_CHECK(lo != nullptr && (M == 0 || obj != nullptr), QAIA_INVALID_ARGUMENT, "null obj or lo");
        QAIA_CHECK(accumulate == 0 || accumulate == 1, QAIA_INVALID_ARGUMENT, "accumulate must be 0 or 1");
        launch_objective_min(obj, M, m, lo, accumulate != 0, (hipStream_t)hip_stream);
        return QAIA_OK;
    });
}

int32_t qaia_pareto_ranks_workspace_bytes(int64_t M, int32_t m, size_t *bytes) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(bytes != nullptr, QAIA_INVALID_ARGUMENT, "null argument");
        QAIA_CHECK(M >= 0 && M < (int64_t(1) << 31), QAIA_INVALID_ARGUMENT, "M must be in [0, 2^31)");
        QAIA_CHECK(m >= 1 && m <= 8, QAIA_INVALID_ARGUMENT, "m must be in [1, 8]");
        *bytes = pareto_ranks_ws_bytes(M, m);
        return QAIA_OK;
    });
}

int32_t qaia_pareto_ranks(const int64_t *obj, int64_t M, int32_t m, int32_t max_rank, int32_t *rank,
                          int32_t *num_ranks, void *workspace, size_t ws_bytes, void *hip_stream) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(M >= 0 && M < (int64_t(1) << 31), QAIA_INVALID_ARGUMENT, "M must be in [0, 2^31)");
        QAIA_CHECK(m >= 1 && m <= 8, QAIA_INVALID_ARGUMENT, "m must be in [1, 8]");
        QAIA_CHECK(max_rank >= 1, QAIA_INVALID_ARGUMENT, "max_rank must be >= 1");
        QAIA_CHECK(num_ranks != nullptr, QAIA_INVALID_ARGUMENT, "null num_ranks");
        QAIA_CHECK(M == 0 || (obj && rank && workspace), QAIA_INVALID_ARGUMENT, "null obj, rank or workspace");
        *num_ranks = launch_pareto_ranks(obj, M, m, max_rank, rank, workspace, ws_bytes, (hipStream_t)hip_stream);
        return QAIA_OK;
    });
}

int32_t qaia_hypervolume(const int64_t *pts, int64_t P, int32_t m, const int64_t *ref,
                         uint64_t hv[4], double *hv_approx) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(P >= 0, QAIA_INVALID_ARGUMENT, "P must be >= 0");
        QAIA_CHECK(m >= 1 && m <= 64, QAIA_INVALID_ARGUMENT, "m must be in [1, 64]");
        QAIA_CHECK(ref != nullptr && hv != nullptr, QAIA_INVALID_ARGUMENT, "null ref or hv");
        QAIA_CHECK(P == 0 || pts != nullptr, QAIA_INVALID_ARGUMENT, "null points");
        return hypervolume_exact(pts, P, m, ref, hv, hv_approx);
    });
}

// ---------------------------------------------------------------- learned proposer

int32_t qaia_mlp_param_count(int32_t in_dim, int64_t *count) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(count != nullptr, QAIA_INVALID_ARGUMENT, "null count");
        QAIA_CHECK(in_dim >= 1 && in_dim <= 16, QAIA_INVALID_ARGUMENT, "in_dim must be in [1, 16]");
        *count = mlp_param_count(in_dim);
        return QAIA_OK;
    });
}

int32_t qaia_mlp_forward_workspace_bytes(int64_t N, size_t *bytes) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(bytes != nullptr && N >= 0, QAIA_INVALID_ARGUMENT, "bad argument");
        *bytes = mlp_forward_ws_bytes(N);
        return QAIA_OK;
    });
}

int32_t qaia_mlp_forward(const uint16_t *params, int32_t in_dim, const float *X, int64_t N, float *logits,
                         void *workspace, size_t ws_bytes, void *hip_stream) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(N >= 0 && N <= (int64_t(1) << 26), QAIA_INVALID_ARGUMENT, "N out of range");
        QAIA_CHECK(N == 0 || (params && X && logits && workspace), QAIA_INVALID_ARGUMENT, "null buffer");
        QAIA_CHECK(ws_bytes >= mlp_forward_ws_bytes(N), QAIA_WORKSPACE_TOO_SMALL, "forward workspace too small");
        launch_mlp_forward(params, in_dim, X, N, logits, workspace, (hipStream_t)hip_stream);
        return QAIA_OK;
    });
}

int32_t qaia_mlp_backward_workspace_bytes(int32_t in_dim, int64_t B, size_t *bytes) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(bytes != nullptr && B >= 1, QAIA_INVALID_ARGUMENT, "bad argument");
        *bytes = mlp_backward_ws_bytes(in_dim, B);
        return QAIA_OK;
    });
}

int32_t qaia_mlp_backward(const uint16_t *params, int32_t in_dim, const float *X, const float *labels,
                          int64_t B, float *grad, float *logits, void *workspace, size_t ws_bytes,
                          void *hip_stream) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(B >= 1 && B <= (int64_t(1) << 24), QAIA_INVALID_ARGUMENT, "B out of range");
        QAIA_CHECK(params && X && labels && grad && workspace, QAIA_INVALID_ARGUMENT, "null buffer");
        QAIA_CHECK(ws_bytes >= mlp_backward_ws_bytes(in_dim, B), QAIA_WORKSPACE_TOO_SMALL,
                   "backward workspace too small");
        launch_mlp_backward(params, in_dim, X, labels, B, grad, logits, workspace, (hipStream_t)hip_stream);
        return QAIA_OK;
    });
}

int32_t qaia_mlp_train_workspace_bytes(int32_t in_dim, int64_t n, int32_t batch, size_t *bytes) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(bytes != nullptr, QAIA_INVALID_ARGUMENT, "null argument");
        QAIA_CHECK(in_dim >= 1 && in_dim <= 16 && n >= 1 && batch >= 1, QAIA_INVALID_ARGUMENT,
                   "need 1 <= in_dim <= 16, n >= 1, batch >= 1");
        *bytes = mlp_train_ws_bytes(in_dim, n, batch);
        return QAIA_OK;
    });
}

int32_t qaia_mlp_train(float *master, uint16_t *params, float *moment1, float *moment2, int32_t in_dim,
                       const float *X, const float *labels, int64_t n, int32_t batch, int32_t steps,
                       int32_t first_step, float lr, uint64_t seed, void *workspace, size_t ws_bytes,
                       void *hip_stream) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(master && params && moment1 && moment2 && X && labels && workspace, QAIA_INVALID_ARGUMENT,
                   "null buffer");
        QAIA_CHECK(lr > 0.0f && std::isfinite(lr), QAIA_INVALID_ARGUMENT, "lr must be finite and > 0");
        QAIA_CHECK(n < (int64_t(1) << 31), QAIA_INVALID_ARGUMENT, "n must be < 2^31");
        launch_mlp_train(master, params, moment1, moment2, in_dim, X, labels, n, batch, steps, first_step, lr, seed,
                         workspace, ws_bytes, (hipStream_t)hip_stream);
        return QAIA_OK;
    });
}

int32_t qaia_mlp_adam(float *master, uint16_t *params, float *moment1, float *moment2, const float *grad,
                      int64_t count, int32_t step, float lr, float beta1, float beta2, float eps,
                      void *hip_stream) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(count >= 0, QAIA_INVALID_ARGUMENT, "count must be >= 0");
        QAIA_CHECK(count == 0 || (master && params && moment1 && moment2 && grad), QAIA_INVALID_ARGUMENT,
                   "null buffer");
        QAIA_CHECK(lr > 0.0f && beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f,
                   QAIA_INVALID_ARGUMENT, "bad Adam hyper-parameters");
        if (count) launch_adam(master, params, moment1, moment2, grad, count, step, lr, beta1, beta2, eps,
                               (hipStream_t)hip_stream);
        return QAIA_OK;
    });
}

int32_t qaia_front_features_workspace_bytes(int64_t P, int32_t m, size_t *bytes) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(bytes != nullptr && P >= 0 && m >= 1 && m <= 8, QAIA_INVALID_ARGUMENT, "bad argument");
        *bytes = features_ws_bytes(P, m);
        return QAIA_OK;
    });
}

int32_t qaia_front_features(const int64_t *front, int64_t P, int32_t m, const float *cands, int64_t N,
                            const float *hits, int64_t n_hits, const float *misses, int64_t n_misses,
                            float *feat, void *workspace, size_t ws_bytes, void *hip_stream) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(P >= 0 && N >= 0 && n_hits >= 0 && n_misses >= 0, QAIA_INVALID_ARGUMENT, "negative size");
        QAIA_CHECK((P == 0 || front) && (N == 0 || (cands && feat)) && (n_hits == 0 || hits) &&
                       (n_misses == 0 || misses) && workspace,
                   QAIA_INVALID_ARGUMENT, "null buffer");
        launch_features(front, P, m, cands, N, hits, n_hits, misses, n_misses, feat, workspace, ws_bytes,
                        (hipStream_t)hip_stream);
        return QAIA_OK;
    });
}

int32_t qaia_topk_workspace_bytes(int64_t N, size_t *bytes) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(bytes != nullptr && N >= 1 && N < (int64_t(1) << 31), QAIA_INVALID_ARGUMENT, "bad argument");
        *bytes = topk_ws_bytes(N);
        return QAIA_OK;
    });
}

int32_t qaia_topk(const float *scores, int64_t N, int64_t k, float temperature, uint64_t seed, int64_t *idx,
                  void *workspace, size_t ws_bytes, void *hip_stream) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(scores && idx && workspace, QAIA_INVALID_ARGUMENT, "null buffer");
        launch_topk(scores, N, k, temperature, seed, idx, workspace, ws_bytes, (hipStream_t)hip_stream);
        return QAIA_OK;
    });
}

int32_t qaia_new_point_labels(const int64_t *keep_idx, const int64_t *num_keep, int64_t archive_rows,
                              int32_t R, int64_t W, float *labels, void *hip_stream) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(keep_idx && num_keep && (W == 0 || labels), QAIA_INVALID_ARGUMENT, "null buffer");
        launch_labels(keep_idx, num_keep, archive_rows, R, W, labels, (hipStream_t)hip_stream);
        return QAIA_OK;
    });
}

int32_t qaia_gather_rows(const void *src, int32_t width, const int64_t *idx, const int64_t *count,
                         int64_t cap, void *dst, void *hip_stream) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(src && idx && count && dst, QAIA_INVALID_ARGUMENT, "null buffer");
        launch_gather_rows((const uint32_t *)src, width, idx, count, cap, (uint32_t *)dst,
                           (hipStream_t)hip_stream);
        return QAIA_OK;
    });
}

// ---------------------------------------------------------------- measurement kernels

int32_t qaia_peak_fma(int64_t blocks, int32_t iters, float a, float b, float *out, void *hip_stream) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(blocks >= 1 && blocks <= INT32_MAX, QAIA_INVALID_ARGUMENT, "blocks must be in [1, 2^31)");
        QAIA_CHECK(iters >= 1, QAIA_INVALID_ARGUMENT, "iters must be >= 1");
        QAIA_CHECK(out != nullptr, QAIA_INVALID_ARGUMENT, "null out");
        launch_peak_fma(blocks, iters, a, b, out, (hipStream_t)hip_stream);
        return QAIA_OK;
    });
}

int32_t qaia_peak_valu(int64_t blocks, int32_t iters, float k, float *out, void *hip_stream) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(blocks >= 1 && blocks <= INT32_MAX, QAIA_INVALID_ARGUMENT, "blocks must be in [1, 2^31)");
        QAIA_CHECK(iters >= 1, QAIA_INVALID_ARGUMENT, "iters must be >= 1");
        QAIA_CHECK(out != nullptr, QAIA_INVALID_ARGUMENT, "null out");
        QAIA_CHECK(std::isfinite(k), QAIA_INVALID_ARGUMENT, "k must be finite");
        launch_peak_valu(blocks, iters, k, out, (hipStream_t)hip_stream);
        return QAIA_OK;
    });
}

int32_t qaia_peak_mfma(int32_t precision, int64_t blocks, int32_t iters, float *out, void *hip_stream) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(precision == QAIA_FP32 || precision == QAIA_BF16 || precision == QAIA_FP8,
                   QAIA_INVALID_ARGUMENT, "unknown precision");
        QAIA_CHECK(blocks >= 1 && blocks <= INT32_MAX, QAIA_INVALID_ARGUMENT, "blocks must be in [1, 2^31)");
        const int64_t K = precision == QAIA_FP32 ? 2 : (precision == QAIA_BF16 ? 16 : 64);
        QAIA_CHECK(iters >= 1 && 4 * K * (int64_t)iters < (int64_t(1) << 24), QAIA_INVALID_ARGUMENT,
                   "iters must be >= 1 with 4 K iters < 2^24");
        QAIA_CHECK(out != nullptr, QAIA_INVALID_ARGUMENT, "null out");
        launch_peak_mfma(precision, blocks, iters, out, (hipStream_t)hip_stream);
        return QAIA_OK;
    });
}

int32_t qaia_peak_copy(const void *src, void *dst, size_t bytes, void *hip_stream) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(bytes % 16 == 0, QAIA_INVALID_ARGUMENT, "bytes must be a multiple of 16");
        QAIA_CHECK(bytes == 0 || (src && dst), QAIA_INVALID_ARGUMENT, "null buffer");
        QAIA_CHECK(((uintptr_t)src | (uintptr_t)dst) % 16 == 0, QAIA_INVALID_ARGUMENT,
                   "buffers must be 16-byte aligned");
        const uintptr_t s0 = (uintptr_t)src, d0 = (uintptr_t)dst;
        QAIA_CHECK(bytes == 0 || s0 + bytes <= d0 || d0 + bytes <= s0, QAIA_INVALID_ARGUMENT,
                   "buffers overlap");
        launch_peak_copy(src, dst, bytes, (hipStream_t)hip_stream);
        return QAIA_OK;
    });
}

// ---------------------------------------------------------------- batching form

int32_t qaia_sample_batch_workspace_bytes(const qaia_batch_item *items, int32_t count, const qaia_schedule *s,
                                          size_t *bytes) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(bytes != nullptr && count >= 0 && (count == 0 || items), QAIA_INVALID_ARGUMENT, "bad argument");
        if (count == 0) {
            *bytes = 256;
            return QAIA_OK;
        }
        check_schedule(*reinterpret_cast<const Problem *>(items[0].problem), s);
        *bytes = batch_ws_bytes(items, count, *s);
        return QAIA_OK;
    });
}

int32_t qaia_sample_batch(const qaia_batch_item *items, int32_t count, const qaia_schedule *s, void *workspace,
                          size_t ws_bytes, void *hip_stream) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(count >= 0 && (count == 0 || items), QAIA_INVALID_ARGUMENT, "bad items");
        if (count == 0) return QAIA_OK;
        QAIA_CHECK(items[0].problem != nullptr, QAIA_INVALID_ARGUMENT, "null problem");
        check_schedule(*reinterpret_cast<const Problem *>(items[0].problem), s);
        sample_batch(items, count, *s, workspace, ws_bytes, (hipStream_t)hip_stream);
        return QAIA_OK;
    });
}

int32_t qaia_plan_autotune_workspace_bytes(const qaia_batch_item *items, int32_t count, const qaia_schedule *s,
                                           int32_t probe_steps, size_t *bytes) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(bytes != nullptr && count >= 0 && (count == 0 || items) && probe_steps >= 1,
                   QAIA_INVALID_ARGUMENT, "bad argument");
        if (count == 0) {
            *bytes = 256;
            return QAIA_OK;
        }
        check_schedule(*reinterpret_cast<const Problem *>(items[0].problem), s);
        *bytes = autotune_ws_bytes(items, count, *s, probe_steps);
        return QAIA_OK;
    });
}

int32_t qaia_plan_autotune(qaia_batch_item *items, int32_t count, const qaia_schedule *s, int32_t probe_steps,
                           double *est_seconds, void *workspace, size_t ws_bytes, void *hip_stream) {
    return guarded([&]() -> int32_t {
        QAIA_CHECK(count >= 0 && (count == 0 || items) && workspace, QAIA_INVALID_ARGUMENT, "bad argument");
        if (count == 0) return QAIA_OK;
        QAIA_CHECK(items[0].problem != nullptr, QAIA_INVALID_ARGUMENT, "null problem");
        check_schedule(*reinterpret_cast<const Problem *>(items[0].problem), s);
        autotune(items, count, *s, probe_steps, est_seconds, workspace, ws_bytes, (hipStream_t)hip_stream);
        return QAIA_OK;
    });
}

}  // extern "C"
