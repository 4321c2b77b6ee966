// Weight preparation, the generic sparse SB kernel (one spin per lane, state
// and adjacency in LDS) and exact cut evaluation.
#include <climits>

#include <algorithm>

#include "device_common.hpp"
#include "internal.hpp"

namespace qaia {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// Workspace header reset (a fill kernel rather than a memset so the sequence
// stays valid inside a captured graph).
__global__ void ws_header_init(WsHeader *h, int64_t W) {
    if (threadIdx.x == 0) {
        h->magic = kWsMagic;
        h->bad_row = INT64_MAX;
        h->W = W;
        h->reserved = 0;
    }
}

// ---------------------------------------------------------------------------
// Weight preparation, one block per weight row w (Eq. 7 and the coupling scale
// of section "Simulated Bifurcation with Gaussian noise"):
//   c0 = 1 / max_i |sum_k c_k rho_{k,i}|, rho_{k,i} = sum_j W_k,ij (exact ints);
//   if that maximum is 0: c0 = 1 / max_i sum_j |J(c)_ij|; if 0 too: c0 = 0.
//   jcp[w][e] = float(-dt * c0 * sum_k c_k W_k,e)  (float64 then one rounding)
// Rows with a negative, non-finite or all-zero c are marked invalid
// (c0s[w] = -1) and reported through the workspace header.
// The first blocks also fill the per-step table kt[t] = -dt (a0 - a_t).
__global__ __launch_bounds__(kBlock) void prep_kernel(
    const float *__restrict__ weights, int64_t W, int m, int n, int64_t E,
    const int64_t *__restrict__ rho, const int32_t *__restrict__ Wt,
    const int32_t *__restrict__ rowptr, const int32_t *__restrict__ eid, double dt, double a0,
    int T, float *__restrict__ kt, double *__restrict__ c0s, float *__restrict__ jcp,
    WsHeader *hdr) {
    __shared__ double c_sh[8];
    __shared__ double red[kBlock / 64];
    __shared__ int valid_sh;
    const int tid = threadIdx.x;
    const int64_t w = blockIdx.x;

    for (int64_t t = (int64_t)blockIdx.x * kBlock + tid; t < T; t += (int64_t)gridDim.x * kBlock) {
        double at = T > 1 ? a0 * (double)t / (double)(T - 1) : 0.0;
        kt[t] = (float)(-dt * (a0 - at));
    }
    if (w >= W) return;

    if (tid == 0) {
        double s = 0.0;
        int ok = 1;
        for (int k = 0; k < m; ++k) {
            float c = weights[w * m + k];
            if (!(c >= 0.0f) || !isfinite(c)) ok = 0;  // catches NaN too
            c_sh[k] = (double)c;
            s += (double)c;
        }
        if (!(s > 0.0)) ok = 0;
        valid_sh = ok;
    }
    __syncthreads();
    if (!valid_sh) {
        if (tid == 0) {
            c0s[w] = -1.0;
            atomicMin((unsigned long long *)&hdr->bad_row, (unsigned long long)w);
        }
        if (jcp)
            for (int64_t e = tid; e < E; e += kBlock) jcp[w * E + e] = 0.0f;
        return;
    }

    auto block_max = [&](double v) -> double {
        for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
        if ((tid & 63) == 0) red[tid >> 6] = v;
        __syncthreads();
        double r = red[0];
        for (int i = 1; i < kBlock / 64; ++i) r = fmax(r, red[i]);
        __syncthreads();
        return r;
    };

    double mx = 0.0;
    for (int i = tid; i < n; i += kBlock) {
        double row = 0.0;
        for (int k = 0; k < m; ++k) row += c_sh[k] * (double)rho[(int64_t)k * n + i];
        mx = fmax(mx, fabs(row));
    }
    mx = block_max(mx);
    double c0;
    if (mx > 0.0) {
        c0 = 1.0 / mx;
    } else {
        double mxa = 0.0;
        for (int i = tid; i < n; i += kBlock) {
            double a = 0.0;
            for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
                double j = 0.0;
                for (int k = 0; k < m; ++k) j += c_sh[k] * (double)Wt[(int64_t)k * E + eid[p]];
                a += fabs(j);
            }
            mxa = fmax(mxa, a);
        }
        mxa = block_max(mxa);
        c0 = mxa > 0.0 ? 1.0 / mxa : 0.0;
    }
    if (tid == 0) c0s[w] = c0;
    if (jcp) {
        const double coef = -dt * c0;
        for (int64_t e = tid; e < E; e += kBlock) {
            double j = 0.0;
            for (int k = 0; k < m; ++k) j += c_sh[k] * (double)Wt[(int64_t)k * E + e];
            jcp[w * E + e] = (float)(coef * j);
        }
    }
}

WsLayout sample_ws_layout(const Problem &p, int64_t W, int32_t R, const qaia_schedule &s, bool edge_coefs) {
    (void)R;
    WsLayout L;
    size_t off = 0;
    L.header = off;
    off += align256(sizeof(WsHeader));
    L.kt = off;
    off += align256(sizeof(float) * (size_t)s.steps);
    L.c0s = off;
    off += align256(sizeof(double) * (size_t)W);
    L.jcp = off;
    L.has_jcp = edge_coefs && W > 0 && p.E > 0;
    if (L.has_jcp) off += align256(sizeof(float) * (size_t)W * (size_t)p.E);
    L.total = off;
    return L;
}

void launch_prep(const Problem &p, const float *weights, int64_t W, const qaia_schedule &s,
                 void *ws, const WsLayout &L, hipStream_t st) {
    char *b = (char *)ws;
    WsHeader *hdr = (WsHeader *)(b + L.header);
    hipLaunchKernelGGL(ws_header_init, dim3(1), dim3(64), 0, st, hdr, W);
    QAIA_HIP(hipGetLastError());
    int64_t grid = W > 0 ? W : 1;
    int64_t need_kt = (s.steps + kBlock - 1) / kBlock;
    if (grid < need_kt) grid = need_kt;
    QAIA_CHECK(grid <= INT32_MAX, QAIA_INVALID_ARGUMENT, "too many weight rows");
    hipLaunchKernelGGL(prep_kernel, dim3((unsigned)grid), dim3(kBlock), 0, st, weights, W, p.m,
                       p.n, p.E, p.d_rho, p.d_W, p.d_rowptr, p.d_eid, (double)s.dt, (double)s.a0,
                       s.steps, (float *)(b + L.kt), (double *)(b + L.c0s),
                       L.has_jcp ? (float *)(b + L.jcp) : nullptr, hdr);
    QAIA_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Generic sparse SB kernel.  Lanes map to (replica, spin) pairs: with
// rpb = max(1, 256 / n) replicas per block, slot L = q * 256 + tid (q < NPT)
// covers spin L % n of local replica L / n.  x is double-buffered in LDS so
// every force uses the pre-step x (Eq. 9); each lane keeps its own y, x and
// its neighbour list (LDS offsets and folded coefficients) in registers.
// After T steps the block reads out sgn(x) and evaluates the exact cut
// vector of each replica with wave reductions.  The body works on one
// SparseJob (one problem's rows); the batched kernel maps blocks to jobs.
template <int MAXDEG, int NPT, bool DSB>
__device__ void sparse_lds_body(const SparseJob &j, int64_t block, float *xs) {
    const int n = j.n, rpb = j.rpb, R = j.R, T = j.T;
    const int64_t E = j.E, rows = j.rows;
    const int tid = threadIdx.x;
    const int span = rpb * n;
    const int64_t row0 = block * rpb;

    float x[NPT], y[NPT], jv[NPT][MAXDEG];
    int nb[NPT][MAXDEG], deg[NPT], node[NPT];
    int64_t rowq[NPT];
    bool act[NPT];
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
        const int L = q * kBlock + tid;
        const int rl = L / n;
        node[q] = L - rl * n;
        rowq[q] = row0 + rl;
        act[q] = L < span && rowq[q] < rows;
        deg[q] = 0;
        x[q] = y[q] = 0.0f;
        if (act[q]) {
            const int i = node[q];
            const int64_t w = rowq[q] / R;
            const uint64_t g = (uint64_t)rowq[q] + j.offset;
            x[q] = init_value(j.seed, init_counter(g, n, i, 0), j.amp);
            y[q] = init_value(j.seed, init_counter(g, n, i, 1), j.amp);
            const int p0 = j.rowptr[i];
            deg[q] = j.rowptr[i + 1] - p0;
#pragma unroll
            for (int d = 0; d < MAXDEG; ++d) {
                if (d < deg[q]) {
                    nb[q][d] = rl * n + j.col[p0 + d];
                    jv[q][d] = j.jcp[w * E + j.eid[p0 + d]];
                } else {
                    nb[q][d] = 0;
                    jv[q][d] = 0.0f;
                }
            }
            xs[L] = x[q];
        }
    }
    __syncthreads();
    int cur = 0;
    for (int t = 0; t < T; ++t) {
        const float kt = j.kt_tab[t];
        const float *xc = xs + cur * span;
        float *xn = xs + (cur ^ 1) * span;
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
            if (!act[q]) continue;
            float acc = fmaf(kt, x[q], y[q]);
#pragma unroll
            for (int d = 0; d < MAXDEG; ++d) {
                if (d < deg[q]) {
                    float v = xc[nb[q][d]];
                    if (DSB) v = sgn1(v);
                    acc = fmaf(jv[q][d], v, acc);
                }
            }
            if (j.dt_alpha != 0.0f) {
                const uint64_t g = (uint64_t)rowq[q] + j.offset;
                const uint64_t nidx = (g * (uint64_t)T + (uint64_t)t) * (uint64_t)n + node[q];
                acc = fmaf(j.dt_alpha, noise_value(j.seed, nidx), acc);
            }
            y[q] = acc;
            x[q] = fmaf(j.dta0, y[q], x[q]);
            wall(x[q], y[q]);
            xn[q * kBlock + tid] = x[q];
            if (j.trace != nullptr && t < j.trace_steps)
                j.trace[(rowq[q] * j.trace_steps + t) * n + node[q]] = x[q];
        }
        __syncthreads();
        cur ^= 1;
    }

    // read-out and exact cut evaluation, one wave per local replica
    const float *xf = xs + cur * span;
    const int lane = tid & 63, wave = tid >> 6;
    const int m = j.m, words = j.words;
    for (int rl = wave; rl < rpb; rl += kBlock / 64) {
        const int64_t row = row0 + rl;
        if (row >= rows) break;
        const bool valid = j.c0s[row / R] >= 0.0;
        const float *xr = xf + rl * n;
        for (int wd = lane; wd < words; wd += 64) {
            uint64_t bits = 0;
            if (valid)
                for (int b = 0; b < 64 && wd * 64 + b < n; ++b)
                    bits |= (uint64_t)(xr[wd * 64 + b] < 0.0f) << b;
            j.spins[row * words + wd] = bits;
        }
        int64_t acc[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] = 0;
        if (valid) {
            for (int64_t e = lane; e < E; e += 64) {
                const bool cut = (xr[j.eu[e]] < 0.0f) != (xr[j.ev[e]] < 0.0f);
                if (cut) {
#pragma unroll
                    for (int k = 0; k < 8; ++k)
                        if (k < m) acc[k] += (int64_t)j.Wt[(int64_t)k * E + e];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (k >= m) break;
            int64_t v = acc[k];
            for (int off = 32; off > 0; off >>= 1) {
                int lo = __shfl_xor((int)(uint32_t)v, off);
                int hi = __shfl_xor((int)(v >> 32), off);
                v += (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
            }
            if (lane == 0) j.obj[row * m + k] = v;
        }
    }
}

template <int MAXDEG, int NPT, bool DSB>
__global__ __launch_bounds__(kBlock) void sparse_lds_kernel(SparseJob j) {
    extern __shared__ float xs[];  // [2][rpb * n]
    sparse_lds_body<MAXDEG, NPT, DSB>(j, blockIdx.x, xs);
}

// Ragged batch: block b runs job i with block_start[i] <= b < block_start[i + 1].
template <int MAXDEG, int NPT, bool DSB>
__global__ __launch_bounds__(kBlock) void sparse_lds_batch_kernel(const SparseJob *__restrict__ jobs,
                                                                  int count,
                                                                  const int64_t *__restrict__ block_start) {
    extern __shared__ float xs[];
    const int64_t b = blockIdx.x;
    int i = 0;
    while (i + 1 < count && block_start[i + 1] <= b) ++i;
    const SparseJob j = jobs[i];
    sparse_lds_body<MAXDEG, NPT, DSB>(j, b - block_start[i], xs);
}

// Persistent ragged batch: the grid is what the GPU holds at once, and each
// block takes work units (one block's worth of one job's replicas) from a
// device queue until it is empty; unit u belongs to job i with
// block_start[i] <= u < block_start[i + 1] (jobs in decreasing cost per unit,
// so the long units start first).
template <int MAXDEG, int NPT, bool DSB>
__global__ __launch_bounds__(kBlock) void sparse_lds_queue_kernel(const SparseJob *__restrict__ jobs, int count,
                                                                  const int64_t *__restrict__ block_start,
                                                                  int64_t units,
                                                                  unsigned long long *__restrict__ queue) {
    extern __shared__ float xs[];
    __shared__ int64_t unit_sh;
    while (true) {
        if (threadIdx.x == 0) unit_sh = (int64_t)atomicAdd(queue, 1ull);
        __syncthreads();
        const int64_t u = unit_sh;
        __syncthreads();  // every thread has read unit_sh (and the previous unit's LDS use is over)
        if (u >= units) break;
        int lo = 0, hi = count - 1;  // the last job whose start is <= u
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (block_start[mid] <= u) lo = mid;
            else hi = mid - 1;
        }
        const SparseJob j = jobs[lo];
        sparse_lds_body<MAXDEG, NPT, DSB>(j, u - block_start[lo], xs);
    }
}

__global__ void queue_reset_kernel(unsigned long long *q) {
    if (threadIdx.x == 0) *q = 0ull;
}

bool sparse_lds_supported(const Problem &p, std::string *why) {
    if (p.max_degree > 32) {
        if (why) *why = "maximum degree above 32 (use the dense path)";
        return false;
    }
    if (p.n > 16 * kBlock) {
        if (why) *why = "more than 4096 spins";
        return false;
    }
    if (p.m > 8) {
        if (why) *why = "more than 8 objectives";
        return false;
    }
    return true;
}

int sparse_lds_default_rpb(const Problem &p) { return p.n <= kBlock ? kBlock / p.n : 1; }

SparseShape sparse_lds_shape(const Problem &p, int64_t rows, int rpb) {
    SparseShape sh;
    sh.rpb = rpb > 0 ? rpb : sparse_lds_default_rpb(p);
    QAIA_CHECK((int64_t)sh.rpb * p.n <= 16 * kBlock, QAIA_UNSUPPORTED,
               "replicas per block x spins exceeds 16 spins per lane");
    const int span = sh.rpb * p.n;
    sh.npt = 1;
    while (sh.npt * kBlock < span) sh.npt <<= 1;
    sh.maxdeg = p.max_degree <= 4 ? 4 : (p.max_degree <= 8 ? 8 : (p.max_degree <= 16 ? 16 : 32));
    sh.blocks = (rows + sh.rpb - 1) / sh.rpb;
    sh.shmem = sizeof(float) * 2 * (size_t)span;
    return sh;
}

SparseJob sparse_job(const Problem &p, int64_t W, int32_t R, const qaia_schedule &s, void *ws,
                     const WsLayout &L, uint64_t *spins, int64_t *obj, float *trace, int32_t trace_steps,
                     int rpb) {
    char *b = (char *)ws;
    SparseJob j{};
    j.n = p.n;
    j.E = p.E;
    j.m = p.m;
    j.words = p.words;
    j.R = R;
    j.T = s.steps;
    j.rows = W * (int64_t)R;
    j.rpb = sparse_lds_shape(p, j.rows, rpb).rpb;
    j.rowptr = p.d_rowptr;
    j.col = p.d_col;
    j.eid = p.d_eid;
    j.Wt = p.d_W;
    j.eu = p.d_eu;
    j.ev = p.d_ev;
    j.jcp = (const float *)(b + L.jcp);
    j.c0s = (const double *)(b + L.c0s);
    j.kt_tab = (const float *)(b + L.kt);
    j.dta0 = s.dt * s.a0;
    j.dt_alpha = s.dt * s.noise_alpha;
    j.seed = s.seed;
    j.offset = s.replica_offset;
    j.amp = s.init_amp;
    j.spins = spins;
    j.obj = obj;
    j.trace = trace;
    j.trace_steps = trace_steps;
    return j;
}

template <int MAXDEG, int NPT, bool DSB>
static void launch_one(const SparseJob *single, const SparseJob *jobs, int count, const int64_t *starts,
                       int64_t blocks, size_t shmem, hipStream_t st) {
    if (single)
        hipLaunchKernelGGL((sparse_lds_kernel<MAXDEG, NPT, DSB>), dim3((unsigned)blocks), dim3(kBlock), shmem,
                           st, *single);
    else
        hipLaunchKernelGGL((sparse_lds_batch_kernel<MAXDEG, NPT, DSB>), dim3((unsigned)blocks), dim3(kBlock),
                           shmem, st, jobs, count, starts);
}

template <int MAXDEG, int NPT, bool DSB>
static void launch_queue(const SparseJob *jobs, int count, const int64_t *starts, int64_t units, size_t shmem,
                         unsigned long long *queue, hipStream_t st) {
    auto kern = sparse_lds_queue_kernel<MAXDEG, NPT, DSB>;
    int per_cu = 0, dev = 0, cus = 0;
    QAIA_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBlock, shmem));
    QAIA_HIP(hipGetDevice(&dev));
    QAIA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int64_t grid = std::min<int64_t>(units, (int64_t)std::max(per_cu, 1) * cus);
    hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(64), 0, st, queue);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kBlock), shmem, st, jobs, count, starts, units, queue);
}

template <int MAXDEG>
static void dispatch_queue(int npt, bool dsb, const SparseJob *jobs, int count, const int64_t *starts, int64_t units,
                           size_t shmem, unsigned long long *queue, hipStream_t st) {
#define QAIA_NPT(N)                                                                       \
    case N:                                                                               \
        if (dsb) launch_queue<MAXDEG, N, true>(jobs, count, starts, units, shmem, queue, st);  \
        else launch_queue<MAXDEG, N, false>(jobs, count, starts, units, shmem, queue, st);     \
        break;
    switch (npt) {
        QAIA_NPT(1)
        QAIA_NPT(2)
        QAIA_NPT(4)
        QAIA_NPT(8)
        QAIA_NPT(16)
        default:
            throw Error{QAIA_UNSUPPORTED, "spins per lane out of range"};
    }
#undef QAIA_NPT
}

void launch_sparse_lds_queue(const SparseJob *jobs, int count, const int64_t *starts, int64_t units, int maxdeg,
                             int npt, size_t shmem, bool dsb, unsigned long long *queue, hipStream_t st) {
    if (units == 0) return;
    switch (maxdeg) {
        case 4: dispatch_queue<4>(npt, dsb, jobs, count, starts, units, shmem, queue, st); break;
        case 8: dispatch_queue<8>(npt, dsb, jobs, count, starts, units, shmem, queue, st); break;
        case 16: dispatch_queue<16>(npt, dsb, jobs, count, starts, units, shmem, queue, st); break;
        default: dispatch_queue<32>(npt, dsb, jobs, count, starts, units, shmem, queue, st); break;
    }
    QAIA_HIP(hipGetLastError());
}

template <int MAXDEG>
static void dispatch_npt(int npt, bool dsb, const SparseJob *single, const SparseJob *jobs, int count,
                         const int64_t *starts, int64_t blocks, size_t shmem, hipStream_t st) {
#define QAIA_NPT(N)                                                                                   \
    case N:                                                                                           \
        if (dsb) launch_one<MAXDEG, N, true>(single, jobs, count, starts, blocks, shmem, st);         \
        else launch_one<MAXDEG, N, false>(single, jobs, count, starts, blocks, shmem, st);            \
        break;
    switch (npt) {
        QAIA_NPT(1)
        QAIA_NPT(2)
        QAIA_NPT(4)
        QAIA_NPT(8)
        QAIA_NPT(16)
        default:
            throw Error{QAIA_UNSUPPORTED, "spins per lane out of range"};
    }
#undef QAIA_NPT
}

void launch_sparse_lds_jobs(const SparseJob *single, const SparseJob *jobs, int count, const int64_t *starts,
                            int64_t blocks, int maxdeg, int npt, size_t shmem, bool dsb, hipStream_t st) {
    QAIA_CHECK(blocks <= INT32_MAX, QAIA_INVALID_ARGUMENT, "too many replicas for one launch");
    if (blocks == 0) return;
    switch (maxdeg) {
        case 4: dispatch_npt<4>(npt, dsb, single, jobs, count, starts, blocks, shmem, st); break;
        case 8: dispatch_npt<8>(npt, dsb, single, jobs, count, starts, blocks, shmem, st); break;
        case 16: dispatch_npt<16>(npt, dsb, single, jobs, count, starts, blocks, shmem, st); break;
        default: dispatch_npt<32>(npt, dsb, single, jobs, count, starts, blocks, shmem, st); break;
    }
    QAIA_HIP(hipGetLastError());
}

void launch_sparse_lds(const Problem &p, int64_t W, int32_t R, const qaia_schedule &s, void *ws,
                       const WsLayout &L, uint64_t *spins, int64_t *obj, float *trace,
                       int32_t trace_steps, hipStream_t st, int rpb) {
    std::string why;
    QAIA_CHECK(sparse_lds_supported(p, &why), QAIA_UNSUPPORTED, "sparse LDS path: " + why);
    const int64_t rows = W * (int64_t)R;
    if (rows == 0) return;
    const SparseShape sh = sparse_lds_shape(p, rows, rpb);
    const SparseJob j = sparse_job(p, W, R, s, ws, L, spins, obj, trace, trace_steps, rpb);
    launch_sparse_lds_jobs(&j, nullptr, 1, nullptr, sh.blocks, sh.maxdeg, sh.npt, sh.shmem,
                           s.variant == QAIA_DSB, st);
}

// ---------------------------------------------------------------------------
// Exact cut evaluation, Eq. (1), for given packed spins.
// Few edges: one thread per sample.  Many edges: one block per sample with a
// block reduction.
__device__ __forceinline__ int spin_bit(const uint64_t *row, int i) {
    return (int)((row[i >> 6] >> (i & 63)) & 1ull);
}

__global__ __launch_bounds__(kBlock) void eval_thread_kernel(
    const uint64_t *__restrict__ spins, int64_t count, int words, int m, int64_t E,
    const int32_t *__restrict__ eu, const int32_t *__restrict__ ev,
    const int32_t *__restrict__ Wt, int64_t *__restrict__ obj) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= count) return;
    const uint64_t *row = spins + s * words;
    int64_t acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t e = 0; e < E; ++e) {
        if (spin_bit(row, eu[e]) != spin_bit(row, ev[e])) {
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (k < m) acc[k] += (int64_t)Wt[(int64_t)k * E + e];
        }
    }
    for (int k = 0; k < m; ++k) obj[s * m + k] = acc[k];
}

__global__ __launch_bounds__(kBlock) void eval_block_kernel(
    const uint64_t *__restrict__ spins, int64_t count, int words, int m, int64_t E,
    const int32_t *__restrict__ eu, const int32_t *__restrict__ ev,
    const int32_t *__restrict__ Wt, int64_t *__restrict__ obj) {
    __shared__ int64_t red[8][kBlock / 64];
    const int64_t s = blockIdx.x;
    const uint64_t *row = spins + s * words;
    int64_t acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t e = threadIdx.x; e < E; e += kBlock) {
        if (spin_bit(row, eu[e]) != spin_bit(row, ev[e])) {
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (k < m) acc[k] += (int64_t)Wt[(int64_t)k * E + e];
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        int64_t v = acc[k];
        for (int off = 32; off > 0; off >>= 1) {
            int lo = __shfl_xor((int)(uint32_t)v, off);
            int hi = __shfl_xor((int)(v >> 32), off);
            v += (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
        }
        if (lane == 0) red[k][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < m) {
        int64_t v = 0;
        for (int i = 0; i < kBlock / 64; ++i) v += red[threadIdx.x][i];
        obj[s * m + threadIdx.x] = v;
    }
}

// Enumeration: thread r evaluates the configuration with spin word first + r.
// The edge list and weights are read at wave-uniform addresses.
__global__ __launch_bounds__(kBlock) void enumerate_kernel(uint64_t first, int64_t count, int m, int64_t E,
                                                           const int32_t *__restrict__ eu,
                                                           const int32_t *__restrict__ ev,
                                                           const int32_t *__restrict__ Wt,
                                                           int64_t *__restrict__ obj) {
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r >= count) return;
    const uint64_t code = first + (uint64_t)r;
    int64_t acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t e = 0; e < E; ++e) {
        const int64_t mask = -(int64_t)(((code >> eu[e]) ^ (code >> ev[e])) & 1ull);
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (k < m) acc[k] += (int64_t)Wt[(int64_t)k * E + e] & mask;
    }
    for (int k = 0; k < m; ++k) obj[r * m + k] = acc[k];
}

void launch_enumerate(const Problem &p, uint64_t first, int64_t count, int64_t *obj, hipStream_t st) {
    if (count == 0) return;
    QAIA_CHECK(p.m <= 8, QAIA_UNSUPPORTED, "enumeration supports at most 8 objectives");
    const int64_t blocks = (count + kBlock - 1) / kBlock;
    QAIA_CHECK(blocks <= INT32_MAX, QAIA_INVALID_ARGUMENT, "too many configurations for one call");
    hipLaunchKernelGGL(enumerate_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, st, first, count, p.m, p.E,
                       p.d_eu, p.d_ev, p.d_W, obj);
    QAIA_HIP(hipGetLastError());
}

constexpr uint64_t kRandomSpinKey = 0x6a09e667f3bcc909ull;

__global__ __launch_bounds__(kBlock) void random_spins_kernel(int n, int words, int64_t total, uint64_t seed,
                                                              uint64_t offset, uint64_t *__restrict__ spins) {
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;  // (row, word) flattened
    if (idx >= total) return;
    const int64_t row = idx / words;
    const int wd = (int)(idx % words);
    uint64_t b = splitmix64(seed ^ kRandomSpinKey, ((uint64_t)row + offset) * (uint64_t)words + (uint64_t)wd);
    const int valid = n - wd * 64;
    if (valid < 64) b &= (1ull << valid) - 1ull;
    spins[idx] = b;
}

void launch_random_spins(int n, int64_t count, uint64_t seed, uint64_t offset, uint64_t *spins, hipStream_t st) {
    const int words = (n + 63) / 64;
    const int64_t total = count * words;
    if (total == 0) return;
    const int64_t blocks = (total + kBlock - 1) / kBlock;
    QAIA_CHECK(blocks <= INT32_MAX, QAIA_INVALID_ARGUMENT, "too many rows for one call");
    hipLaunchKernelGGL(random_spins_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, st, n, words, total, seed,
                       offset, spins);
    QAIA_HIP(hipGetLastError());
}

// Uniform weight vectors on the simplex: Dirichlet(1, ..., 1) as m i.i.d.
// Exp(1) draws -log(u), u in (0, 1] from 24 bits of the counter stream keyed
// seed ^ 0xbb67ae8584caa73b (draw (row + offset) * m + k), divided by their sum.
constexpr uint64_t kDirichletKey = 0xbb67ae8584caa73bull;

__global__ __launch_bounds__(kBlock) void dirichlet_kernel(int m, int64_t count, uint64_t seed, uint64_t offset,
                                                           float *__restrict__ out) {
    const int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (row >= count) return;
    float e[8];
    float sum = 0.0f;
    for (int k = 0; k < m; ++k) {
        const uint64_t b = splitmix64(seed ^ kDirichletKey, ((uint64_t)row + offset) * (uint64_t)m + (uint64_t)k);
        const float u = (float)((uint32_t)(b >> 40) + 1u) * 0x1p-24f;
        e[k] = -logf(u);
        sum += e[k];
    }
    const float inv = 1.0f / sum;
    for (int k = 0; k < m; ++k) out[row * m + k] = e[k] * inv;
}

void launch_dirichlet(int m, int64_t count, uint64_t seed, uint64_t offset, float *out, hipStream_t st) {
    if (count == 0) return;
    const int64_t blocks = (count + kBlock - 1) / kBlock;
    QAIA_CHECK(blocks <= INT32_MAX, QAIA_INVALID_ARGUMENT, "too many rows for one call");
    hipLaunchKernelGGL(dirichlet_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, st, m, count, seed, offset, out);
    QAIA_HIP(hipGetLastError());
}

// Replica-tiled evaluation for large edge sets: a block stages the spins of 64
// replicas in LDS (32-bit words, row pitch 2*words + 1 so the 64 lanes, one
// replica each, read distinct banks) and its four waves walk four contiguous
// parts of the block's edge range with the edge data at wave-uniform
// addresses.  Partial sums are combined over the waves in LDS and added to the
// zeroed output with 64-bit integer atomics (exact, order independent).
constexpr int kEvalTile = 64;

__global__ __launch_bounds__(kBlock) void eval_zero_kernel(int64_t *__restrict__ obj, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) obj[i] = 0;
}

__global__ __launch_bounds__(kBlock) void eval_tile_kernel(
    const uint64_t *__restrict__ spins, int64_t count, int words, int m, int64_t E,
    const int32_t *__restrict__ eu, const int32_t *__restrict__ ev, const int32_t *__restrict__ Wt,
    int64_t edges_per_block, int64_t *__restrict__ obj) {
    extern __shared__ uint32_t sp[];
    __shared__ int64_t red[kBlock / 64][kEvalTile][8];
    const int pitch = 2 * words + 1;
    const int64_t r0 = (int64_t)blockIdx.x * kEvalTile;
    for (int i = threadIdx.x; i < kEvalTile * 2 * words; i += kBlock) {
        const int r = i / (2 * words), wd = i % (2 * words);
        sp[r * pitch + wd] = r0 + r < count ? ((const uint32_t *)(spins + (r0 + r) * words))[wd] : 0u;
    }
    __syncthreads();
    // the wave index is uniform across the wave; saying so lets the edge loads use scalar loads
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t b0 = (int64_t)blockIdx.y * edges_per_block;
    const int64_t b1 = b0 + edges_per_block < E ? b0 + edges_per_block : E;
    const int64_t part = (b1 - b0 + 3) / 4;
    const int64_t e0 = b0 + wave * part;
    const int64_t e1 = e0 + part < b1 ? e0 + part : b1;
    const uint32_t *my = sp + lane * pitch;
    int64_t acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    // groups of 8 edges, so the uniform edge and weight loads batch into wide scalar loads
    int64_t e = e0;
    for (; e + 8 <= e1; e += 8) {
        int uu[8], vv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            uu[q] = eu[e + q];
            vv[q] = ev[e + q];
        }
        int64_t mask[8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            mask[q] = -(int64_t)(((my[uu[q] >> 5] >> (uu[q] & 31)) ^ (my[vv[q] >> 5] >> (vv[q] & 31))) & 1u);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (k >= m) break;
            const int32_t *wk = Wt + (int64_t)k * E + e;
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[k] += (int64_t)wk[q] & mask[q];
        }
    }
    for (; e < e1; ++e) {
        const int u = eu[e], v = ev[e];
        const uint32_t cut = ((my[u >> 5] >> (u & 31)) ^ (my[v >> 5] >> (v & 31))) & 1u;
        const int64_t mask = -(int64_t)cut;
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (k < m) acc[k] += (int64_t)Wt[(int64_t)k * E + e] & mask;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) red[wave][lane][k] = acc[k];
    __syncthreads();
    if (wave == 0 && r0 + lane < count) {
        for (int k = 0; k < m; ++k) {
            const int64_t v = red[0][lane][k] + red[1][lane][k] + red[2][lane][k] + red[3][lane][k];
            atomicAdd((unsigned long long *)&obj[(r0 + lane) * m + k], (unsigned long long)v);
        }
    }
}

void launch_evaluate(const Problem &p, const uint64_t *spins, int64_t count, int64_t *obj,
                     hipStream_t st) {
    if (count == 0) return;
    QAIA_CHECK(p.m <= 8, QAIA_UNSUPPORTED, "evaluation supports at most 8 objectives");
    const size_t tile_lds = sizeof(uint32_t) * (size_t)kEvalTile * (2 * (size_t)p.words + 1);
    if (p.E <= 4096) {
        int64_t blocks = (count + kBlock - 1) / kBlock;
        QAIA_CHECK(blocks <= INT32_MAX, QAIA_INVALID_ARGUMENT, "too many samples");
        hipLaunchKernelGGL(eval_thread_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, st, spins,
                           count, p.words, p.m, p.E, p.d_eu, p.d_ev, p.d_W, obj);
    } else if (tile_lds <= 48 * 1024) {
        const int64_t tiles = (count + kEvalTile - 1) / kEvalTile;
        QAIA_CHECK(tiles <= INT32_MAX, QAIA_INVALID_ARGUMENT, "too many samples");
        // about 2048 blocks in all, at least 4096 edges per block
        int64_t chunks = std::max<int64_t>(1, 2048 / tiles);
        int64_t epb = std::max<int64_t>(4096, (p.E + chunks - 1) / chunks);
        chunks = (p.E + epb - 1) / epb;
        QAIA_CHECK(chunks <= 65535, QAIA_INVALID_ARGUMENT, "edge set too large");
        const int64_t n = count * p.m;
        hipLaunchKernelGGL(eval_zero_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                           obj, n);
        hipLaunchKernelGGL(eval_tile_kernel, dim3((unsigned)tiles, (unsigned)chunks), dim3(kBlock), tile_lds, st,
                           spins, count, p.words, p.m, p.E, p.d_eu, p.d_ev, p.d_W, epb, obj);
    } else {
        QAIA_CHECK(count <= INT32_MAX, QAIA_INVALID_ARGUMENT, "too many samples");
        hipLaunchKernelGGL(eval_block_kernel, dim3((unsigned)count), dim3(kBlock), 0, st, spins,
                           count, p.words, p.m, p.E, p.d_eu, p.d_ev, p.d_W, obj);
    }
    QAIA_HIP(hipGetLastError());
}

}  // namespace qaia
