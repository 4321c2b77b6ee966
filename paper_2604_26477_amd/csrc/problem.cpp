// Problem construction (validation, CSR adjacency, row sums, device images)
// and error state.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <utility>

#include "internal.hpp"

namespace qaia {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }
int32_t fail(int32_t status, const std::string &msg) {
    g_last_error = msg;
    return status;
}
const char *last_error_cstr() { return g_last_error.c_str(); }

DeviceGuard::DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
}
DeviceGuard::~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
}

Problem::~Problem() {
    for (auto &k : jit) {
        jit_release(k);
        k = nullptr;
    }
    for (auto &k : jit_trace) {
        jit_release(k);
        k = nullptr;
    }
    for (auto &row : jit_noise)
        for (auto &k : row) {
            jit_release(k);
            k = nullptr;
        }
    for (auto &plane : jit16)
        for (auto &row : plane)
            for (auto &k : row) {
                jit_release(k);
                k = nullptr;
            }
    dense_release(*this);
    DeviceGuard g(device);
    for (void *ptr : {(void *)d_eu, (void *)d_ev, (void *)d_W, (void *)d_rowptr, (void *)d_col,
                      (void *)d_eid, (void *)d_rho})
        if (ptr) (void)hipFree(ptr);
}

template <typename T>
static T *upload(const std::vector<T> &v) {
    T *d = nullptr;
    size_t bytes = sizeof(T) * std::max<size_t>(v.size(), 1);
    hipError_t e = hipMalloc((void **)&d, bytes);
    if (e == hipErrorOutOfMemory) throw Error{QAIA_OUT_OF_MEMORY, "device allocation failed"};
    QAIA_HIP(e);
    if (!v.empty()) QAIA_HIP(hipMemcpy(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
    return d;
}

// Validates the instance and builds every image.  Throws Error.
Problem *build_problem(int32_t n, int32_t m, int64_t E, const int32_t *eu, const int32_t *ev,
                       const int32_t *W, int32_t frac_bits, int32_t device) {
    QAIA_CHECK(n >= 1 && n <= (1 << 20), QAIA_INVALID_ARGUMENT, "n must be in [1, 2^20]");
    QAIA_CHECK(m >= 1 && m <= 8, QAIA_INVALID_ARGUMENT, "m must be in [1, 8]");
    QAIA_CHECK(E >= 0 && E <= (int64_t)n * (n - 1) / 2, QAIA_INVALID_ARGUMENT,
               "num_edges must be in [0, n(n-1)/2]");
    QAIA_CHECK(E == 0 || (eu && ev && W), QAIA_INVALID_ARGUMENT, "null edge or weight array");
    QAIA_CHECK(frac_bits >= 0 && frac_bits <= 30, QAIA_INVALID_ARGUMENT, "frac_bits must be in [0, 30]");
    std::vector<std::pair<int32_t, int32_t>> pairs((size_t)E);
    for (int64_t e = 0; e < E; ++e) {
        QAIA_CHECK(eu[e] >= 0 && eu[e] < ev[e] && ev[e] < n, QAIA_INVALID_ARGUMENT,
                   "edge " + std::to_string(e) + " violates 0 <= u < v < n");
        pairs[(size_t)e] = {eu[e], ev[e]};
    }
    std::sort(pairs.begin(), pairs.end());
    QAIA_CHECK(std::adjacent_find(pairs.begin(), pairs.end()) == pairs.end(),
               QAIA_INVALID_ARGUMENT, "repeated edge");
    QAIA_CHECK(device >= 0, QAIA_INVALID_ARGUMENT, "device must be >= 0");
    int ndev = 0;
    QAIA_HIP(hipGetDeviceCount(&ndev));
    QAIA_CHECK(device < ndev, QAIA_INVALID_ARGUMENT, "no such device");

    Problem *p = new Problem();
    try {
        p->n = n;
        p->m = m;
        p->E = E;
        p->frac_bits = frac_bits;
        p->device = device;
        p->words = (n + 63) / 64;
        p->eu.assign(eu, eu + E);
        p->ev.assign(ev, ev + E);
        p->W.assign(W, W + (size_t)m * E);
        // CSR over both directions, neighbours of each node in increasing order
        std::vector<int32_t> deg(n, 0);
        for (int64_t e = 0; e < E; ++e) {
            ++deg[eu[e]];
            ++deg[ev[e]];
        }
        p->rowptr.assign(n + 1, 0);
        for (int i = 0; i < n; ++i) p->rowptr[i + 1] = p->rowptr[i] + deg[i];
        p->max_degree = n ? *std::max_element(deg.begin(), deg.end()) : 0;
        std::vector<int32_t> fill(p->rowptr.begin(), p->rowptr.end() - 1);
        p->col.assign((size_t)2 * E, 0);
        p->eid.assign((size_t)2 * E, 0);
        for (int64_t e = 0; e < E; ++e) {
            int32_t a = eu[e], b = ev[e];
            p->col[fill[a]] = b;
            p->eid[fill[a]++] = (int32_t)e;
            p->col[fill[b]] = a;
            p->eid[fill[b]++] = (int32_t)e;
        }
        for (int i = 0; i < n; ++i) {
            int32_t lo = p->rowptr[i], hi = p->rowptr[i + 1];
            std::vector<std::pair<int32_t, int32_t>> tmp;
            for (int32_t q = lo; q < hi; ++q) tmp.push_back({p->col[q], p->eid[q]});
            std::sort(tmp.begin(), tmp.end());
            for (int32_t q = lo; q < hi; ++q) {
                p->col[q] = tmp[q - lo].first;
                p->eid[q] = tmp[q - lo].second;
            }
        }
        // exact row sums rho_{k,i} = sum_j W_k,ij and totals T_k
        std::vector<int64_t> rho((size_t)m * n, 0);
        p->total.assign(m, 0);
        for (int k = 0; k < m; ++k)
            for (int64_t e = 0; e < E; ++e) {
                int64_t w = W[(size_t)k * E + e];
                rho[(size_t)k * n + eu[e]] += w;
                rho[(size_t)k * n + ev[e]] += w;
                p->total[k] += w;
            }
        DeviceGuard g(device);
        p->d_eu = upload(p->eu);
        p->d_ev = upload(p->ev);
        p->d_W = upload(p->W);
        p->d_rowptr = upload(p->rowptr);
        p->d_col = upload(p->col);
        p->d_eid = upload(p->eid);
        p->d_rho = upload(rho);
        dense_build(*p);
        jit_prepare(*p);
    } catch (...) {
        delete p;
        throw;
    }
    return p;
}

}  // namespace qaia
