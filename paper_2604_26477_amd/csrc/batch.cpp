// Batching form: a ragged batch of (problem, weight vectors, replicas) items
// sampled by one graph launch, and the autotuner that picks each item's
// kernel family.
//
// Execution of qaia_sample_batch, captured once into a hipGraph on a private
// stream and launched as one graph:
//   - per item: workspace header reset and weight preparation;
//   - branch A (forked stream): the items on the generic sparse kernel run in
//     one persistent launch per kernel shape: the grid is what the GPU holds
//     at once, and blocks take (item, replica tile) work units from a device
//     queue, items in decreasing cost per unit (each unit's whole T-step loop
//     stays on chip); items on the per-graph generated kernels run their own
//     launches;
//   - branch B: dense items are set up, then each of the T steps is ONE launch
//     of the grouped dense step kernel over the tiles of all dense items, then
//     each dense item is read out and evaluated;
//   - the branches join and the caller's stream waits for the graph.
// The kernel families differ in their tile shape and replicas per wave: one
// replica per lane (64 replicas per wave, generated kernel), one spin per
// lane (floor(256/n) replicas per 256-lane block by default, or the item's
// tile knob: more replicas per block put several spins on each lane, generic
// kernel), or 64- / 128-spin x 128-replica matrix-core tiles (dense kernels).
#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace qaia {

namespace {

// generic-sparse kernel shapes: maximum degree class {4, 8, 16, 32} x spins
// per lane {1, 2, 4, 8, 16}; dense groups: register tiles, staged tiles m = 1..4
constexpr int kSparseClasses = 20;
constexpr int kDenseGroups = 5;

int sparse_class(const SparseShape &sh) {
    const int d = sh.maxdeg <= 4 ? 0 : sh.maxdeg <= 8 ? 1 : sh.maxdeg <= 16 ? 2 : 3;
    int q = 0;
    while ((1 << q) < sh.npt) ++q;
    return d * 5 + q;
}

struct ItemPlan {
    const Problem *p;
    int path;
    WsLayout L;
    size_t base;  // offset of the item's region in the batch workspace
};

int default_path(const Problem &p, const qaia_schedule &s) {
    if (s.precision == QAIA_FP16) return QAIA_PATH_SPARSE_REG;
    if (s.precision != QAIA_FP32) return QAIA_PATH_DENSE_STAGED;
    if (p.jit[s.variant] != nullptr) return QAIA_PATH_SPARSE_REG;
    if (sparse_lds_supported(p, nullptr)) return QAIA_PATH_SPARSE_LDS;
    return QAIA_PATH_DENSE_STAGED;
}

void check_path(const Problem &p, const qaia_schedule &s, int path) {
    std::string why;
    if (path == QAIA_PATH_SPARSE_REG) {
        QAIA_CHECK(p.jit[s.variant] != nullptr, QAIA_UNSUPPORTED, "generated kernel unavailable: " + p.jit_error);
        QAIA_CHECK(s.precision == QAIA_FP32 || s.precision == QAIA_FP16, QAIA_UNSUPPORTED,
                   "generated kernel runs FP32 or binary16");
    } else if (path == QAIA_PATH_SPARSE_LDS) {
        QAIA_CHECK(sparse_lds_supported(p, &why), QAIA_UNSUPPORTED, "sparse LDS path: " + why);
        QAIA_CHECK(s.precision == QAIA_FP32, QAIA_UNSUPPORTED, "the generic sparse kernel runs FP32");
    } else if (is_dense_path(path)) {
        QAIA_CHECK(s.precision != QAIA_FP16, QAIA_UNSUPPORTED, "binary16 runs on the generated sparse kernel only");
        QAIA_CHECK(dense_supported(p, &why), QAIA_UNSUPPORTED, "dense path: " + why);
        QAIA_CHECK(p.m <= 4, QAIA_UNSUPPORTED, "dense path supports m <= 4");
    } else {
        throw Error{QAIA_INVALID_ARGUMENT, "unknown path"};
    }
}

void check_tile(const Problem &p, int path, int tile, int64_t rows) {
    QAIA_CHECK(tile >= 0, QAIA_INVALID_ARGUMENT, "tile must be >= 0");
    if (tile == 0) return;
    QAIA_CHECK(path == QAIA_PATH_SPARSE_LDS, QAIA_INVALID_ARGUMENT,
               "a tile knob applies to the generic sparse kernel only");
    (void)sparse_lds_shape(p, std::max<int64_t>(rows, 1), tile);  // throws past 16 spins per lane
}

struct BatchLayout {
    std::vector<ItemPlan> items;
    size_t jobs_off = 0, queue_off = 0, total = 0;
    int n_sparse = 0, n_dense = 0;
};

BatchLayout batch_layout(const qaia_batch_item *items, int32_t count, const qaia_schedule &s) {
    BatchLayout B;
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
        const qaia_batch_item &it = items[i];
        QAIA_CHECK(it.problem != nullptr, QAIA_INVALID_ARGUMENT, "item " + std::to_string(i) + ": null problem");
        const Problem &p = *reinterpret_cast<const Problem *>(it.problem);
        QAIA_CHECK(it.W >= 0 && it.R >= 1 && it.W <= (int64_t(1) << 40) / it.R, QAIA_INVALID_ARGUMENT,
                   "item " + std::to_string(i) + ": bad W or R");
        QAIA_CHECK(it.W * it.R == 0 || (it.weights && it.spins && it.obj), QAIA_INVALID_ARGUMENT,
                   "item " + std::to_string(i) + ": null buffer");
        const int path = it.path == QAIA_PATH_AUTO ? default_path(p, s) : it.path;
        check_path(p, s, path);
        check_tile(p, path, it.tile, it.W * (int64_t)it.R);
        ItemPlan ip{&p, path, sample_ws_layout(p, it.W, it.R, s, !is_dense_path(path)), off};
        if (is_dense_path(path)) {
            dense_ws_extend(p, it.W, it.R, s, ip.L);
            ++B.n_dense;
        } else if (path == QAIA_PATH_SPARSE_LDS) {
            ++B.n_sparse;
        }
        off += align256(ip.L.total);
        B.items.push_back(ip);
    }
    B.jobs_off = off;
    off += align256(sizeof(SparseJob) * (size_t)std::max(B.n_sparse, 1));
    off += align256(sizeof(DenseJob) * (size_t)std::max(B.n_dense, 1));
    // start tables: one per generic-sparse shape class and one per dense group
    off += (kSparseClasses + kDenseGroups) * align256(sizeof(int64_t) * (size_t)(count + 1));
    // work-queue counters of the persistent sparse launches, one per shape class
    B.queue_off = off;
    off += align256(sizeof(unsigned long long) * kSparseClasses);
    B.total = off;
    return B;
}

// Graphs launched by earlier calls, destroyed once their completion event has fired.
struct PendingGraph {
    hipGraphExec_t exec;
    hipEvent_t done;
};
std::mutex g_pending_mu;
std::vector<PendingGraph> g_pending;

void reap_graphs() {
    std::lock_guard<std::mutex> lk(g_pending_mu);
    std::vector<PendingGraph> keep;
    for (auto &g : g_pending) {
        if (hipEventQuery(g.done) == hipSuccess) {
            (void)hipGraphExecDestroy(g.exec);
            (void)hipEventDestroy(g.done);
        } else {
            keep.push_back(g);
        }
    }
    g_pending.swap(keep);
}

struct Streams {
    hipStream_t a = nullptr, b = nullptr;
};
std::mutex g_streams_mu;
std::vector<Streams> g_streams;  // per device, default priority, created on first use

Streams private_streams(int device) {
    std::lock_guard<std::mutex> lk(g_streams_mu);
    if ((int)g_streams.size() <= device) g_streams.resize(device + 1);
    Streams &s = g_streams[device];
    if (!s.a) {
        QAIA_HIP(hipStreamCreateWithFlags(&s.a, hipStreamNonBlocking));
        QAIA_HIP(hipStreamCreateWithFlags(&s.b, hipStreamNonBlocking));
    }
    return s;
}

}  // namespace

size_t batch_ws_bytes(const qaia_batch_item *items, int32_t count, const qaia_schedule &s) {
    return batch_layout(items, count, s).total;
}

void sample_batch(const qaia_batch_item *items, int32_t count, const qaia_schedule &s, void *ws, size_t ws_bytes,
                  hipStream_t caller) {
    QAIA_CHECK(count >= 0, QAIA_INVALID_ARGUMENT, "count must be >= 0");
    QAIA_CHECK(count == 0 || items != nullptr, QAIA_INVALID_ARGUMENT, "null items");
    if (count == 0) return;
    const BatchLayout B = batch_layout(items, count, s);
    QAIA_CHECK(ws != nullptr, QAIA_INVALID_ARGUMENT, "null workspace");
    QAIA_CHECK(ws_bytes >= B.total, QAIA_WORKSPACE_TOO_SMALL,
               "batch workspace needs " + std::to_string(B.total) + " bytes");
    const int device = B.items[0].p->device;
    for (const ItemPlan &ip : B.items)
        QAIA_CHECK(ip.p->device == device, QAIA_INVALID_ARGUMENT, "all items must live on one device");
    DeviceGuard g(device);
    reap_graphs();
    char *base = (char *)ws;
    const bool dsb = s.variant == QAIA_DSB;

    // descriptors of the batched launches
    // generic-sparse jobs grouped by kernel shape (maximum degree class x spins
    // per lane), so that no item runs with a larger unrolled neighbour loop or
    // more spins per lane than its own graph needs
    struct SparseCand {
        SparseJob job;
        int64_t units;
        double cost;  // work per unit: replicas x spins x maximum degree (the step loop's length is common)
    };
    std::vector<SparseCand> scand[kSparseClasses];
    std::vector<SparseJob> sjobs[kSparseClasses];
    std::vector<int64_t> sstart[kSparseClasses];
    for (auto &v : sstart) v.assign(1, 0);
    size_t shmem[kSparseClasses] = {};
    int smaxdeg[kSparseClasses] = {}, snpt[kSparseClasses] = {};
    // dense jobs grouped by kernel: [0] 64 x 128 register tiles (any m <= 4),
    // [g = 1..4] staged 128 x 128 tiles for m = g, with 8-aligned job starts
    constexpr int kGroups = kDenseGroups;
    std::vector<DenseJob> djobs[kGroups];
    std::vector<int64_t> dstart[kGroups];
    for (auto &v : dstart) v.assign(1, 0);
    auto group_of = [](const ItemPlan &ip) { return ip.path == QAIA_PATH_DENSE_STAGED ? ip.p->m : 0; };
    for (int i = 0; i < count; ++i) {
        const ItemPlan &ip = B.items[i];
        const qaia_batch_item &it = items[i];
        void *iws = base + ip.base;
        if (it.W * it.R == 0) continue;
        if (ip.path == QAIA_PATH_SPARSE_LDS) {
            const SparseShape sh = sparse_lds_shape(*ip.p, it.W * (int64_t)it.R, it.tile);
            const int c = sparse_class(sh);
            scand[c].push_back({sparse_job(*ip.p, it.W, it.R, s, iws, ip.L, it.spins, it.obj, nullptr, 0, it.tile),
                                sh.blocks, (double)sh.rpb * ip.p->n * std::max(ip.p->max_degree, 1)});
            smaxdeg[c] = sh.maxdeg;
            snpt[c] = sh.npt;
            shmem[c] = std::max(shmem[c], sh.shmem);
        } else if (is_dense_path(ip.path)) {
            const int g = group_of(ip);
            DenseJob j = dense_job(*ip.p, it.W, it.R, s, iws, ip.L, nullptr, 0, g != 0);
            djobs[g].push_back(j);
            const int64_t tiles = (int64_t)j.tiles_x * j.tiles_y;
            dstart[g].push_back(dstart[g].back() + (g != 0 ? (tiles + 7) / 8 * 8 : tiles));
        }
    }
    // queue order inside a shape class: decreasing work per unit, so the long
    // units start first and the short ones fill the tail
    for (int c = 0; c < kSparseClasses; ++c) {
        std::stable_sort(scand[c].begin(), scand[c].end(),
                         [](const SparseCand &a, const SparseCand &b) { return a.cost > b.cost; });
        for (const SparseCand &sc : scand[c]) {
            sjobs[c].push_back(sc.job);
            sstart[c].push_back(sstart[c].back() + sc.units);
        }
    }
    unsigned long long *queues = (unsigned long long *)(base + B.queue_off);
    char *jobs = base + B.jobs_off;
    SparseJob *d_sjobs = (SparseJob *)jobs;
    DenseJob *d_djobs = (DenseJob *)(jobs + align256(sizeof(SparseJob) * (size_t)std::max(B.n_sparse, 1)));
    char *starts_base = (char *)d_djobs + align256(sizeof(DenseJob) * (size_t)std::max(B.n_dense, 1));
    const size_t start_bytes = align256(sizeof(int64_t) * (size_t)(count + 1));
    SparseJob *d_sjobs_c[kSparseClasses];
    int64_t *d_sstart_c[kSparseClasses];
    {
        size_t jo = 0;
        for (int c = 0; c < kSparseClasses; ++c) {
            d_sjobs_c[c] = d_sjobs + jo;
            jo += sjobs[c].size();
            d_sstart_c[c] = (int64_t *)(starts_base + c * start_bytes);
        }
    }
    int64_t *d_sstart = (int64_t *)(starts_base + (kSparseClasses - 1) * start_bytes);
    DenseJob *d_djobs_g[kGroups];
    int64_t *d_dstart_g[kGroups];
    {
        size_t jo = 0;
        char *so = (char *)d_sstart + start_bytes;
        for (int g = 0; g < kGroups; ++g) {
            d_djobs_g[g] = d_djobs + jo;
            jo += djobs[g].size();
            d_dstart_g[g] = (int64_t *)so;
            so += align256(sizeof(int64_t) * (size_t)(count + 1));
        }
    }

    Streams ps = private_streams(device);
    hipEvent_t ev_start, ev_fork, ev_join, ev_done;
    QAIA_HIP(hipEventCreateWithFlags(&ev_start, hipEventDisableTiming));
    QAIA_HIP(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
    QAIA_HIP(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
    QAIA_HIP(hipEventCreateWithFlags(&ev_done, hipEventDisableTiming));
    // the private stream follows the caller's prior work; descriptor uploads
    // are ordered there too (outside the graph)
    QAIA_HIP(hipEventRecord(ev_start, caller));
    QAIA_HIP(hipStreamWaitEvent(ps.a, ev_start, 0));
    for (int c = 0; c < kSparseClasses; ++c)
        if (!sjobs[c].empty()) {
            QAIA_HIP(hipMemcpyAsync(d_sjobs_c[c], sjobs[c].data(), sizeof(SparseJob) * sjobs[c].size(),
                                    hipMemcpyHostToDevice, ps.a));
            QAIA_HIP(hipMemcpyAsync(d_sstart_c[c], sstart[c].data(), sizeof(int64_t) * sstart[c].size(),
                                    hipMemcpyHostToDevice, ps.a));
        }
    for (int g = 0; g < kGroups; ++g)
        if (!djobs[g].empty()) {
            QAIA_HIP(hipMemcpyAsync(d_djobs_g[g], djobs[g].data(), sizeof(DenseJob) * djobs[g].size(),
                                    hipMemcpyHostToDevice, ps.a));
            QAIA_HIP(hipMemcpyAsync(d_dstart_g[g], dstart[g].data(), sizeof(int64_t) * dstart[g].size(),
                                    hipMemcpyHostToDevice, ps.a));
        }
    // the host vectors above are released when this call returns
    QAIA_HIP(hipStreamSynchronize(ps.a));

    hipGraph_t graph = nullptr;
    QAIA_HIP(hipStreamBeginCapture(ps.a, hipStreamCaptureModeThreadLocal));
    try {
        for (int i = 0; i < count; ++i) {
            const ItemPlan &ip = B.items[i];
            launch_prep(*ip.p, items[i].weights, items[i].W, s, base + ip.base, ip.L, ps.a);
        }
        QAIA_HIP(hipEventRecord(ev_fork, ps.a));
        QAIA_HIP(hipStreamWaitEvent(ps.b, ev_fork, 0));
        // branch A: sparse items
        for (int c = 0; c < kSparseClasses; ++c)
            if (!sjobs[c].empty())
                launch_sparse_lds_queue(d_sjobs_c[c], (int)sjobs[c].size(), d_sstart_c[c], sstart[c].back(),
                                        smaxdeg[c], snpt[c], shmem[c], dsb, queues + c, ps.b);
        for (int i = 0; i < count; ++i) {
            const ItemPlan &ip = B.items[i];
            const qaia_batch_item &it = items[i];
            if (ip.path == QAIA_PATH_SPARSE_REG && it.W * it.R > 0)
                launch_sparse_reg(*ip.p, s.variant, it.W, it.R, s, base + ip.base, ip.L, it.spins, it.obj, nullptr, 0,
                                  ps.b);
        }
        QAIA_HIP(hipEventRecord(ev_join, ps.b));
        // branch B: dense items
        if (B.n_dense > 0) {
            int di[kGroups] = {0, 0, 0, 0, 0};
            for (int i = 0; i < count; ++i) {
                const ItemPlan &ip = B.items[i];
                const qaia_batch_item &it = items[i];
                if (is_dense_path(ip.path) && it.W * it.R > 0) {
                    const int g = group_of(ip);
                    launch_dense_setup(*ip.p, it.weights, it.R, s, base + ip.base, ip.L, djobs[g][di[g]++], ps.a);
                }
            }
            for (int t = 0; t < s.steps; ++t)
                for (int g = 0; g < kGroups; ++g)
                    if (!djobs[g].empty())
                        launch_dense_batch_step(s.precision, dsb, g != 0, g, d_djobs_g[g], (int)djobs[g].size(),
                                                d_dstart_g[g], dstart[g].back(), t, ps.a);
            QAIA_HIP(hipGetLastError());
            for (int &d : di) d = 0;
            for (int i = 0; i < count; ++i) {
                const ItemPlan &ip = B.items[i];
                const qaia_batch_item &it = items[i];
                if (is_dense_path(ip.path) && it.W * it.R > 0) {
                    const int g = group_of(ip);
                    launch_dense_finish(*ip.p, it.R, s, base + ip.base, ip.L, djobs[g][di[g]++], it.spins, it.obj,
                                        ps.a);
                }
            }
        }
        QAIA_HIP(hipStreamWaitEvent(ps.a, ev_join, 0));
    } catch (...) {
        hipGraph_t dropped = nullptr;
        (void)hipStreamEndCapture(ps.a, &dropped);
        if (dropped) (void)hipGraphDestroy(dropped);
        throw;
    }
    QAIA_HIP(hipStreamEndCapture(ps.a, &graph));
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    QAIA_HIP(e);
    QAIA_HIP(hipGraphLaunch(exec, ps.a));
    QAIA_HIP(hipEventRecord(ev_done, ps.a));
    QAIA_HIP(hipStreamWaitEvent(caller, ev_done, 0));
    for (hipEvent_t ev : {ev_start, ev_fork, ev_join}) (void)hipEventDestroy(ev);
    std::lock_guard<std::mutex> lk(g_pending_mu);
    g_pending.push_back({exec, ev_done});
}

// Times every kernel family available to each item on `probe_steps` steps of
// its real shape (its own outputs and workspace region serve as scratch) and
// writes the fastest into items[i].path; est_seconds[i] scales the probe to
// the schedule's steps.
void autotune(qaia_batch_item *items, int32_t count, const qaia_schedule &s, int32_t probe_steps,
              double *est_seconds, void *ws, size_t ws_bytes, hipStream_t st) {
    QAIA_CHECK(probe_steps >= 1, QAIA_INVALID_ARGUMENT, "probe_steps must be >= 1");
    for (int i = 0; i < count; ++i) {
        items[i].path = QAIA_PATH_AUTO;
        items[i].tile = 0;
    }
    // a layout with every item on its default path bounds nothing: size each
    // probe by its own single-item layout, placed at the workspace start
    qaia_schedule ps = s;
    ps.steps = probe_steps;
    hipEvent_t e0, e1;
    QAIA_HIP(hipEventCreate(&e0));
    QAIA_HIP(hipEventCreate(&e1));
    for (int i = 0; i < count; ++i) {
        qaia_batch_item &it = items[i];
        QAIA_CHECK(it.problem != nullptr, QAIA_INVALID_ARGUMENT, "null problem");
        const Problem &p = *reinterpret_cast<const Problem *>(it.problem);
        DeviceGuard g(p.device);
        double best = 1e300;
        int best_path = default_path(p, s), best_tile = 0;
        for (int path : {QAIA_PATH_SPARSE_REG, QAIA_PATH_SPARSE_LDS, QAIA_PATH_DENSE, QAIA_PATH_DENSE_STAGED}) {
            try {
                check_path(p, s, path);
            } catch (const Error &) {
                continue;
            }
            WsLayout L = sample_ws_layout(p, it.W, it.R, ps, !is_dense_path(path));
            if (is_dense_path(path)) dense_ws_extend(p, it.W, it.R, ps, L);
            if (L.total > ws_bytes) continue;
            if (it.W * it.R == 0) break;
            // tiles of the family: the generic sparse kernel at 1x, 2x and 4x
            // its default replicas per block (more spins per lane), others one
            std::vector<int> tiles{0};
            if (path == QAIA_PATH_SPARSE_LDS) {
                const int base_rpb = sparse_lds_default_rpb(p);
                for (int k : {2, 4})
                    if ((int64_t)base_rpb * k * p.n <= 16 * 256 && base_rpb * k <= it.W * (int64_t)it.R)
                        tiles.push_back(base_rpb * k);
            }
            for (int tile : tiles) {
                QAIA_HIP(hipEventRecord(e0, st));
                launch_prep(p, it.weights, it.W, ps, ws, L, st);
                if (is_dense_path(path))
                    launch_dense(p, it.weights, it.W, it.R, ps, ws, L, it.spins, it.obj, nullptr, 0,
                                 path == QAIA_PATH_DENSE_STAGED, st);
                else if (path == QAIA_PATH_SPARSE_REG)
                    launch_sparse_reg(p, s.variant, it.W, it.R, ps, ws, L, it.spins, it.obj, nullptr, 0, st);
                else
                    launch_sparse_lds(p, it.W, it.R, ps, ws, L, it.spins, it.obj, nullptr, 0, st, tile);
                QAIA_HIP(hipEventRecord(e1, st));
                QAIA_HIP(hipEventSynchronize(e1));
                float ms = 0.0f;
                QAIA_HIP(hipEventElapsedTime(&ms, e0, e1));
                const double est = ms * 1e-3 * (double)s.steps / (double)probe_steps;
                if (est < best) {
                    best = est;
                    best_path = path;
                    best_tile = tile;
                }
            }
        }
        it.path = best_path;
        it.tile = best_tile;
        if (est_seconds) est_seconds[i] = best < 1e299 ? best : 0.0;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

size_t autotune_ws_bytes(const qaia_batch_item *items, int32_t count, const qaia_schedule &s, int32_t probe_steps) {
    qaia_schedule ps = s;
    ps.steps = probe_steps;
    size_t need = 256;
    for (int i = 0; i < count; ++i) {
        QAIA_CHECK(items[i].problem != nullptr, QAIA_INVALID_ARGUMENT, "null problem");
        const Problem &p = *reinterpret_cast<const Problem *>(items[i].problem);
        for (int path : {QAIA_PATH_SPARSE_REG, QAIA_PATH_SPARSE_LDS, QAIA_PATH_DENSE, QAIA_PATH_DENSE_STAGED}) {
            try {
                check_path(p, s, path);
            } catch (const Error &) {
                continue;
            }
            WsLayout L = sample_ws_layout(p, items[i].W, items[i].R, ps, !is_dense_path(path));
            if (is_dense_path(path)) dense_ws_extend(p, items[i].W, items[i].R, ps, L);
            need = std::max(need, L.total);
        }
    }
    return need;
}

}  // namespace qaia
