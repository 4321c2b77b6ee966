// Exact hypervolume on the host, Eq. (6) and Appendix A.
//
// Points are translated to extents e = max(y - ref, 0) (clipping leaves the
// union of boxes [ref, y] unchanged).  The volume is accumulated exactly in a
// 256-bit unsigned integer:
//   m = 1: the largest extent;
//   m = 2: the staircase area;
//   m = 3: a sweep in decreasing third coordinate that keeps the
//          two-dimensional non-dominated staircase of the points seen so far
//          in an ordered map and updates its area incrementally on insertion
//          (the dimension-sweep idea of Fonseca, Paquete and Lopez-Ibanez,
//          CEC 2006), O(P log P);
//   m >= 4: the exclusive-volume recursion of the WFG algorithm (While,
//          Bradstreet and Barone, IEEE TEVC 2012): with the points in
//          increasing last coordinate, HV(S) = sum_i p_i,last *
//          (prod_{k<last} p_i,k - HV_{m-1}(limit_i)), where limit_i holds
//          min(q, p_i) over the later points q projected to the first m-1
//          coordinates (their last coordinate is p_i,last for all of them).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <numeric>
#include <thread>
#include <vector>

#include <sched.h>

#include "internal.hpp"

namespace qaia {
namespace {

typedef unsigned __int128 u128;

struct U256 {
    uint64_t w[4] = {0, 0, 0, 0};
};

U256 from128(u128 v) {
    U256 r;
    r.w[0] = (uint64_t)v;
    r.w[1] = (uint64_t)(v >> 64);
    return r;
}

U256 add(const U256 &a, const U256 &b) {
    U256 r;
    u128 c = 0;
    for (int i = 0; i < 4; ++i) {
        u128 s = (u128)a.w[i] + b.w[i] + c;
        r.w[i] = (uint64_t)s;
        c = s >> 64;
    }
    return r;
}

// a - b with a >= b
U256 sub(const U256 &a, const U256 &b) {
    U256 r;
    uint64_t borrow = 0;
    for (int i = 0; i < 4; ++i) {
        uint64_t bi = b.w[i] + borrow;
        uint64_t nb = (bi < borrow) || (a.w[i] < bi) ? 1 : 0;
        r.w[i] = a.w[i] - bi;
        borrow = nb;
    }
    return r;
}

U256 mul64(const U256 &a, uint64_t b) {
    U256 r;
    u128 c = 0;
    for (int i = 0; i < 4; ++i) {
        u128 p = (u128)a.w[i] * b + c;
        r.w[i] = (uint64_t)p;
        c = p >> 64;
    }
    return r;
}

double to_double(const U256 &a) {
    double r = 0.0;
    for (int i = 3; i >= 0; --i) r = r * 18446744073709551616.0 + (double)a.w[i];
    return r;
}

// 2-D staircase area of the points seen so far, updated on insertion.  The
// points are kept in a flat vector sorted by x (ascending); non-dominated, so
// y descends with x.  An insertion removes a contiguous run, so the update is
// a binary search, a short backward scan and one block move (no per-point
// allocation, unlike a tree).
struct Staircase {
    typedef std::pair<uint64_t, uint64_t> Pt;
    std::vector<Pt> pts;
    u128 area = 0;

    // area of the segments of the points in [first, last) given the x of the
    // point left of first (0 if none)
    static u128 seg_sum(const Pt *first, const Pt *last, uint64_t left_x) {
        u128 s = 0;
        for (const Pt *it = first; it != last; ++it) {
            s += (u128)(it->first - left_x) * it->second;
            left_x = it->first;
        }
        return s;
    }

    void insert(uint64_t x, uint64_t y) {
        if (x == 0 || y == 0) return;
        Pt *b = pts.data(), *e = b + pts.size();
        // dominated by (or equal to) a stored point: some stored px >= x with py >= y;
        // among the points with px >= x the first one has the largest y.
        Pt *ge = std::lower_bound(b, e, x, [](const Pt &p, uint64_t v) { return p.first < v; });
        if (ge != e && ge->second >= y) return;
        // every stored point with px >= x now has py < y.  Stored points
        // dominated by (x, y) (px <= x and py <= y) form a contiguous run: the
        // points left of `ge` with py <= y, plus `ge` itself when px == x.
        Pt *right = ge;  // first surviving point to the right of x
        if (right != e && right->first == x) ++right;
        Pt *first = ge;
        while (first != b && (first - 1)->second <= y) --first;
        const uint64_t left_x = first == b ? 0 : (first - 1)->first;
        // segments whose area changes: the removed run and the right neighbour
        const Pt *stop = right == e ? right : right + 1;
        const u128 before = seg_sum(first, stop, left_x);
        u128 after = (u128)(x - left_x) * y;
        if (right != e) after += (u128)(right->first - x) * right->second;
        area = area - before + after;
        const size_t fi = (size_t)(first - b), ri = (size_t)(right - b);
        if (fi == ri) {
            pts.insert(pts.begin() + fi, Pt(x, y));
        } else {
            pts[fi] = Pt(x, y);
            pts.erase(pts.begin() + fi + 1, pts.begin() + ri);
        }
    }
};

U256 hv2(std::vector<const uint64_t *> &P, int kx, int ky) {
    std::sort(P.begin(), P.end(), [ky](const uint64_t *a, const uint64_t *b) { return a[ky] > b[ky]; });
    U256 vol;
    uint64_t best = 0;
    for (size_t i = 0; i < P.size(); ++i) {
        best = std::max(best, P[i][kx]);
        uint64_t next = i + 1 < P.size() ? P[i + 1][ky] : 0;
        uint64_t h = P[i][ky] - next;
        if (h) vol = add(vol, from128((u128)best * h));
    }
    return vol;
}

// 3-D sweep over coordinates (0, 1, 2); dominated points are harmless.
U256 hv3(std::vector<const uint64_t *> &P) {
    std::sort(P.begin(), P.end(), [](const uint64_t *a, const uint64_t *b) { return a[2] > b[2]; });
    Staircase st;
    U256 vol;
    for (size_t i = 0; i < P.size(); ++i) {
        st.insert(P[i][0], P[i][1]);
        uint64_t next = i + 1 < P.size() ? P[i + 1][2] : 0;
        uint64_t h = P[i][2] - next;
        if (h && st.area) {
            U256 a = from128(st.area);
            vol = add(vol, mul64(a, h));
        }
    }
    return vol;
}

// Non-dominated subset in the first d coordinates (dominated and repeated
// points removed), used to keep the WFG limit sets small.  In descending
// order of the coordinate sum, a point is dropped iff some earlier point is
// >= it in every coordinate (a dominator has a larger sum; of equal points
// the first is kept); with `threads` > 1 the points are checked in parallel.
void nondominated(std::vector<uint64_t> &buf, int stride, int d, size_t &count, int threads = 1) {
    std::vector<size_t> order(count);
    for (size_t i = 0; i < count; ++i) order[i] = i;
    auto sum = [&](size_t i) {
        long double s = 0;
        for (int k = 0; k < d; ++k) s += (long double)buf[i * stride + k];
        return s;
    };
    std::vector<long double> key(count);
    for (size_t i = 0; i < count; ++i) key[i] = sum(i);
    std::sort(order.begin(), order.end(), [&](size_t a, size_t b) { return key[a] != key[b] ? key[a] > key[b] : a < b; });
    std::vector<char> keep(count, 0);
    auto check = [&](size_t oi) {
        const uint64_t *q = &buf[order[oi] * stride];
        for (int k = 0; k < d; ++k)
            if (q[k] == 0) return;  // zero extent: no volume
        for (size_t oj = 0; oj < oi; ++oj) {
            const uint64_t *p = &buf[order[oj] * stride];
            bool ge = true;
            for (int k = 0; k < d && ge; ++k) ge = p[k] >= q[k];
            if (ge) return;
        }
        keep[oi] = 1;
    };
    const int nt = (int)std::max<size_t>(1, std::min<size_t>((size_t)threads, count / 256));
    if (nt == 1) {
        for (size_t oi = 0; oi < count; ++oi) check(oi);
    } else {
        std::vector<std::thread> pool;
        for (int t = 0; t < nt; ++t)
            pool.emplace_back([&, t]() {
                for (size_t oi = (size_t)t; oi < count; oi += (size_t)nt) check(oi);
            });
        for (auto &th : pool) th.join();
    }
    size_t kept = 0;
    for (size_t oi = 0; oi < count; ++oi) kept += keep[oi];
    std::vector<uint64_t> out(kept * stride);
    size_t w = 0;
    for (size_t oi = 0; oi < count; ++oi)
        if (keep[oi]) std::memcpy(&out[(w++) * stride], &buf[order[oi] * stride], sizeof(uint64_t) * stride);
    buf.swap(out);
    count = kept;
}

U256 wfg(std::vector<uint64_t> buf, int stride, int d, size_t count, int threads);

// Exclusive volume of the point at order[oi] with respect to the points after
// it (all of which have a last coordinate >= its own).
U256 exclusive(const std::vector<uint64_t> &buf, const std::vector<size_t> &order, size_t oi,
               int stride, int d, std::vector<uint64_t> &lim) {
    const int last = d - 1;
    const size_t count = order.size();
    const uint64_t *p = &buf[order[oi] * stride];
    if (p[last] == 0) return U256();
    U256 box;
    box.w[0] = 1;
    for (int k = 0; k < last; ++k) box = mul64(box, p[k]);
    size_t L = count - oi - 1;
    lim.assign(L * stride, 0);
    for (size_t j = 0; j < L; ++j) {
        const uint64_t *q = &buf[order[oi + 1 + j] * stride];
        for (int k = 0; k < last; ++k) lim[j * stride + k] = std::min(p[k], q[k]);
    }
    // the 3-D sweep tolerates dominated points; deeper recursion filters first
    if (last > 3) nondominated(lim, stride, last, L);
    U256 covered = wfg(lim, stride, last, L, 1);
    return mul64(sub(box, covered), p[last]);
}

// HV of `count` points (rows of `buf` with `stride`) in the first d >= 3
// coordinates; the top level splits its exclusive volumes over threads.
U256 wfg(std::vector<uint64_t> buf, int stride, int d, size_t count, int threads) {
    if (count == 0) return U256();
    if (d == 3) {
        std::vector<const uint64_t *> P(count);
        for (size_t i = 0; i < count; ++i) P[i] = &buf[i * stride];
        return hv3(P);
    }
    const int last = d - 1;
    std::vector<size_t> order(count);
    for (size_t i = 0; i < count; ++i) order[i] = i;
    std::sort(order.begin(), order.end(),
              [&](size_t a, size_t b) { return buf[a * stride + last] < buf[b * stride + last]; });
    const int nt = (int)std::max<size_t>(1, std::min<size_t>((size_t)threads, count / 64));
    std::vector<U256> part(nt);
    auto work = [&](int t) {
        std::vector<uint64_t> lim;
        // interleaved assignment balances the decreasing cost along the order
        for (size_t oi = (size_t)t; oi < count; oi += (size_t)nt)
            part[t] = add(part[t], exclusive(buf, order, oi, stride, d, lim));
    };
    if (nt == 1) {
        work(0);
    } else {
        std::vector<std::thread> pool;
        for (int t = 0; t < nt; ++t) pool.emplace_back(work, t);
        for (auto &th : pool) th.join();
    }
    U256 total;
    for (const U256 &v : part) total = add(total, v);
    return total;
}

// m = 4: the top level of the recursion above with two exact shortcuts.
// (1) Clipping by min(q, p) keeps the order of the third coordinate, so one
// descending sort of all points serves every limit set's sweep (filtered to
// the points after p in the order of the fourth coordinate).  (2) Once the
// staircase covers p's whole (x, y) face, every lower slab is full, and the
// sweep stops.
U256 hv4(const std::vector<uint64_t> &buf, size_t count, int threads) {
    std::vector<size_t> order(count), zdesc(count), rank(count);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](size_t a, size_t b) {
        return buf[a * 4 + 3] != buf[b * 4 + 3] ? buf[a * 4 + 3] < buf[b * 4 + 3] : a < b;
    });
    for (size_t r = 0; r < count; ++r) rank[order[r]] = r;
    std::iota(zdesc.begin(), zdesc.end(), 0);
    std::sort(zdesc.begin(), zdesc.end(), [&](size_t a, size_t b) {
        return buf[a * 4 + 2] != buf[b * 4 + 2] ? buf[a * 4 + 2] > buf[b * 4 + 2] : a < b;
    });
    const int nt = (int)std::max<size_t>(1, std::min<size_t>((size_t)threads, count / 64));
    std::vector<U256> part(nt);
    auto work = [&](int t) {
        // interleaved assignment balances the decreasing cost along the order
        for (size_t r = (size_t)t; r < count; r += (size_t)nt) {
            const uint64_t *p = &buf[order[r] * 4];
            if (p[3] == 0) continue;
            U256 box;
            box.w[0] = 1;
            for (int k = 0; k < 3; ++k) box = mul64(box, p[k]);
            const u128 full = (u128)p[0] * p[1];
            Staircase st;
            U256 cov;
            uint64_t prev = p[2];
            bool filled = false;
            for (size_t j : zdesc) {
                if (rank[j] <= r) continue;
                const uint64_t *q = &buf[j * 4];
                const uint64_t z = std::min(q[2], p[2]);
                if (prev > z && st.area) cov = add(cov, mul64(from128(st.area), prev - z));
                prev = z;
                st.insert(std::min(q[0], p[0]), std::min(q[1], p[1]));
                if (st.area == full) {
                    if (prev) cov = add(cov, mul64(from128(full), prev));
                    filled = true;
                    break;
                }
            }
            if (!filled && st.area && prev) cov = add(cov, mul64(from128(st.area), prev));
            part[t] = add(part[t], mul64(sub(box, cov), p[3]));
        }
    };
    if (nt == 1) {
        work(0);
    } else {
        std::vector<std::thread> pool;
        for (int t = 0; t < nt; ++t) pool.emplace_back(work, t);
        for (auto &th : pool) th.join();
    }
    U256 total;
    for (const U256 &v : part) total = add(total, v);
    return total;
}

// Host threads: the CPUs this process may run on (the affinity mask), or
// QAIA_HV_THREADS.
int hv_threads() {
    int n = (int)std::thread::hardware_concurrency();
    cpu_set_t set;
    CPU_ZERO(&set);
    if (sched_getaffinity(0, sizeof(set), &set) == 0 && CPU_COUNT(&set) > 0) n = CPU_COUNT(&set);
    if (const char *e = std::getenv("QAIA_HV_THREADS")) n = std::atoi(e);
    return std::max(1, n);
}

}  // namespace

int32_t hypervolume_exact(const int64_t *pts, int64_t P, int32_t m, const int64_t *ref,
                          uint64_t hv[4], double *approx) {
    for (int i = 0; i < 4; ++i) hv[i] = 0;
    if (approx) *approx = 0.0;
    if (P == 0) return QAIA_OK;
    std::vector<uint64_t> ext((size_t)P * m);
    int bits_total = 0;
    for (int k = 0; k < m; ++k) {
        uint64_t mx = 0;
        for (int64_t i = 0; i < P; ++i) {
            __int128 d = (__int128)pts[i * m + k] - (__int128)ref[k];
            uint64_t v = d > 0 ? (uint64_t)d : 0;
            ext[(size_t)i * m + k] = v;
            mx = std::max(mx, v);
        }
        int b = 0;
        while (b < 64 && (mx >> b) != 0) ++b;
        bits_total += b;
    }
    if (bits_total > 256) return fail(QAIA_OVERFLOW, "hypervolume range exceeds 2^256");
    U256 v;
    if (m == 1) {
        uint64_t mx = 0;
        for (int64_t i = 0; i < P; ++i) mx = std::max(mx, ext[i]);
        v.w[0] = mx;
    } else if (m == 2) {
        std::vector<const uint64_t *> Pp(P);
        for (int64_t i = 0; i < P; ++i) Pp[i] = &ext[(size_t)i * 2];
        v = hv2(Pp, 0, 1);
    } else {
        size_t count = (size_t)P;
        const int threads = hv_threads();
        nondominated(ext, m, m, count, threads);
        v = m == 4 ? hv4(ext, count, threads) : wfg(ext, m, m, count, threads);
    }
    for (int i = 0; i < 4; ++i) hv[i] = v.w[i];
    if (approx) *approx = to_double(v);
    return QAIA_OK;
}

}  // namespace qaia
