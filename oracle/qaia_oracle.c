/*
 * CPU oracle for simulated-bifurcation sampling of multi-objective MaxCut.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, obviously-correct
 * statement of what the GPU library computes.  Only the test-suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it; the library never
 * does, and the two share no code (not even headers: the types below are
 * declared here and nowhere else).
 *
 * Paper: "Multi-Objective Optimization by Quantum-Annealing-Inspired
 * Algorithms" (arXiv 2604.26477).  Each function cites the passage it
 * follows.  Floating point is float64 throughout the dynamics; cut values,
 * filtering and hypervolume are exact integers.
 *
 * Readings of the paper that are not spelled out there (all restated in the
 * project's design notes):
 *   - coupling sign: the Ising energy H = sum_E J s_i s_j is *minimised*
 *     (Eq. 2, Eq. 7), so the SB force that descends it is -c0 * J(c) phi(x);
 *   - integration: symplectic Euler, y first (from the pre-step x and the
 *     pre-step field), then x from the new y, then the inelastic wall;
 *   - a(t) = a0 * t / (T - 1) for t = 0..T-1 (a = 0 when T = 1);
 *   - wall: strictly |x| > 1 sets x = sgn(x) and y = 0;
 *   - sgn(0) = +1 for both the dSB force and the read-out;
 *   - c0 = 1 / max_i |sum_j J(c)_ij|; if that maximum is 0, use
 *     1 / max_i sum_j |J(c)_ij|; if that is 0 too, c0 = 0;
 *   - initial x, y ~ U(-amp, amp) from a counter-based SplitMix64 stream.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers.                                             */
/* SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number   */
/* generators", OOPSLA 2014): state advances by the golden-ratio gamma and   */
/* each output is the state passed through the variant-13 finaliser.  The    */
/* value for counter idx is the (idx+1)-th output of the stream whose state  */
/* starts at seed.                                                           */
/* ------------------------------------------------------------------------ */
static uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

uint64_t orc_splitmix64(uint64_t seed, uint64_t idx)
{
    return orc_mix64(seed + (idx + 1ULL) * 0x9e3779b97f4a7c15ULL);
}

/* x0 / y0 draw: 24-bit uniform u on [0,1), v = 2u - 1 (exact in float32),
 * value = float32(amp * v) -- the float64 product of two float32 numbers is
 * exact, so the single rounding to float32 equals a float32 multiply. */
float orc_init_value(uint64_t seed, uint64_t idx, float amp)
{
    uint64_t bits = orc_splitmix64(seed, idx);
    double u = (double)(bits >> 40) * 0x1p-24;
    float v = (float)(2.0 * u - 1.0);
    return (float)((double)amp * (double)v);
}

/* Counter of the initial draw for spin i of global replica g (x: comp = 0,
 * y: comp = 1). */
static uint64_t orc_init_counter(uint64_t g, int n, int i, int comp)
{
    return ((g * (uint64_t)n + (uint64_t)i) << 1) | (uint64_t)comp;
}

/* Standard normal for the noise-injected variant (Eq. 10): Box-Muller on two
 * 24-bit uniforms from one SplitMix64 draw of a separate stream. */
#define ORC_NOISE_KEY 0xd1b54a32d192ed03ULL
double orc_noise_value(uint64_t seed, uint64_t idx)
{
    uint64_t bits = orc_splitmix64(seed ^ ORC_NOISE_KEY, idx);
    double u1 = (double)((bits >> 40) + 1ULL) * 0x1p-24; /* (0, 1] */
    double u2 = (double)(bits & 0xffffffULL) * 0x1p-24;  /* [0, 1) */
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
}

/* ------------------------------------------------------------------------ */
/* Cut values, Eq. (1): C_k(s) = sum over edges (i,j) with s_i != s_j of     */
/* J^(k)_ij.  Exact int64 in the fixed-point units of the weights.           */
/* spins: int8 [count][n] with entries +1 / -1.  weights: int32 [m][E].      */
/* ------------------------------------------------------------------------ */
void orc_cut_values(int n, int m, int64_t num_edges, const int32_t *eu, const int32_t *ev,
                    const int32_t *weights, int64_t count, const int8_t *spins, int64_t *obj)
{
    for (int64_t s = 0; s < count; ++s) {
        const int8_t *sv = spins + s * (int64_t)n;
        for (int k = 0; k < m; ++k) {
            int64_t c = 0;
            for (int64_t e = 0; e < num_edges; ++e)
                if (sv[eu[e]] != sv[ev[e]])
                    c += (int64_t)weights[(int64_t)k * num_edges + e];
            obj[s * m + k] = c;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Scalarised coupling (Eq. 7) and the coupling scale c0 (section            */
/* "Simulated Bifurcation with Gaussian noise").                             */
/* jc[e] = sum_k c_k J^(k)_e in float64, J in real units (W * 2^-frac).      */
/* ------------------------------------------------------------------------ */
static void orc_scalarise(int n, int m, int64_t num_edges, const int32_t *eu, const int32_t *ev,
                          const int32_t *weights, double scale, const float *c, double *jc,
                          double *c0_out)
{
    for (int64_t e = 0; e < num_edges; ++e) {
        double s = 0.0;
        for (int k = 0; k < m; ++k)
            s += (double)c[k] * ((double)weights[(int64_t)k * num_edges + e] * scale);
        jc[e] = s;
    }
    double *row = (double *)calloc((size_t)n, sizeof(double));
    double *rowabs = (double *)calloc((size_t)n, sizeof(double));
    for (int64_t e = 0; e < num_edges; ++e) {
        row[eu[e]] += jc[e];
        row[ev[e]] += jc[e];
        rowabs[eu[e]] += fabs(jc[e]);
        rowabs[ev[e]] += fabs(jc[e]);
    }
    double mx = 0.0, mxa = 0.0;
    for (int i = 0; i < n; ++i) {
        if (fabs(row[i]) > mx) mx = fabs(row[i]);
        if (rowabs[i] > mxa) mxa = rowabs[i];
    }
    *c0_out = mx > 0.0 ? 1.0 / mx : (mxa > 0.0 ? 1.0 / mxa : 0.0);
    free(row);
    free(rowabs);
}

double orc_c0(int n, int m, int64_t num_edges, const int32_t *eu, const int32_t *ev,
              const int32_t *weights, double scale, const float *c)
{
    double *jc = (double *)malloc(sizeof(double) * (size_t)(num_edges > 0 ? num_edges : 1));
    double c0;
    orc_scalarise(n, m, num_edges, eu, ev, weights, scale, c, jc, &c0);
    free(jc);
    return c0;
}

/* ------------------------------------------------------------------------ */
/* Simulated bifurcation, Eq. (9) (and Eq. (10) when alpha > 0):             */
/*   dx/dt = a0 y,                                                           */
/*   dy/dt = -(a0 - a(t)) x - c0 J(c) phi(x) + alpha eta,                    */
/* phi = identity (ballistic, variant 0) or sgn (discrete, variant 1), then  */
/* the inelastic wall and the read-out s = sgn(x).                           */
/*                                                                           */
/* One trajectory per (weight vector w, replica r); its global replica id is */
/* g = w * R + r + replica_offset.  spins: int8 [nw*R][n] (+1/-1).           */
/* x_trace (optional): float64 [nw*R][trace_steps][n], x after each step.    */
/* ------------------------------------------------------------------------ */
int orc_sb_sample(int n, int m, int64_t num_edges, const int32_t *eu, const int32_t *ev,
                  const int32_t *weights, int frac_bits, const float *cvec, int64_t nw, int32_t R,
                  int variant, int32_t T, float dt, float a0, float amp, double alpha,
                  uint64_t seed, uint64_t replica_offset, int8_t *spins, double *x_trace,
                  int32_t trace_steps, int nthreads)
{
    if (n < 1 || m < 1 || num_edges < 0 || nw < 0 || R < 1 || T < 1 || (variant != 0 && variant != 1))
        return 1;
    const double scale = ldexp(1.0, -frac_bits);
    const int64_t total = nw * (int64_t)R;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        double *jc = (double *)malloc(sizeof(double) * (size_t)(num_edges > 0 ? num_edges : 1));
        double *x = (double *)malloc(sizeof(double) * (size_t)n);
        double *y = (double *)malloc(sizeof(double) * (size_t)n);
        double *f = (double *)malloc(sizeof(double) * (size_t)n);
        double *phi = (double *)malloc(sizeof(double) * (size_t)n);
        int64_t cur_w = -1;
        double c0 = 0.0;
#pragma omp for schedule(dynamic, 16)
        for (int64_t row = 0; row < total; ++row) {
            int64_t w = row / R;
            if (w != cur_w) {
                orc_scalarise(n, m, num_edges, eu, ev, weights, scale, cvec + w * m, jc, &c0);
                cur_w = w;
            }
            uint64_t g = (uint64_t)row + replica_offset;
            for (int i = 0; i < n; ++i) {
                x[i] = (double)orc_init_value(seed, orc_init_counter(g, n, i, 0), amp);
                y[i] = (double)orc_init_value(seed, orc_init_counter(g, n, i, 1), amp);
            }
            for (int32_t t = 0; t < T; ++t) {
                double at = T > 1 ? (double)a0 * (double)t / (double)(T - 1) : 0.0;
                for (int i = 0; i < n; ++i) {
                    phi[i] = variant == 0 ? x[i] : (x[i] >= 0.0 ? 1.0 : -1.0);
                    f[i] = 0.0;
                }
                /* f_i = sum_j J(c)_ij phi(x_j), J symmetric over the edge list */
                for (int64_t e = 0; e < num_edges; ++e) {
                    f[eu[e]] += jc[e] * phi[ev[e]];
                    f[ev[e]] += jc[e] * phi[eu[e]];
                }
                for (int i = 0; i < n; ++i) {
                    double force = -((double)a0 - at) * x[i] - c0 * f[i];
                    if (alpha != 0.0) {
                        uint64_t nidx = ((g * (uint64_t)T + (uint64_t)t) * (uint64_t)n) + (uint64_t)i;
                        force += alpha * orc_noise_value(seed, nidx);
                    }
                    y[i] += (double)dt * force;
                }
                for (int i = 0; i < n; ++i) {
                    x[i] += (double)dt * (double)a0 * y[i];
                    if (fabs(x[i]) > 1.0) {
                        x[i] = x[i] > 0.0 ? 1.0 : -1.0;
                        y[i] = 0.0;
                    }
                }
                if (x_trace && t < trace_steps)
                    memcpy(x_trace + (row * (int64_t)trace_steps + t) * n, x, sizeof(double) * (size_t)n);
            }
            for (int i = 0; i < n; ++i)
                spins[row * n + i] = x[i] >= 0.0 ? 1 : -1;
        }
        free(jc);
        free(x);
        free(y);
        free(f);
        free(phi);
    }
    return 0;
}

/* Force on every spin for given soft-spin values (the field the SB update
 * consumes, Eq. 9): out[r][i] = sum_j J^(k)_ij phi_r(x_j) per objective k,
 * in weight units.  phi: float64 [count][n]; out: float64 [count][m][n].
 * Used to state the field error of reduced-precision products. */
void orc_objective_fields(int n, int m, int64_t num_edges, const int32_t *eu, const int32_t *ev,
                          const int32_t *weights, int64_t count, const double *phi, double *out)
{
    for (int64_t r = 0; r < count; ++r) {
        const double *p = phi + r * n;
        double *o = out + r * (int64_t)m * n;
        memset(o, 0, sizeof(double) * (size_t)m * (size_t)n);
        for (int k = 0; k < m; ++k)
            for (int64_t e = 0; e < num_edges; ++e) {
                double w = (double)weights[(int64_t)k * num_edges + e];
                o[(int64_t)k * n + eu[e]] += w * p[ev[e]];
                o[(int64_t)k * n + ev[e]] += w * p[eu[e]];
            }
    }
}

/* ------------------------------------------------------------------------ */
/* Pareto filtering, section "Pareto filtering" with the dominance of Eq.(4) */
/* written in cut (maximisation) space: y' dominates y iff y'_k >= y_k for   */
/* every k and y' != y.  Duplicate objective vectors are merged and the      */
/* smallest sample index represents each one.  Returns the number kept;     */
/* keep_idx receives the representatives in ascending order.                 */
/* ------------------------------------------------------------------------ */
static const int64_t *orc_sort_obj;
static int orc_sort_m;

static int orc_cmp_rows(const void *a, const void *b)
{
    int64_t ia = *(const int64_t *)a, ib = *(const int64_t *)b;
    const int64_t *ra = orc_sort_obj + ia * orc_sort_m, *rb = orc_sort_obj + ib * orc_sort_m;
    for (int k = 0; k < orc_sort_m; ++k) {
        if (ra[k] < rb[k]) return -1;
        if (ra[k] > rb[k]) return 1;
    }
    return ia < ib ? -1 : (ia > ib ? 1 : 0);
}

static int orc_cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

int64_t orc_pareto_filter(const int64_t *obj, int64_t M, int m, int64_t *keep_idx)
{
    if (M <= 0) return 0;
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)M);
    for (int64_t i = 0; i < M; ++i) order[i] = i;
    orc_sort_obj = obj;
    orc_sort_m = m;
    qsort(order, (size_t)M, sizeof(int64_t), orc_cmp_rows);
    /* unique vectors: first of each run of equal rows has the smallest index */
    int64_t *uniq = (int64_t *)malloc(sizeof(int64_t) * (size_t)M);
    int64_t U = 0;
    for (int64_t i = 0; i < M; ++i) {
        if (i == 0 || memcmp(obj + order[i] * m, obj + order[i - 1] * m, sizeof(int64_t) * (size_t)m) != 0)
            uniq[U++] = order[i];
    }
    int64_t P = 0;
    for (int64_t a = 0; a < U; ++a) {
        const int64_t *ya = obj + uniq[a] * m;
        int dominated = 0;
        for (int64_t b = 0; b < U && !dominated; ++b) {
            if (b == a) continue;
            const int64_t *yb = obj + uniq[b] * m;
            int ge = 1;
            for (int k = 0; k < m; ++k)
                if (yb[k] < ya[k]) { ge = 0; break; }
            dominated = ge; /* distinct unique rows: >= everywhere means dominates */
        }
        if (!dominated) keep_idx[P++] = uniq[a];
    }
    qsort(keep_idx, (size_t)P, sizeof(int64_t), orc_cmp_i64);
    free(order);
    free(uniq);
    return P;
}

/* ------------------------------------------------------------------------ */
/* Non-dominated ranks (non-dominated sorting; the fronts behind the         */
/* section "Pareto filtering"): rank 0 is the non-dominated set of all rows, */
/* rank r the non-dominated set of the rows left after removing ranks < r.   */
/* Equal rows share their rank (neither dominates the other).  Plain peeling */
/* over the unique vectors, O(R U^2 m).  Returns the number of ranks R.      */
/* ------------------------------------------------------------------------ */
int32_t orc_pareto_ranks(const int64_t *obj, int64_t M, int m, int32_t *rank)
{
    if (M <= 0) return 0;
    for (int64_t i = 0; i < M; ++i) rank[i] = -1;
    int32_t r = 0;
    int64_t left = M;
    char *front = (char *)malloc((size_t)M);
    while (left > 0) {
        /* rows still unranked that no other unranked row dominates */
        for (int64_t a = 0; a < M; ++a) {
            front[a] = 0;
            if (rank[a] >= 0) continue;
            const int64_t *ya = obj + a * m;
            int dominated = 0;
            for (int64_t b = 0; b < M && !dominated; ++b) {
                if (rank[b] >= 0) continue;
                const int64_t *yb = obj + b * m;
                int ge = 1, gt = 0;
                for (int k = 0; k < m; ++k) {
                    if (yb[k] < ya[k]) { ge = 0; break; }
                    if (yb[k] > ya[k]) gt = 1;
                }
                dominated = ge && gt;
            }
            front[a] = (char)!dominated;
        }
        for (int64_t a = 0; a < M; ++a)
            if (front[a]) { rank[a] = r; --left; }
        ++r;
    }
    free(front);
    return r;
}

/* ------------------------------------------------------------------------ */
/* Exact hypervolume, Eq. (6) and Appendix A: the Lebesgue measure of the    */
/* union of boxes [r, y].  Points are first clipped to max(y, r), which      */
/* leaves the union unchanged.  Computed by slicing along the last          */
/* objective: HV_d(S) = sum_i (z_i - z_{i+1}) * HV_{d-1}(points with z >=    */
/* z_i), with the two-dimensional staircase as the base case.  Integers are */
/* exact with a 256-bit unsigned accumulator (four 64-bit limbs, little      */
/* endian).  Returns 0, 1 (invalid argument) or 5 (range above 2^256).       */
/* ------------------------------------------------------------------------ */
typedef struct { uint64_t w[4]; } orc_u256;

static orc_u256 orc_u256_add(orc_u256 a, orc_u256 b)
{
    orc_u256 r;
    unsigned __int128 carry = 0;
    for (int i = 0; i < 4; ++i) {
        unsigned __int128 s = (unsigned __int128)a.w[i] + b.w[i] + carry;
        r.w[i] = (uint64_t)s;
        carry = s >> 64;
    }
    return r;
}

static orc_u256 orc_u256_mul64(orc_u256 a, uint64_t b)
{
    orc_u256 r;
    unsigned __int128 carry = 0;
    for (int i = 0; i < 4; ++i) {
        unsigned __int128 p = (unsigned __int128)a.w[i] * b + carry;
        r.w[i] = (uint64_t)p;
        carry = p >> 64;
    }
    return r;
}

static int orc_hv_dim; /* coordinate used by the comparator */

static int orc_cmp_desc(const void *a, const void *b)
{
    uint64_t x = (*(const uint64_t *const *)a)[orc_hv_dim];
    uint64_t y = (*(const uint64_t *const *)b)[orc_hv_dim];
    return x > y ? -1 : (x < y ? 1 : 0);
}

/* pts: array of pointers to extent vectors (y - r, all >= 0); d >= 2. */
static orc_u256 orc_hv_slice(const uint64_t **pts, int64_t count, int d)
{
    orc_u256 vol = {{0, 0, 0, 0}};
    if (count == 0) return vol;
    const uint64_t **s = (const uint64_t **)malloc(sizeof(uint64_t *) * (size_t)count);
    memcpy(s, pts, sizeof(uint64_t *) * (size_t)count);
    orc_hv_dim = d - 1;
    qsort(s, (size_t)count, sizeof(uint64_t *), orc_cmp_desc);
    if (d == 2) {
        uint64_t best = 0;
        for (int64_t i = 0; i < count; ++i) {
            if (s[i][0] > best) best = s[i][0];
            uint64_t next = i + 1 < count ? s[i + 1][1] : 0;
            uint64_t h = s[i][1] - next;
            if (h) {
                orc_u256 area = {{best, 0, 0, 0}};
                vol = orc_u256_add(vol, orc_u256_mul64(area, h));
            }
        }
    } else {
        for (int64_t i = 0; i < count; ++i) {
            uint64_t next = i + 1 < count ? s[i + 1][d - 1] : 0;
            uint64_t h = s[i][d - 1] - next;
            if (h) {
                orc_u256 sub = orc_hv_slice(s, i + 1, d - 1);
                vol = orc_u256_add(vol, orc_u256_mul64(sub, h));
            }
        }
    }
    free(s);
    return vol;
}

int orc_hypervolume(const int64_t *pts, int64_t P, int m, const int64_t *ref, uint64_t *hv_out)
{
    if (P < 0 || m < 1 || m > 64 || (P > 0 && !pts) || !ref || !hv_out) return 1;
    for (int i = 0; i < 4; ++i) hv_out[i] = 0;
    if (P == 0) return 0;
    uint64_t *ext = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)P * (size_t)m);
    const uint64_t **ptr = (const uint64_t **)malloc(sizeof(uint64_t *) * (size_t)P);
    int bits_total = 0;
    for (int k = 0; k < m; ++k) {
        uint64_t mx = 0;
        for (int64_t p = 0; p < P; ++p) {
            __int128 d = (__int128)pts[p * m + k] - (__int128)ref[k];
            uint64_t v = d > 0 ? (uint64_t)d : 0; /* a difference of two int64 fits in uint64 */
            ext[p * m + k] = v;
            if (v > mx) mx = v;
        }
        int b = 0;
        while (b < 64 && (mx >> b) != 0) ++b;
        bits_total += b;
    }
    if (bits_total > 256) {
        free(ext);
        free(ptr);
        return 5;
    }
    orc_u256 v;
    if (m == 1) {
        uint64_t mx = 0;
        for (int64_t p = 0; p < P; ++p)
            if (ext[p] > mx) mx = ext[p];
        v.w[0] = mx;
        v.w[1] = v.w[2] = v.w[3] = 0;
    } else {
        for (int64_t p = 0; p < P; ++p) ptr[p] = ext + p * m;
        v = orc_hv_slice(ptr, P, m);
    }
    for (int i = 0; i < 4; ++i) hv_out[i] = v.w[i];
    free(ext);
    free(ptr);
    return 0;
}
