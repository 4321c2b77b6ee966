// Dense SB path: the coupling product runs on the matrix cores.
//
// For every step, per objective k, H_k = J^(k) Phi with Phi = phi(x) for all
// replicas at once ([Np x Np] . [Np x cols], the per-objective stacked form
// of Eq. 7: the scalarised matrix J(c) differs per weight vector, so it is
// never formed); the epilogue reduces h = sum_k coef_k(col) H_k with the
// column's folded coefficient coef_k = -dt c0 c_k 2^e_k, applies the
// symplectic update and the wall (Eq. 9), and writes phi(x) for the next step.
//
// Operand formats (J stored per objective, scaled by a power of two 2^-e_k):
//   FP32: J fp32 (exact for |W| < 2^24), Phi fp32 (x for ballistic SB,
//         sgn x for discrete SB), 32x32x2 fp32 MFMA;
//   BF16: discrete SB only: J bf16, Phi = +-1 exact in bf16, 32x32x16 MFMA;
//   FP8 : discrete SB only: J e4m3, Phi = +-1 exact in e4m3, 32x32x64 MFMA.
// All accumulate in fp32.
//
// Layout (all device, zero padded to Np = ceil128(n) spins and colsP =
// ceil128(W*R) columns): x, y fp32 [colsP][Np]; Phi [colsP][Np]; J [m][Np][Np]
// (symmetric, so rows serve as the A operand directly).
//
// Tiling: a 256-thread block owns 64 spins x 128 columns; wave (wr, wc) owns
// 32 spins x 64 columns (two 32x32 accumulators per objective).  For every
// MFMA the A and B fragments of a lane come from the same k positions
// (lane half h, slot j -> k0 + h*KG/2 + j), which pairs them correctly for
// any internal k order of the instruction.  The staged tile (below) doubles
// the block to 128 x 128 and reads each operand chunk once through LDS.
#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "device_common.hpp"
#include "internal.hpp"

namespace qaia {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kDB = 256;      // threads per block
constexpr int kTileM = 64;    // spins per block
constexpr int kTileN = 128;   // columns per block

// accumulator slot i of lane l holds row (i/4)*8 + (l/32)*4 + i%4, column l%32
__device__ __forceinline__ int acc_row(int half, int i) { return (i >> 2) * 8 + half * 4 + (i & 3); }

template <int PREC> struct PrecInfo;
template <> struct PrecInfo<QAIA_FP32> { typedef float T; static constexpr int KG = 8; };
template <> struct PrecInfo<QAIA_BF16> { typedef uint16_t T; static constexpr int KG = 16; };
template <> struct PrecInfo<QAIA_FP8> { typedef uint8_t T; static constexpr int KG = 64; };

__device__ __forceinline__ uint16_t bf16_pm1(float x) { return x >= 0.0f ? 0x3F80u : 0xBF80u; }
__device__ __forceinline__ uint8_t fp8_pm1(float x) { return x >= 0.0f ? 0x38u : 0xB8u; }

// MT: compile-time objective count (accumulator tiles); objectives k >= m
// (run time, m <= MT) are skipped uniformly across the block.
template <int PREC, int MT>
__device__ __forceinline__ void mma_tile(const void *Jv, const void *phiv, int Np_, int m, int row_w,
                                         int col_w, int half, int lr, f16v (&acc)[MT][2]) {
    typedef typename PrecInfo<PREC>::T T;
    constexpr int KG = PrecInfo<PREC>::KG;
    constexpr int M = MT;
    const T *J = (const T *)Jv;
    const T *phi = (const T *)phiv;
    const size_t Np = (size_t)Np_;
    const T *arow[M];
#pragma unroll
    for (int k = 0; k < M; ++k) arow[k] = J + ((size_t)(k < m ? k : 0) * Np + row_w + lr) * Np + half * (KG / 2);
    const T *bcol[2];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) bcol[cb] = phi + (size_t)(col_w + cb * 32 + lr) * Np + half * (KG / 2);

    for (int k0 = 0; k0 < Np_; k0 += KG) {
        if constexpr (PREC == QAIA_FP32) {
            float4 av[M], bv[2];
#pragma unroll
            for (int k = 0; k < M; ++k) av[k] = k < m ? *(const float4 *)(arow[k] + k0) : make_float4(0, 0, 0, 0);
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) bv[cb] = *(const float4 *)(bcol[cb] + k0);
#pragma unroll
            for (int k = 0; k < M; ++k)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) {
                    if (k >= m) continue;
                    acc[k][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[k].x, bv[cb].x, acc[k][cb], 0, 0, 0);
                    acc[k][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[k].y, bv[cb].y, acc[k][cb], 0, 0, 0);
                    acc[k][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[k].z, bv[cb].z, acc[k][cb], 0, 0, 0);
                    acc[k][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[k].w, bv[cb].w, acc[k][cb], 0, 0, 0);
                }
        } else if constexpr (PREC == QAIA_BF16) {
            bf16x8 av[M], bv[2];
#pragma unroll
            for (int k = 0; k < M; ++k) av[k] = *(const bf16x8 *)(arow[k] + k0);  // k >= m reads objective 0
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) bv[cb] = *(const bf16x8 *)(bcol[cb] + k0);
#pragma unroll
            for (int k = 0; k < M; ++k)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
                    if (k < m) acc[k][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[k], bv[cb], acc[k][cb], 0, 0, 0);
        } else {
            i32x8 av[M], bv[2];
#pragma unroll
            for (int k = 0; k < M; ++k) av[k] = *(const i32x8 *)(arow[k] + k0);  // k >= m reads objective 0
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) bv[cb] = *(const i32x8 *)(bcol[cb] + k0);
            // format 0 = e4m3 for both operands, block scales 127 = 2^0
#pragma unroll
            for (int k = 0; k < M; ++k)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
                    if (k < m)
                        acc[k][cb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                            av[k], bv[cb], acc[k][cb], 0, 0, 0, 127, 0, 127);
        }
    }
}

// One step for the tile (bx, by) of a job; MT accumulator tiles, j.m <= MT.
template <int PREC, int MT, bool DSB>
__device__ __forceinline__ void dense_step_body(const DenseJob &j, int t, int bx, int by) {
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int half = l >> 5, lr = l & 31;
    const int row_w = by * kTileM + (wv & 1) * 32;
    const int col_w = bx * kTileN + (wv >> 1) * 64;
    constexpr int M = MT;
    const int m = j.m;
    // discrete SB: x in place, Phi double-buffered; ballistic SB: x double-buffered, Phi = x
    const bool even = (t & 1) == 0;
    const float *x_in = DSB ? j.xa : (even ? j.xa : j.xb);
    float *x_out = DSB ? j.xa : (even ? j.xb : j.xa);
    const void *phi_in = DSB ? (even ? j.pa : j.pb) : (const void *)x_in;
    void *phi_out = DSB ? (even ? j.pb : j.pa) : nullptr;
    f16v acc[M][2];
#pragma unroll
    for (int k = 0; k < M; ++k)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[k][cb][i] = 0.0f;
    mma_tile<PREC, M>(j.J, phi_in, j.Np, m, row_w, col_w, half, lr, acc);

    const float kt = j.kt_tab[t];
    const size_t Np = (size_t)j.Np;
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        const int col = col_w + cb * 32 + lr;
        float cf[M];
#pragma unroll
        for (int k = 0; k < M; ++k) cf[k] = k < m ? j.coef[(size_t)col * m + k] : 0.0f;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int row = row_w + acc_row(half, g * 4);  // four consecutive spins row..row+3
            const size_t off = (size_t)col * Np + row;
            float4 xv = *(const float4 *)(x_in + off);
            float4 yv = *(const float4 *)(j.y + off);
            float xs[4] = {xv.x, xv.y, xv.z, xv.w}, ys[4] = {yv.x, yv.y, yv.z, yv.w};
#pragma unroll
            for (int ii = 0; ii < 4; ++ii) {
                float h = 0.0f;
#pragma unroll
                for (int k = 0; k < M; ++k)
                    if (k < m) h = fmaf(cf[k], acc[k][cb][g * 4 + ii], h);
                float yn = fmaf(kt, xs[ii], ys[ii]) + h;
                if (j.dt_alpha != 0.0f && col < j.cols && row + ii < j.N) {
                    const uint64_t g = (uint64_t)col + j.offset;
                    const uint64_t nidx = (g * (uint64_t)j.steps + (uint64_t)t) * (uint64_t)j.N + (uint64_t)(row + ii);
                    yn = fmaf(j.dt_alpha, noise_value(j.seed, nidx), yn);
                }
                float xn = fmaf(j.dta0, yn, xs[ii]);
                wall(xn, yn);
                xs[ii] = xn;
                ys[ii] = yn;
            }
            *(float4 *)(x_out + off) = make_float4(xs[0], xs[1], xs[2], xs[3]);
            *(float4 *)(j.y + off) = make_float4(ys[0], ys[1], ys[2], ys[3]);
            if (DSB) {
                if constexpr (PREC == QAIA_FP32) {
                    *(float4 *)((float *)phi_out + off) =
                        make_float4(sgn1(xs[0]), sgn1(xs[1]), sgn1(xs[2]), sgn1(xs[3]));
                } else if constexpr (PREC == QAIA_BF16) {
                    uint2 v;
                    v.x = (uint32_t)bf16_pm1(xs[0]) | ((uint32_t)bf16_pm1(xs[1]) << 16);
                    v.y = (uint32_t)bf16_pm1(xs[2]) | ((uint32_t)bf16_pm1(xs[3]) << 16);
                    *(uint2 *)((uint16_t *)phi_out + off) = v;
                } else {
                    uint32_t v = (uint32_t)fp8_pm1(xs[0]) | ((uint32_t)fp8_pm1(xs[1]) << 8) |
                                 ((uint32_t)fp8_pm1(xs[2]) << 16) | ((uint32_t)fp8_pm1(xs[3]) << 24);
                    *(uint32_t *)((uint8_t *)phi_out + off) = v;
                }
            }
            if (j.trace != nullptr && t < j.trace_steps && col < j.cols) {
#pragma unroll
                for (int ii = 0; ii < 4; ++ii)
                    if (row + ii < j.N)
                        j.trace[((size_t)col * j.trace_steps + t) * j.N + row + ii] = xs[ii];
            }
        }
    }
}

template <int PREC, int M, bool DSB>
__global__ __launch_bounds__(kDB) void dense_step_kernel(DenseJob j, int t) {
    dense_step_body<PREC, M, DSB>(j, t, blockIdx.x, blockIdx.y);
}

// Grouped step over a ragged batch of dense jobs (each with its own n, m,
// columns): block b runs tile b - block_start[i] of job i.
template <int PREC, bool DSB>
__global__ __launch_bounds__(kDB) void dense_batch_step_kernel(const DenseJob *__restrict__ jobs, int count,
                                                               const int64_t *__restrict__ block_start, int t) {
    const int64_t b = blockIdx.x;
    int i = 0;
    while (i + 1 < count && block_start[i + 1] <= b) ++i;
    const DenseJob j = jobs[i];
    const int64_t local = b - block_start[i];
    dense_step_body<PREC, 4, DSB>(j, t, (int)(local % j.tiles_x), (int)(local / j.tiles_x));
}

// ---------------------------------------------------------------------------
// Staged tile: a block of NW waves owns 128 spins x 64 CBW columns (CBW = 2,
// or 4 for the wide BF16 tile); wave (wr, wc) owns (32 RB) x (32 CBW) (RB x CBW
// accumulators per objective, RB = 8 / NW).  The k dimension runs in chunks
// of CB bytes per row (64 or 128).  Each chunk of the
// block's J rows (all objectives) and Phi columns is copied to LDS once (by
// global_load_lds, below) and read there by every wave that needs it; D stage
// buffers form a ring and there is one barrier per chunk.  Loads of
// objectives k >= m (batched jobs with m < MT) read objective m-1; their
// MFMAs are skipped by a uniform branch and their accumulators unused.
constexpr int kT2 = 128;          // tile height and width
constexpr int kHsPitch = kT2 + 4; // LDS pitch (floats) of the epilogue's h tile

// In LDS a chunk row is CB bytes (the row pitch, no padding) of 16-byte parts;
// logical part p of row r sits at physical part p ^ sw(r), with sw(r) =
// (r >> 2) & 3 for 64-byte rows and (r >> 1) & 7 for 128-byte rows.  Either
// way the 16 rows of a 16-lane fragment read (one logical part) land on 16
// distinct 4-bank groups, and a 64-lane chunk copy writes 1024 contiguous
// bytes: both free of bank conflicts.
template <int CB>
__host__ __device__ constexpr int row_swizzle(int r) { return CB == 64 ? (r >> 2) & 3 : (r >> 1) & 7; }

template <int MT, int CB>
constexpr int staged_buf_bytes() { return (MT + 1) * kT2 * CB; }

// 128-byte chunks (whole 128-byte requests per row) where the stage ring fits
// LDS; m = 4 keeps 64-byte chunks (five 128-row operands per stage).
template <int MT>
constexpr int staged_chunk() { return MT <= 3 ? 128 : 64; }

// Work on one LDS chunk is split into two units so that the fragment reads of
// one unit overlap the MFMAs of the other (with a single fragment set, wide
// tiles, into one unit per k-group, run one after the other).  A unit is KPU
// consecutive k-groups
// of the chunk (k-groups of 32 bytes for FP32 and BF16, 64 bytes for FP8);
// when a chunk holds a single k-group (FP8 in 64-byte chunks) a unit is one
// half of the wave's accumulators instead (its two 32-row halves with all
// its column blocks, or, when the wave owns 32 rows, half of its CBW 32-column
// blocks).  Each accumulator receives
// the chunk's k-groups in increasing order whatever the split.  For every
// MFMA the A and B fragments of a lane come from the same k positions (lane
// half h, slot j), so any internal k order of the instruction pairs them.
template <int PREC, int CB>
constexpr int kgroups_per_chunk() { return CB / (PrecInfo<PREC>::KG * (int)sizeof(typename PrecInfo<PREC>::T)); }
template <int PREC, int CB>
constexpr bool half_units() { return kgroups_per_chunk<PREC, CB>() == 1; }
// k-groups per unit: half of the chunk's, or one with a single fragment set
// (wide tiles, CBW > 2), whose loop takes the chunk's k-groups one by one
template <int PREC, int CB, int CBW = 2>
constexpr int kg_per_unit() {
    return half_units<PREC, CB>() || CBW > 2 ? 1 : kgroups_per_chunk<PREC, CB>() / 2;
}
template <int PREC, int CB, int CBW>
constexpr int units_per_chunk() {
    return half_units<PREC, CB>() ? 2 : kgroups_per_chunk<PREC, CB>() / kg_per_unit<PREC, CB, CBW>();
}

template <int PREC> struct FragType;
template <> struct FragType<QAIA_FP32> { typedef float4 V; };
template <> struct FragType<QAIA_BF16> { typedef bf16x8 V; };
template <> struct FragType<QAIA_FP8> { typedef i32x8 V; };

template <int PREC, int MT, int RB, int KPU, int CBW = 2> struct Frags {
    typename FragType<PREC>::V a[KPU][MT][RB], b[KPU][CBW];
};

struct LaneLds {
    const char *a, *b;  // this lane's first A row and first B row in a stage buffer
    int sw;             // swizzle of every row this lane reads (rows lr + 32 j)
    int half;
};

__device__ __forceinline__ u32x4 lds16(const char *row, int part, int sw) {
    return *(const u32x4 *)(row + ((part ^ sw) << 4));
}

template <int PREC, int MT, int RB, int CB, int CBW = 2>
__device__ __forceinline__ void frag_load(Frags<PREC, MT, RB, kg_per_unit<PREC, CB, CBW>(), CBW> &f, const LaneLds &L, int u) {
    constexpr int KPU = kg_per_unit<PREC, CB, CBW>();
    if constexpr (PREC == QAIA_FP8) {
        // lane half h holds k = 32h + 0..31 of a 64-byte k-group: parts 4g + 2h, 4g + 2h + 1
        auto frag = [&](const char *row, int g) {
            const u32x4 lo = lds16(row, 4 * g + 2 * L.half, L.sw), hi = lds16(row, 4 * g + 2 * L.half + 1, L.sw);
            return __builtin_bit_cast(i32x8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
        };
        if constexpr (half_units<PREC, CB>()) {
            if constexpr (RB == 2) {
                // unit u = rows r2 = u, every column block
#pragma unroll
                for (int c2 = 0; c2 < CBW; ++c2) f.b[0][c2] = frag(L.b + c2 * 32 * CB, 0);
#pragma unroll
                for (int k = 0; k < MT; ++k) f.a[0][k][0] = frag(L.a + (k * kT2 + u * 32) * CB, 0);
            } else {
                // unit u = column blocks u CBW / 2 .. (u + 1) CBW / 2 - 1, the wave's 32 rows
#pragma unroll
                for (int j = 0; j < CBW / 2; ++j) f.b[0][j] = frag(L.b + (u * CBW / 2 + j) * 32 * CB, 0);
#pragma unroll
                for (int k = 0; k < MT; ++k) f.a[0][k][0] = frag(L.a + k * kT2 * CB, 0);
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < KPU; ++kk) {
                const int g = u * KPU + kk;
#pragma unroll
                for (int c2 = 0; c2 < CBW; ++c2) f.b[kk][c2] = frag(L.b + c2 * 32 * CB, g);
#pragma unroll
                for (int k = 0; k < MT; ++k)
#pragma unroll
                    for (int r2 = 0; r2 < RB; ++r2) f.a[kk][k][r2] = frag(L.a + (k * kT2 + r2 * 32) * CB, g);
            }
        }
    } else {
        // k-group g: lane half h holds its 16 bytes at logical part 2g + h
        typedef typename FragType<PREC>::V VT;
#pragma unroll
        for (int kk = 0; kk < KPU; ++kk) {
            const int p = 2 * (u * KPU + kk) + L.half;
#pragma unroll
            for (int c2 = 0; c2 < CBW; ++c2) f.b[kk][c2] = __builtin_bit_cast(VT, lds16(L.b + c2 * 32 * CB, p, L.sw));
#pragma unroll
            for (int k = 0; k < MT; ++k)
#pragma unroll
                for (int r2 = 0; r2 < RB; ++r2)
                    f.a[kk][k][r2] = __builtin_bit_cast(VT, lds16(L.a + (k * kT2 + r2 * 32) * CB, p, L.sw));
        }
    }
}

// One MFMA of objective k on accumulator (r2, c2) with unit-local k-group kk.
template <int PREC, int MT, int RB, int KPU, int CBW>
__device__ __forceinline__ void mma_one(const Frags<PREC, MT, RB, KPU, CBW> &f, f16v &a, int kk, int k, int ra, int cb,
                                        int j) {
    if constexpr (PREC == QAIA_FP8) {
        a = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(f.a[kk][k][ra], f.b[kk][cb], a, 0, 0, 0, 127, 0, 127);
    } else if constexpr (PREC == QAIA_BF16) {
        a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[kk][k][ra], f.b[kk][cb], a, 0, 0, 0);
    } else {
        const float av = j == 0 ? f.a[kk][k][ra].x : j == 1 ? f.a[kk][k][ra].y : j == 2 ? f.a[kk][k][ra].z
                                                                                       : f.a[kk][k][ra].w;
        const float bv = j == 0 ? f.b[kk][cb].x : j == 1 ? f.b[kk][cb].y : j == 2 ? f.b[kk][cb].z : f.b[kk][cb].w;
        a = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, a, 0, 0, 0);
    }
}

// The MFMAs of unit u in a fixed order; after the i-th, hook(i) runs (the
// copy interleaving below).  MFMAs per unit with m = MT: unit_mfmas().
template <int PREC, int MT, int RB, int CB, int CBW = 2>
constexpr int unit_mfmas() {
    return half_units<PREC, CB>() ? MT * (RB == 2 ? CBW : CBW / 2)
                                  : kg_per_unit<PREC, CB, CBW>() * MT * RB * CBW * (PREC == QAIA_FP32 ? 4 : 1);
}

template <int PREC, int MT, int RB, int CB, int CBW, typename Hook>
__device__ __forceinline__ void unit_mma(const Frags<PREC, MT, RB, kg_per_unit<PREC, CB, CBW>(), CBW> &f, int m, int u,
                                         f16v (&acc)[MT][RB][CBW], Hook &&hook) {
    constexpr int KPU = kg_per_unit<PREC, CB, CBW>();
    constexpr int NJ = PREC == QAIA_FP32 ? 4 : 1;  // fp32: four 32x32x2 steps per 16-byte fragment
    int i = 0;
    if constexpr (half_units<PREC, CB>()) {
#pragma unroll
        for (int k = 0; k < MT; ++k) {
            if (k >= m) break;
            if constexpr (RB == 2) {
#pragma unroll
                for (int c2 = 0; c2 < CBW; ++c2) {
                    mma_one(f, acc[k][u][c2], 0, k, 0, c2, 0);
                    hook(i++);
                }
            } else {
#pragma unroll
                for (int j = 0; j < CBW / 2; ++j) {
                    mma_one(f, acc[k][0][u * CBW / 2 + j], 0, k, 0, j, 0);
                    hook(i++);
                }
            }
        }
    } else {
#pragma unroll
        for (int kk = 0; kk < KPU; ++kk)
#pragma unroll
            for (int k = 0; k < MT; ++k) {
                if (k >= m) break;
#pragma unroll
                for (int r2 = 0; r2 < RB; ++r2)
#pragma unroll
                    for (int c2 = 0; c2 < CBW; ++c2)
#pragma unroll
                        for (int j = 0; j < NJ; ++j) {
                            mma_one(f, acc[k][r2][c2], kk, k, r2, c2, j);
                            hook(i++);
                        }
            }
    }
}

template <int PREC, int MT, int RB, int CB, int CBW = 2>
__device__ __forceinline__ void frag_mma(const Frags<PREC, MT, RB, kg_per_unit<PREC, CB, CBW>(), CBW> &f, int m, int u,
                                         f16v (&acc)[MT][RB][CBW]) {
    unit_mma<PREC, MT, RB, CB, CBW>(f, m, u, acc, [](int) {});
}

// frag_mma with NC copies of the next chunk interleaved: copy j is issued
// after MFMA (j * NM) / NC of the unit (NM MFMAs when m == MT), so a copy that
// waits for room in the memory queue stalls behind queued matrix work instead
// of in front of an idle matrix pipe.  Copies not yet issued (m < MT) follow.
template <int PREC, int MT, int RB, int CB, int NC, int CBW = 2, typename Copy>
__device__ __forceinline__ void frag_mma_cp(const Frags<PREC, MT, RB, kg_per_unit<PREC, CB, CBW>(), CBW> &f, int m, int u,
                                            f16v (&acc)[MT][RB][CBW], Copy &&copy) {
    constexpr int NM = unit_mfmas<PREC, MT, RB, CB, CBW>();
    int j = 0;
    unit_mma<PREC, MT, RB, CB, CBW>(f, m, u, acc, [&](int i) {
        if constexpr (NC > 0) {
            if (j < NC && i == (j * NM) / NC) {
                __builtin_amdgcn_sched_barrier(0);
                copy(j);
                __builtin_amdgcn_sched_barrier(0);
                ++j;
            }
        }
    });
#pragma unroll
    for (; j < NC; ++j) copy(j);
}

// Direct-to-LDS variant of the staged tile: every chunk is copied by
// global_load_lds (16 bytes per lane straight into LDS, no registers), into a
// ring of D stage buffers, D - 1 chunks ahead of the MFMAs.  A stage holds
// (MT + 1) x 128 rows x CB / 16 granules of 16 bytes; with NW waves, each
// makes PER = (MT + 1) x 128 x CB / 16 / (64 NW) copies per chunk, wave w
// copying granules [(w * PER + i) * 64, +64) with its i-th copy; lane L of
// that copy fetches the global 16 bytes that belong at granule g = base + L
// of the swizzled layout (row g / (CB / 16), physical part g % (CB / 16)).
typedef __attribute__((address_space(3))) void lds_void_t;

template <int MT, int CB>
constexpr int dma_stages() {
    // 64-byte chunks: four stage buffers (three for m = 4: 3 x 40 KB); filling
    // all 160 KB of LDS with five measured slower.  128-byte chunks: two for
    // m = 3 (2 x 64 KB), three below
    if constexpr (CB == 128) return MT <= 2 ? 3 : 2;
    return MT <= 3 ? 4 : 3;
}

// The copy is issued from inline assembly (M0 = the wave's LDS destination,
// one wait state, then global_load_lds_dwordx4) so that the compiler's wait
// insertion does not see an LDS-writing memory operation: with one pending it
// treats the LDS counter as out of order and drains it completely before every
// MFMA group, serialising the fragment reads with the MFMAs.  The copies are
// ordered by hand (dma_wait, lds_barrier).  M0 is listed as clobbered, but
// it is a register the compiler reserves (it warns that such a clobber is not
// guaranteed to be honoured): what makes the write safe is that the compiler
// allocates no values of its own to M0, and no compiler-generated instruction
// in these kernels reads it (in their ISA every M0 write is this copy's).
// The compiler's own LDS-DMA builtin would manage M0 itself, but brings back
// the waits described above.
template <int PER>
__device__ __forceinline__ void dma_copy(char *stage, const char *src, size_t koff, int wave, int i) {
    const uint32_t base = (uint32_t)(uintptr_t)(lds_void_t *)stage;
    const uint32_t dst = __builtin_amdgcn_readfirstlane(base + (uint32_t)(wave * PER + i) * 64 * 16);
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(src + koff), "s"(dst)
                 : "memory", "m0");
}

template <int PER>
__device__ __forceinline__ void dma_chunk(char *stage, const char *const (&src)[PER], size_t koff, int wave) {
#pragma unroll
    for (int i = 0; i < PER; ++i) dma_copy<PER>(stage, src[i], koff, wave, i);
}

// this wave's copies of all but the newest `later` chunks have landed, with
// X further loads (the epilogue's prefetch) issued after those chunks'
// copies; later <= 6, and (later * PER + X) must fit the 6-bit vmcnt field
// for every reachable `later` (asserted by the caller; unreachable cases clamp)
constexpr int vm_imm(int n) { return n < 63 ? n : 63; }

template <int PER, int X = 0>
__device__ __forceinline__ void dma_wait(int later) {
    switch (later) {
        case 0: asm volatile("s_waitcnt vmcnt(%0)" ::"n"(vm_imm(X)) : "memory"); break;
        case 1: asm volatile("s_waitcnt vmcnt(%0)" ::"n"(vm_imm(PER + X)) : "memory"); break;
        case 2: asm volatile("s_waitcnt vmcnt(%0)" ::"n"(vm_imm(2 * PER + X)) : "memory"); break;
        case 3: asm volatile("s_waitcnt vmcnt(%0)" ::"n"(vm_imm(3 * PER + X)) : "memory"); break;
        case 4: asm volatile("s_waitcnt vmcnt(%0)" ::"n"(vm_imm(4 * PER + X)) : "memory"); break;
        case 5: asm volatile("s_waitcnt vmcnt(%0)" ::"n"(vm_imm(5 * PER + X)) : "memory"); break;
        default: asm volatile("s_waitcnt vmcnt(%0)" ::"n"(vm_imm(6 * PER + X)) : "memory"); break;
    }
}

// This wave's LDS reads have returned (so a stage it read may be refilled once
// every wave is past the barrier), then the block barrier.  The wait is a
// compiler-visible s_waitcnt (lgkmcnt 0, vmcnt and expcnt left at their
// maxima, gfx9 encoding): it also retires any scalar load the compiler hoisted
// above the loop, which would otherwise force a full LDS drain before every
// MFMA group instead of a wait for the older fragment unit only.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_s_waitcnt(0xC07F);
    asm volatile("s_barrier" ::: "memory");
}

// Epilogue prefetch: NPF / 2 rows of 16 bytes from each of px and py, row i
// at element offset off0 + i * stride, into xpf / ypf, issued a few chunks
// before the end of the k loop (the waits that follow count the NPF loads).
template <int NPF>
struct EpiPrefetch {
    static constexpr int N = NPF > 0 ? NPF / 2 : 1;
    const float *px, *py;
    size_t off0, stride;
    f32x4 xpf[N], ypf[N];
};

// Global-address-space loads: a flat load (what a pointer read from memory
// compiles to) would also count against the LDS counter that the k loop's
// barriers drain.
typedef __attribute__((address_space(1))) const f32x4 global_f32x4;

template <int NPF>
__device__ __forceinline__ void epi_prefetch(EpiPrefetch<NPF> &pf) {
    if constexpr (NPF > 0) {
#pragma unroll
        for (int i = 0; i < NPF / 2; ++i) {
            const size_t off = pf.off0 + (size_t)i * pf.stride;
            pf.xpf[i] = *(global_f32x4 *)(pf.px + off);
            pf.ypf[i] = *(global_f32x4 *)(pf.py + off);
        }
    }
}

// The wide tile (CBW = 4) copies 3 x 128 + 256 rows of 64 bytes per chunk
// into three 40 KB stages; its epilogue's 256-column h tile (135 KB) reuses
// them.  It keeps one fragment set (the 192 accumulator registers of m = 3
// leave no room for two; the second wave on each SIMD overlaps the fragment
// reads instead).
template <int MT, int CB, int CBW>
constexpr int wide_stages() { return CBW == 2 ? dma_stages<MT, CB>() : CB == 128 ? 2 : 3; }
// wide tiles: 128-byte chunks (two stages, all 160 KB of LDS) for BF16 with
// m = 3 (94.4 against 96.5 ms per 1000 C3 steps with 64-byte chunks in three
// stages); 64-byte chunks otherwise
template <int PREC, int MT>
constexpr int wide_chunk() { return PREC == QAIA_BF16 && MT == 3 ? 128 : 64; }

template <int PREC, int MT, int NPF, int NW, int CB, int CBW = 2>
__device__ __forceinline__ void mma_tile_dma(const void *Jv, const void *phiv, int Np_, int m, int row0, int col0,
                                             int wr, int wc, int half, int lr, f16v (&acc)[MT][8 / NW][CBW],
                                             char *lds, EpiPrefetch<NPF> &pf) {
    typedef typename PrecInfo<PREC>::T T;
    constexpr int ES = sizeof(T);
    constexpr int RB = 8 / NW;                // 32-row accumulator blocks per wave
    constexpr int GPR = CB / 16;              // 16-byte granules per chunk row
    constexpr int TW = 64 * CBW;              // tile columns
    constexpr int ROWS = MT * kT2 + TW;       // stage rows
    static_assert((ROWS * GPR) % (64 * NW) == 0, "copies per wave");
    constexpr int PER = ROWS * GPR / (64 * NW);  // copies per wave per chunk
    constexpr int P0 = PER / 2, P1 = PER - P0;    // spread over the two MFMA groups
    constexpr int KPU = kg_per_unit<PREC, CB, CBW>();
    constexpr bool SINGLE = CBW > 2;          // one fragment set (register budget)
    constexpr int D = wide_stages<MT, CB, CBW>();
    static_assert(D >= 2 && D - 2 <= 6, "stage ring depth");
    static_assert((D - 2) * PER + NPF <= 63, "vmcnt range");
    const size_t Np = (size_t)Np_;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const char *src[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int g = (wave * PER + i) * 64 + lane;
        const int R = g / GPR, p = (g % GPR) ^ row_swizzle<CB>(R);
        if (R < MT * kT2) {
            const int k0 = R / kT2 < m ? R / kT2 : m - 1;
            src[i] = (const char *)Jv + (((size_t)k0 * Np + row0 + (R % kT2)) * Np) * ES + p * 16;
        } else {
            src[i] = (const char *)phiv + ((size_t)(col0 + R - MT * kT2) * Np) * ES + p * 16;
        }
    }
    constexpr int SB = ROWS * CB;
    char *S[D];
#pragma unroll
    for (int i = 0; i < D; ++i) S[i] = lds + i * SB;
    const int nk = (int)(Np * ES / CB);
    const int sw = row_swizzle<CB>(lr);
    const int aoff = (wr * 32 * RB + lr) * CB, boff = (MT * kT2 + wc * 32 * CBW + lr) * CB;
    auto lane_lds = [&](int st) { return LaneLds{S[st] + aoff, S[st] + boff, sw, half}; };
#pragma unroll
    for (int q = 0; q < D - 1; ++q)
        if (q < nk) dma_chunk<PER>(S[q], src, (size_t)q * CB, wave);
    // The prefetch is issued at the end of iteration c_pf, PFD chunks before
    // the one that issues the last chunk's copies (or after the prologue when
    // c_pf is -1).  Chunks whose copies were issued before it, c_pf < c <=
    // c_pf + D - 1, wait with its NPF loads counted as newer.  Distances 0 to
    // 8 measured the same within noise (BF16, m = 3); 0 keeps the registers
    // free longest.
    constexpr int PFD = 0;
    const int c_pf = nk - D - PFD > -1 ? nk - D - PFD : -1;
    if constexpr (NPF > 0) {
        if (c_pf < 0) epi_prefetch(pf);
    }
    // Rotation: after the barrier for chunk c, unit 0 of chunk c is read while
    // unit 1 of chunk c - 1 (already in registers) runs, then unit 1 of chunk c
    // is read while unit 0 of chunk c runs.
    Frags<PREC, MT, RB, KPU, CBW> f0, f1;
    for (int c0 = 0; c0 < nk; c0 += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) {
            const int c = c0 + u;
            if (c < nk) {
                const int later = (nk - 1 - c) < (D - 2) ? (nk - 1 - c) : (D - 2);
                if (NPF > 0 && c > c_pf && c <= c_pf + D - 1) dma_wait<PER, NPF>(later);
                else dma_wait<PER>(later);
                lds_barrier();  // chunk c is in LDS for every wave; all waves are done reading chunk c - 1
                // the copies of chunk c + D - 1 (into the stage chunk c - 1 used):
                // BF16 / FP32 spread them over this iteration's two MFMA groups,
                // FP8 (six MFMAs per group for m = 3, measured slower spread)
                // issues them all here
                constexpr bool kSpread = PREC != QAIA_FP8;
                const bool issue = c + D - 1 < nk;
                char *const nst = S[(u + D - 1) % D];
                const size_t koff = (size_t)(c + D - 1) * CB;
                if (!kSpread && issue) dma_chunk<PER>(nst, src, koff, wave);
                auto copy0 = [&](int i) {
                    if (kSpread && issue) dma_copy<PER>(nst, src[i], koff, wave, i);
                };
                auto copy1 = [&](int i) {
                    if (kSpread && issue) dma_copy<PER>(nst, src[P0 + i], koff, wave, P0 + i);
                };
                const LaneLds L = lane_lds(u);
                // scheduling barriers keep each unit's reads ahead of the other unit's MFMAs
                if constexpr (SINGLE) {
                    // units one after the other in one fragment set; the
                    // chunk's copies spread over them in equal groups
                    constexpr int U = units_per_chunk<PREC, CB, CBW>();
                    constexpr int NG = (PER + U - 1) / U;
#pragma unroll
                    for (int uu = 0; uu < U; ++uu) {
                        auto copyg = [&](int i) {
                            const int ci = uu * NG + i;
                            if (kSpread && issue && ci < PER) dma_copy<PER>(nst, src[ci], koff, wave, ci);
                        };
                        frag_load<PREC, MT, RB, CB, CBW>(f0, L, uu);
                        __builtin_amdgcn_sched_barrier(0);
                        frag_mma_cp<PREC, MT, RB, CB, kSpread ? NG : 0, CBW>(f0, m, uu, acc, copyg);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                } else {
                frag_load<PREC, MT, RB, CB, CBW>(f0, L, 0);
                __builtin_amdgcn_sched_barrier(0);
                if (c > 0) {
                    frag_mma_cp<PREC, MT, RB, CB, kSpread ? P0 : 0, CBW>(f1, m, 1, acc, copy0);
                } else {
#pragma unroll
                    for (int i = 0; i < P0; ++i) copy0(i);
                }
                __builtin_amdgcn_sched_barrier(0);
                frag_load<PREC, MT, RB, CB, CBW>(f1, L, 1);
                __builtin_amdgcn_sched_barrier(0);
                frag_mma_cp<PREC, MT, RB, CB, kSpread ? P1 : 0, CBW>(f0, m, 0, acc, copy1);
                }
                __builtin_amdgcn_sched_barrier(0);
                if constexpr (NPF > 0) {
                    if (c == c_pf) epi_prefetch(pf);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
    }
    if constexpr (!SINGLE) frag_mma<PREC, MT, RB, CB, CBW>(f1, m, 1, acc);
    lds_barrier();
}

// Where the epilogue prefetch fits beside the accumulators and fragments
// without spilling (checked on the compiled kernels, 128-byte chunks): m = 1
// everywhere; m = 2 with four waves except FP8 (whose 32-byte fragments
// leave no room).
template <int PREC, int MT, int NW>
constexpr bool staged_prefetch(bool grouped) {
    (void)grouped;
    if constexpr (NW == 8) return MT == 1;
    return MT == 1 || (MT == 2 && PREC != QAIA_FP8);
}

// FIXED_M: the job's m equals MT (single-job launches), so objective guards fold away.
// PF: the epilogue's x and y are prefetched into registers during the k loop
// (where they fit beside the accumulators and fragments without spilling).
template <int PREC, int MT, bool DSB, bool FIXED_M, bool PF, int NW, int CBW = 2>
__device__ __forceinline__ void dense_step_staged_body(const DenseJob &j, int t, int bx, int by, char *lds) {
    constexpr int RB = 8 / NW;   // 32-row accumulator blocks per wave: waves own (32 RB) x (32 CBW)
    constexpr int CPI = 2 * NW;  // columns per pass of the update phase
    constexpr int TW = 64 * CBW; // tile columns
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int half = l >> 5, lr = l & 31;
    const int wr = wv % (NW / 2), wc = wv / (NW / 2);
    const int row0 = by * kT2, col0 = bx * TW;
    constexpr int M = MT;
    const int m = FIXED_M ? MT : j.m;
    const bool even = (t & 1) == 0;
    const float *x_in = DSB ? j.xa : (even ? j.xa : j.xb);
    float *x_out = DSB ? j.xa : (even ? j.xb : j.xa);
    const void *phi_in = DSB ? (even ? j.pa : j.pb) : (const void *)x_in;
    void *phi_out = DSB ? (even ? j.pb : j.pa) : nullptr;
    f16v acc[M][RB][CBW];
#pragma unroll
    for (int k = 0; k < M; ++k)
#pragma unroll
        for (int r2 = 0; r2 < RB; ++r2)
#pragma unroll
            for (int c2 = 0; c2 < CBW; ++c2)
#pragma unroll
                for (int i = 0; i < 16; ++i) acc[k][r2][c2][i] = 0.0f;
    // the epilogue's per-column coefficients and the step coefficient are
    // loaded before the k loop, so their latency hides behind it
    float cfs[CBW][M];
    auto load_cfs = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int c2 = 0; c2 < CBW; ++c2)
#pragma unroll
            for (int k = 0; k < M; ++k)
                cfs[c2][k] = k < m ? j.coef[(size_t)(col0 + wc * 32 * CBW + c2 * 32 + lr) * m + k] : 0.0f;
    };
    if constexpr (CBW == 2) load_cfs();
    const float kt = j.kt_tab[t];
    // PF: the epilogue's x and y (128 / CPI float4 each per thread, the
    // phase-2 mapping below) are loaded into registers once the last chunk's
    // copies are issued, so their HBM latency overlaps the final chunks' MFMAs
    const size_t Np = (size_t)j.Np;
    const int tr = (threadIdx.x & 31) * 4;
    // native vectors: arrays of HIP's float4 struct are not promoted to registers
    constexpr int NPF = PF ? 2 * (TW / CPI) : 0;
    EpiPrefetch<NPF> pf;
    pf.px = x_in;
    pf.py = j.y;
    pf.off0 = (size_t)(col0 + (threadIdx.x >> 5)) * Np + row0 + tr;
    pf.stride = CPI * Np;
    constexpr int CB = CBW == 2 ? staged_chunk<M>() : wide_chunk<PREC, M>();
    mma_tile_dma<PREC, M, NPF, NW, CB, CBW>(j.J, phi_in, j.Np, m, row0, col0, wr, wc, half, lr, acc, lds, pf);
    if constexpr (CBW != 2) load_cfs();

    // Epilogue in two phases.  (1) h = sum_k coef_k(col) H_k(row, col) from the
    // accumulators (same k order as the register-tile kernel) into an LDS tile
    // hs[col][row] (pitch 132 floats: conflict-free 16-byte writes).  (2) The
    // update: thread t takes rows 4 (t mod 32) .. +3 of columns t / 32 + CPI i,
    // so 32 lanes read and write one 512-byte segment of a column of x, y and phi.
    float *hs = (float *)lds;
    __syncthreads();
#pragma unroll
    for (int c2 = 0; c2 < CBW; ++c2) {
        const int cl = wc * 32 * CBW + c2 * 32 + lr;
        const float *cf = cfs[c2];
#pragma unroll
        for (int r2 = 0; r2 < RB; ++r2)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                float hv[4];
#pragma unroll
                for (int ii = 0; ii < 4; ++ii) {
                    float h = 0.0f;
#pragma unroll
                    for (int k = 0; k < M; ++k)
                        if (k < m) h = fmaf(cf[k], acc[k][r2][c2][g * 4 + ii], h);
                    hv[ii] = h;
                }
                *(float4 *)(hs + cl * kHsPitch + wr * 32 * RB + r2 * 32 + acc_row(half, g * 4)) =
                    make_float4(hv[0], hv[1], hv[2], hv[3]);
            }
    }
    __syncthreads();

    // One 4-spin segment of the update: y += kt x + h (+ dt alpha eta), x +=
    // dt a0 y, the wall, then x, y, phi and the trace written back.
    auto update = [&](int it, f32x4 xv, f32x4 yv, auto noise_tag) __attribute__((always_inline)) {
        constexpr bool NOISE = decltype(noise_tag)::value;
        const int cl = it * CPI + (threadIdx.x >> 5);
        const int col = col0 + cl, row = row0 + tr;
        const size_t off = (size_t)col * Np + row;
        const float4 hv4 = *(const float4 *)(hs + cl * kHsPitch + tr);
        float hv[4] = {hv4.x, hv4.y, hv4.z, hv4.w};
        float xs[4] = {xv.x, xv.y, xv.z, xv.w}, ys[4] = {yv.x, yv.y, yv.z, yv.w};
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
            float yn = fmaf(kt, xs[ii], ys[ii]) + hv[ii];
            if (NOISE && col < j.cols && row + ii < j.N) {
                const uint64_t g = (uint64_t)col + j.offset;
                const uint64_t nidx = (g * (uint64_t)j.steps + (uint64_t)t) * (uint64_t)j.N + (uint64_t)(row + ii);
                yn = fmaf(j.dt_alpha, noise_value(j.seed, nidx), yn);
            }
            float xn = fmaf(j.dta0, yn, xs[ii]);
            wall(xn, yn);
            xs[ii] = xn;
            ys[ii] = yn;
        }
        *(float4 *)(x_out + off) = make_float4(xs[0], xs[1], xs[2], xs[3]);
        *(float4 *)(j.y + off) = make_float4(ys[0], ys[1], ys[2], ys[3]);
        if (DSB) {
            if constexpr (PREC == QAIA_FP32) {
                *(float4 *)((float *)phi_out + off) = make_float4(sgn1(xs[0]), sgn1(xs[1]), sgn1(xs[2]), sgn1(xs[3]));
            } else if constexpr (PREC == QAIA_BF16) {
                uint2 v;
                v.x = (uint32_t)bf16_pm1(xs[0]) | ((uint32_t)bf16_pm1(xs[1]) << 16);
                v.y = (uint32_t)bf16_pm1(xs[2]) | ((uint32_t)bf16_pm1(xs[3]) << 16);
                *(uint2 *)((uint16_t *)phi_out + off) = v;
            } else {
                uint32_t v = (uint32_t)fp8_pm1(xs[0]) | ((uint32_t)fp8_pm1(xs[1]) << 8) |
                             ((uint32_t)fp8_pm1(xs[2]) << 16) | ((uint32_t)fp8_pm1(xs[3]) << 24);
                *(uint32_t *)((uint8_t *)phi_out + off) = v;
            }
        }
        if (j.trace != nullptr && t < j.trace_steps && col < j.cols) {
#pragma unroll
            for (int ii = 0; ii < 4; ++ii)
                if (row + ii < j.N) j.trace[((size_t)col * j.trace_steps + t) * j.N + row + ii] = xs[ii];
        }
    };
    auto load = [&](const float *base, int it) __attribute__((always_inline)) {
        return *(const f32x4 *)(base + (size_t)(col0 + it * CPI + (threadIdx.x >> 5)) * Np + row0 + tr);
    };
    if (j.dt_alpha == 0.0f) {
        // plain SB: fully unrolled, so the registers are indexed statically
        if constexpr (PF) {
#pragma unroll
            for (int it = 0; it < TW / CPI; ++it) update(it, pf.xpf[it], pf.ypf[it], std::false_type{});
        } else {
            // every x and y of the update is loaded before the first store: as
            // far as the compiler can tell a store may alias a later load, so
            // it kept each iteration's loads behind the previous stores, one
            // memory round trip per iteration (the accumulators are dead here,
            // the registers free).  The step gained only 0.5 %: with every CU
            // in its epilogue at once, HBM bandwidth bounds this phase.
            f32x4 xl[TW / CPI], yl[TW / CPI];
#pragma unroll
            for (int it = 0; it < TW / CPI; ++it) {
                xl[it] = load(x_in, it);
                yl[it] = load(j.y, it);
            }
#pragma unroll
            for (int it = 0; it < TW / CPI; ++it) update(it, xl[it], yl[it], std::false_type{});
        }
    } else {
        // noise injection (Eq. 10): the Gaussian draw makes the body too large to
        // unroll; x and y are read again here
        for (int it = 0; it < TW / CPI; ++it) update(it, load(x_in, it), load(j.y, it), std::true_type{});
    }
}

// the stage ring, reused after the k loop for the 128 x 132 float h tile
template <int PREC, int MT, int CBW = 2>
constexpr size_t staged_lds_bytes() {
    constexpr int CB = CBW == 2 ? staged_chunk<MT>() : wide_chunk<PREC, MT>();
    constexpr size_t ring = (size_t)wide_stages<MT, CB, CBW>() * (MT * kT2 + 64 * CBW) * CB;
    constexpr size_t hsb = sizeof(float) * 64 * CBW * kHsPitch;
    return ring > hsb ? ring : hsb;
}

// XCD-aware tile order for a single job: blocks are dealt to the eight XCDs
// round robin (block b runs on XCD b % 8).  When the row-tile count divides by
// 8 and the column-tile count is even, XCD x owns a quarter of the row tiles
// (group x & 3) times half of the column tiles (group x >> 2), and its
// consecutive blocks sweep the group's row tiles first: with 16 row tiles its
// 32 CUs hold 4 x 8 patches, so each J and phi chunk they copy serves 8 or 4
// blocks from its own L2 (about 2 % faster in BF16 and FP8 than giving each
// XCD whole row tiles across all columns, which is the order used when the
// column-tile count is odd).
__device__ __forceinline__ void xcd_tile(int tiles_x, int tiles_y, int &bx, int &by) {
    const int b = blockIdx.y * gridDim.x + blockIdx.x;
    if ((tiles_y & 7) != 0) {
        bx = blockIdx.x;
        by = blockIdx.y;
        return;
    }
    const int xcd = b & 7, slot = b >> 3;
    if ((tiles_x & 1) == 0) {
        const int RG = tiles_y >> 2, CG = tiles_x >> 1;
        by = (xcd & 3) * RG + slot % RG;
        bx = (xcd >> 2) * CG + slot / RG;
        return;
    }
    by = xcd * (tiles_y >> 3) + slot / tiles_x;
    bx = slot % tiles_x;
}

template <int PREC, int M, bool DSB, int NW, int CBW = 2>
__global__ __launch_bounds__(64 * NW) void dense_step_staged_kernel(DenseJob j, int t) {
    __shared__ __attribute__((aligned(16))) char lds[staged_lds_bytes<PREC, M, CBW>()];
    int bx, by;
    xcd_tile(j.tiles_x / (CBW / 2), j.tiles_y, bx, by);
    dense_step_staged_body<PREC, M, DSB, true, CBW == 2 && staged_prefetch<PREC, M, NW>(false), NW, CBW>(j, t, bx, by,
                                                                                                     lds);
}

// XCD-aware order inside one job of a grouped launch (its first block index
// is a multiple of 8, so local & 7 is the XCD): with 8 | tiles, each XCD takes
// a contiguous eighth of the row tiles, or else of the column tiles.
__device__ __forceinline__ void xcd_tile_local(int64_t local, int tiles_x, int tiles_y, int &bx, int &by) {
    const int64_t T = (int64_t)tiles_x * tiles_y;
    if ((T & 7) == 0) {
        const int xcd = (int)(local & 7);
        const int64_t slot = local >> 3;
        if ((tiles_y & 7) == 0) {
            by = xcd * (tiles_y >> 3) + (int)(slot / tiles_x);
            bx = (int)(slot % tiles_x);
            return;
        }
        if ((tiles_x & 7) == 0) {
            const int cx = tiles_x >> 3;
            bx = xcd * cx + (int)(slot % cx);
            by = (int)(slot / cx);
            return;
        }
    }
    bx = (int)(local % tiles_x);
    by = (int)(local / tiles_x);
}

// Grouped staged step over jobs that share m = MT; job i owns blocks
// [block_start[i], block_start[i + 1]) (padded to a multiple of 8; blocks past
// its tiles exit at once).
template <int PREC, int MT, bool DSB, int NW>
__global__ __launch_bounds__(64 * NW) void dense_batch_step_staged_kernel(const DenseJob *__restrict__ jobs,
                                                                          int count,
                                                                          const int64_t *__restrict__ block_start,
                                                                          int t) {
    __shared__ __attribute__((aligned(16))) char lds[staged_lds_bytes<PREC, MT>()];
    const int64_t b = blockIdx.x;
    int i = 0;
    while (i + 1 < count && block_start[i + 1] <= b) ++i;
    const DenseJob j = jobs[i];
    const int64_t local = b - block_start[i];
    if (local >= (int64_t)j.tiles_x * j.tiles_y) return;
    int bx, by;
    xcd_tile_local(local, j.tiles_x, j.tiles_y, bx, by);
    dense_step_staged_body<PREC, MT, DSB, true, staged_prefetch<PREC, MT, NW>(true), NW>(j, t, bx, by, lds);
}

// Field mode (reduced-precision error reporting): field[col][k][i] = 2^e_k (J~_k Phi)_i.
struct FieldArgs {
    const void *J;
    const void *phi;
    int Np, N, cols;
    float *field;
    const float *jscale;
};

template <int PREC, int M>
__global__ __launch_bounds__(kDB) void dense_field_kernel(FieldArgs a) {
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int half = l >> 5, lr = l & 31;
    const int row_w = blockIdx.y * kTileM + (wv & 1) * 32;
    const int col_w = blockIdx.x * kTileN + (wv >> 1) * 64;
    f16v acc[M][2];
#pragma unroll
    for (int k = 0; k < M; ++k)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[k][cb][i] = 0.0f;
    mma_tile<PREC, M>(a.J, a.phi, a.Np, M, row_w, col_w, half, lr, acc);
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        const int col = col_w + cb * 32 + lr;
        if (col >= a.cols) continue;
#pragma unroll
        for (int k = 0; k < M; ++k)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int row = row_w + acc_row(half, i);
                if (row < a.N)
                    a.field[((size_t)col * M + k) * a.N + row] = acc[k][cb][i] * a.jscale[k];
            }
    }
}

// ---------------------------------------------------------------------------
// set-up, coefficient and read-out kernels

template <int PREC>
__global__ void dense_init_kernel(float *x, float *y, void *phi, int Np, int N, int cols, int colsP,
                                  uint64_t seed, uint64_t offset, float amp, bool dsb) {
    const size_t idx = (size_t)blockIdx.x * kDB + threadIdx.x;
    if (idx >= (size_t)colsP * Np) return;
    const int col = (int)(idx / Np), i = (int)(idx % Np);
    float xv = 0.0f, yv = 0.0f;
    const bool live = col < cols && i < N;
    if (live) {
        const uint64_t g = (uint64_t)col + offset;
        xv = init_value(seed, init_counter(g, N, i, 0), amp);
        yv = init_value(seed, init_counter(g, N, i, 1), amp);
    }
    x[idx] = xv;
    y[idx] = yv;
    if (dsb) {
        if constexpr (PREC == QAIA_FP32) ((float *)phi)[idx] = live ? sgn1(xv) : 0.0f;
        else if constexpr (PREC == QAIA_BF16) ((uint16_t *)phi)[idx] = live ? bf16_pm1(xv) : 0;
        else ((uint8_t *)phi)[idx] = live ? fp8_pm1(xv) : 0;
    }
}

__global__ void dense_coef_kernel(const float *weights, const double *c0s, int m, int R, int cols,
                                  int colsP, double dt, const float *jscale, float *coef) {
    const int idx = blockIdx.x * kDB + threadIdx.x;
    if (idx >= colsP * m) return;
    const int col = idx / m, k = idx % m;
    float v = 0.0f;
    if (col < cols) {
        const int w = col / R;
        const double c0 = c0s[w];
        if (c0 >= 0.0) v = (float)(-dt * c0 * (double)weights[(size_t)w * m + k] * (double)jscale[k]);
    }
    coef[idx] = v;
}

// Phi for the field hook: float input [count][N] -> padded operand [colsP][Np].
template <int PREC>
__global__ void dense_phi_kernel(const float *in, void *phi, int Np, int N, int count, int colsP) {
    const size_t idx = (size_t)blockIdx.x * kDB + threadIdx.x;
    if (idx >= (size_t)colsP * Np) return;
    const int col = (int)(idx / Np), i = (int)(idx % Np);
    const float v = (col < count && i < N) ? in[(size_t)col * N + i] : 0.0f;
    if constexpr (PREC == QAIA_FP32) ((float *)phi)[idx] = v;
    else if constexpr (PREC == QAIA_BF16) ((uint16_t *)phi)[idx] = v == 0.0f ? 0 : bf16_pm1(v);
    else ((uint8_t *)phi)[idx] = v == 0.0f ? 0 : fp8_pm1(v);
}

// one wave per (column, 64-spin word): ballot of x < 0
__global__ void dense_readout_kernel(const float *x, int Np, int N, int cols, int R, int words,
                                     const double *c0s, uint64_t *spins) {
    const int lane = threadIdx.x & 63;
    const size_t item = (size_t)blockIdx.x * (kDB / 64) + (threadIdx.x >> 6);
    if (item >= (size_t)cols * words) return;
    const int col = (int)(item / words), wd = (int)(item % words);
    const int i = wd * 64 + lane;
    const bool neg = i < N && x[(size_t)col * Np + i] < 0.0f;
    const uint64_t bits = __ballot(neg);
    if (lane == 0) spins[(size_t)col * words + wd] = c0s[col / R] >= 0.0 ? bits : 0ull;
}

// ---------------------------------------------------------------------------
// host side

static uint16_t to_bf16(double v) {
    float f = (float)v;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round half to even (finite inputs)
    return (uint16_t)(u >> 16);
}

// OCP e4m3 (bias 7, no infinities, max 448), round half to even, saturating.
static uint8_t to_e4m3(double v) {
    uint8_t s = v < 0 ? 0x80 : 0;
    double a = std::fabs(v);
    if (a == 0.0) return 0;
    if (a >= 448.0) return s | 0x7E;
    int e;
    std::frexp(a, &e);  // a = f * 2^e, f in [0.5, 1)
    e -= 1;             // a = (1 + m) 2^e
    if (e < -6) {       // subnormal: quantum 2^-9
        double q = std::nearbyint(a * 512.0);
        if (q >= 8.0) return s | 0x08;
        return s | (uint8_t)q;
    }
    double q = std::nearbyint((a / std::ldexp(1.0, e) - 1.0) * 8.0);
    if (q >= 8.0) {
        q = 0.0;
        ++e;
    }
    if (e > 8 || (e == 8 && q > 6.0)) return s | 0x7E;
    return s | (uint8_t)(((e + 7) << 3) | (int)q);
}

void dense_build(Problem &p) {
    if (p.m > 4) {  // the dense kernels hold at most four objective tiles
        p.dense.why = "the dense path supports m <= 4";
        return;
    }
    const int64_t Np = (p.n + 127) / 128 * 128;  // both tile heights (64, 128) divide it
    const double bytes = (double)p.m * Np * Np * 7.0;
    if (bytes > 4.0 * (1ull << 30)) {
        p.dense.why = "dense images would exceed 4 GiB";
        return;
    }
    DenseImages &d = p.dense;
    d.Np = (int32_t)Np;
    const size_t per = (size_t)Np * Np, all = per * p.m;
    std::vector<float> j32(all, 0.0f);
    std::vector<uint16_t> j16(all, 0);
    std::vector<uint8_t> j8(all, 0);
    for (int k = 0; k < p.m; ++k) {
        int64_t mx = 0;
        for (int64_t e = 0; e < p.E; ++e) mx = std::max<int64_t>(mx, std::llabs((long long)p.W[(size_t)k * p.E + e]));
        // bf16: largest magnitude in [128, 256); e4m3: largest magnitude <= 448
        int e16 = 0, e8 = 0;
        if (mx > 0) {
            e16 = (int)std::floor(std::log2((double)mx)) - 7;
            e8 = (int)std::ceil(std::log2((double)mx / 448.0));
            while ((double)mx * std::ldexp(1.0, -e8) > 448.0) ++e8;
        }
        d.scale16[k] = (float)std::ldexp(1.0, e16);
        d.scale8[k] = (float)std::ldexp(1.0, e8);
        for (int64_t e = 0; e < p.E; ++e) {
            const double w = (double)p.W[(size_t)k * p.E + e];
            const size_t a = per * k + (size_t)p.eu[e] * Np + p.ev[e];
            const size_t b = per * k + (size_t)p.ev[e] * Np + p.eu[e];
            j32[a] = j32[b] = (float)w;
            j16[a] = j16[b] = to_bf16(w * std::ldexp(1.0, -e16));
            j8[a] = j8[b] = to_e4m3(w * std::ldexp(1.0, -e8));
        }
    }
    auto up = [](const void *src, size_t bytes) {
        void *dst = nullptr;
        hipError_t e = hipMalloc(&dst, bytes);
        if (e == hipErrorOutOfMemory) throw Error{QAIA_OUT_OF_MEMORY, "device allocation failed"};
        QAIA_HIP(e);
        QAIA_HIP(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
        return dst;
    };
    DeviceGuard g(p.device);
    d.J32 = (float *)up(j32.data(), all * 4);
    d.J16 = (uint16_t *)up(j16.data(), all * 2);
    d.J8 = (uint8_t *)up(j8.data(), all);
    std::vector<float> sc(3 * 8, 1.0f);
    for (int k = 0; k < p.m; ++k) {
        sc[8 + k] = d.scale16[k];
        sc[16 + k] = d.scale8[k];
    }
    d.scales = (float *)up(sc.data(), sc.size() * 4);
    d.ok = true;
}

void dense_release(Problem &p) {
    DeviceGuard g(p.device);
    for (void *ptr : {(void *)p.dense.J32, (void *)p.dense.J16, (void *)p.dense.J8, (void *)p.dense.scales})
        if (ptr) (void)hipFree(ptr);
}

static const void *dense_J(const Problem &p, int prec) {
    return prec == QAIA_FP32 ? (const void *)p.dense.J32
                             : (prec == QAIA_BF16 ? (const void *)p.dense.J16 : (const void *)p.dense.J8);
}
static size_t elem_bytes(int prec) { return prec == QAIA_FP32 ? 4 : (prec == QAIA_BF16 ? 2 : 1); }

void dense_ws_extend(const Problem &p, int64_t W, int32_t R, const qaia_schedule &s, WsLayout &L) {
    const size_t cols = (size_t)W * R;
    const size_t colsP = (cols + kTileN - 1) / kTileN * kTileN;
    const size_t Np = (size_t)p.dense.Np;
    size_t off = L.total;
    auto take = [&](size_t b) {
        size_t o = off;
        off += align256(b);
        return o;
    };
    L.colsP = (int64_t)colsP;
    L.xa = take(4 * colsP * Np);
    L.xb = s.variant == QAIA_BSB ? take(4 * colsP * Np) : L.xa;
    L.y = take(4 * colsP * Np);
    const size_t pb = elem_bytes(s.precision) * colsP * Np;
    L.pa = s.variant == QAIA_DSB ? take(pb) : L.xa;
    L.pb = s.variant == QAIA_DSB ? take(pb) : L.xb;
    L.coef = take(4 * colsP * (size_t)p.m);
    L.total = off;
}

bool dense_supported(const Problem &p, std::string *why) {
    if (!p.dense.ok) {
        if (why) *why = p.dense.why.empty() ? "dense images not built" : p.dense.why;
        return false;
    }
    return true;
}

template <int PREC, int M, bool DSB>
static void step_launch(dim3 grid, hipStream_t st, const DenseJob &j, int t) {
    hipLaunchKernelGGL((dense_step_kernel<PREC, M, DSB>), grid, dim3(kDB), 0, st, j, t);
}

template <int PREC, bool DSB>
static void step_dispatch_m(dim3 grid, hipStream_t st, const DenseJob &j, int t) {
    switch (j.m) {
        case 1: step_launch<PREC, 1, DSB>(grid, st, j, t); break;
        case 2: step_launch<PREC, 2, DSB>(grid, st, j, t); break;
        case 3: step_launch<PREC, 3, DSB>(grid, st, j, t); break;
        case 4: step_launch<PREC, 4, DSB>(grid, st, j, t); break;
        default: throw Error{QAIA_UNSUPPORTED, "dense path supports m <= 4"};
    }
}

// Waves per staged block: eight (two per SIMD, 32 x 64 wave tiles) for the
// BF16 and FP8 operands, whose MFMAs are short beside the operand copies and
// whose second wave per SIMD hides copy and barrier waits (C3 shape: BF16
// 112.5 -> 106.9 us, FP8 73.7 -> 63.6 us per step); four for FP32 (64 x 64
// wave tiles), where eight measured 2-6 % slower.
template <int PREC>
constexpr int staged_waves() { return PREC == QAIA_FP32 ? 4 : 8; }

// BF16 single-job launches with m = 2 or 3, and FP8 ones with m = 3, take the
// wide tile (128 x 256: 37.5 % fewer operand bytes per flop for m = 3, 25 %
// for m = 2) when the columns fill 256-column tiles and those tiles still
// cover every CU (complete N = 2048, 4096 columns: BF16 m = 3 106.1 ->
// 95.3-96.0 us per step, m = 2 82.6 -> 77.9-78.3; FP8 m = 3 63.8-64.1 ->
// 62.5-62.7, its 64-byte chunks one k-group each, so a unit is half of the
// wave's column blocks; m = 1 gains nothing; at N = 1024, 2048 columns the
// 64 wide tiles would leave most CUs idle: 42.3 against 28.5 us).
template <int PREC, int M>
constexpr bool staged_wide() { return (PREC == QAIA_BF16 && (M == 2 || M == 3)) || (PREC == QAIA_FP8 && M == 3); }

static int device_cus() {
    static std::atomic<int> cache[64];
    int dev = 0;
    QAIA_HIP(hipGetDevice(&dev));
    if (dev >= 0 && dev < 64) {
        const int v = cache[dev].load(std::memory_order_relaxed);
        if (v > 0) return v;
    }
    int cus = 0;
    QAIA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (dev >= 0 && dev < 64) cache[dev].store(cus, std::memory_order_relaxed);
    return cus;
}

template <int PREC, int M, bool DSB>
static void staged_launch(dim3 grid, hipStream_t st, const DenseJob &j, int t) {
    constexpr int NW = staged_waves<PREC>();
    if constexpr (staged_wide<PREC, M>()) {
        if ((j.tiles_x % 2) == 0 && (int64_t)(j.tiles_x / 2) * j.tiles_y >= device_cus()) {
            hipLaunchKernelGGL((dense_step_staged_kernel<PREC, M, DSB, NW, 4>), dim3(grid.x / 2, grid.y), dim3(64 * NW),
                               0, st, j, t);
            return;
        }
    }
    hipLaunchKernelGGL((dense_step_staged_kernel<PREC, M, DSB, NW>), grid, dim3(64 * NW), 0, st, j, t);
}

template <int PREC, bool DSB>
static void staged_dispatch_m(dim3 grid, hipStream_t st, const DenseJob &j, int t) {
    switch (j.m) {
        case 1: staged_launch<PREC, 1, DSB>(grid, st, j, t); break;
        case 2: staged_launch<PREC, 2, DSB>(grid, st, j, t); break;
        case 3: staged_launch<PREC, 3, DSB>(grid, st, j, t); break;
        case 4: staged_launch<PREC, 4, DSB>(grid, st, j, t); break;
        default: throw Error{QAIA_UNSUPPORTED, "dense path supports m <= 4"};
    }
}

static void step_dispatch(int prec, bool dsb, dim3 grid, hipStream_t st, const DenseJob &j, int t) {
    if (j.staged) {
        if (prec == QAIA_FP32) {
            if (dsb) staged_dispatch_m<QAIA_FP32, true>(grid, st, j, t);
            else staged_dispatch_m<QAIA_FP32, false>(grid, st, j, t);
        } else if (prec == QAIA_BF16) {
            staged_dispatch_m<QAIA_BF16, true>(grid, st, j, t);
        } else {
            staged_dispatch_m<QAIA_FP8, true>(grid, st, j, t);
        }
        return;
    }
    if (prec == QAIA_FP32) {
        if (dsb) step_dispatch_m<QAIA_FP32, true>(grid, st, j, t);
        else step_dispatch_m<QAIA_FP32, false>(grid, st, j, t);
    } else if (prec == QAIA_BF16) {
        step_dispatch_m<QAIA_BF16, true>(grid, st, j, t);
    } else {
        step_dispatch_m<QAIA_FP8, true>(grid, st, j, t);
    }
}

template <int PREC, bool DSB>
static void staged_batch_launch(int mt, dim3 grid, hipStream_t st, const DenseJob *jobs, int count,
                                const int64_t *starts, int t) {
    constexpr int NW = staged_waves<PREC>();
    switch (mt) {
        case 1: hipLaunchKernelGGL((dense_batch_step_staged_kernel<PREC, 1, DSB, NW>), grid, dim3(64 * NW), 0, st, jobs, count, starts, t); break;
        case 2: hipLaunchKernelGGL((dense_batch_step_staged_kernel<PREC, 2, DSB, NW>), grid, dim3(64 * NW), 0, st, jobs, count, starts, t); break;
        case 3: hipLaunchKernelGGL((dense_batch_step_staged_kernel<PREC, 3, DSB, NW>), grid, dim3(64 * NW), 0, st, jobs, count, starts, t); break;
        case 4: hipLaunchKernelGGL((dense_batch_step_staged_kernel<PREC, 4, DSB, NW>), grid, dim3(64 * NW), 0, st, jobs, count, starts, t); break;
        default: throw Error{QAIA_UNSUPPORTED, "dense path supports m <= 4"};
    }
}

void launch_dense_batch_step(int prec, bool dsb, bool staged, int mt, const DenseJob *jobs, int count,
                             const int64_t *starts, int64_t blocks, int t, hipStream_t st) {
    QAIA_CHECK(blocks <= INT32_MAX, QAIA_INVALID_ARGUMENT, "too many tiles for one launch");
    if (blocks == 0) return;
    const dim3 grid((unsigned)blocks);
    if (staged) {
        if (prec == QAIA_FP32) {
            if (dsb) staged_batch_launch<QAIA_FP32, true>(mt, grid, st, jobs, count, starts, t);
            else staged_batch_launch<QAIA_FP32, false>(mt, grid, st, jobs, count, starts, t);
        } else if (prec == QAIA_BF16) {
            staged_batch_launch<QAIA_BF16, true>(mt, grid, st, jobs, count, starts, t);
        } else {
            staged_batch_launch<QAIA_FP8, true>(mt, grid, st, jobs, count, starts, t);
        }
        return;
    }
    if (prec == QAIA_FP32) {
        if (dsb) hipLaunchKernelGGL((dense_batch_step_kernel<QAIA_FP32, true>), grid, dim3(kDB), 0, st, jobs, count, starts, t);
        else hipLaunchKernelGGL((dense_batch_step_kernel<QAIA_FP32, false>), grid, dim3(kDB), 0, st, jobs, count, starts, t);
    } else if (prec == QAIA_BF16) {
        hipLaunchKernelGGL((dense_batch_step_kernel<QAIA_BF16, true>), grid, dim3(kDB), 0, st, jobs, count, starts, t);
    } else {
        hipLaunchKernelGGL((dense_batch_step_kernel<QAIA_FP8, true>), grid, dim3(kDB), 0, st, jobs, count, starts, t);
    }
}

DenseJob dense_job(const Problem &p, int64_t W, int32_t R, const qaia_schedule &s, void *ws, const WsLayout &L,
                   float *trace, int32_t trace_steps, bool staged) {
    char *b = (char *)ws;
    DenseJob j{};
    j.J = dense_J(p, s.precision);
    j.xa = (float *)(b + L.xa);
    j.xb = (float *)(b + L.xb);
    j.y = (float *)(b + L.y);
    j.pa = b + L.pa;
    j.pb = b + L.pb;
    j.coef = (const float *)(b + L.coef);
    j.kt_tab = (const float *)(b + L.kt);
    j.dta0 = s.dt * s.a0;
    j.Np = p.dense.Np;
    j.N = p.n;
    j.m = p.m;
    j.cols = (int)(W * (int64_t)R);
    j.staged = staged ? 1 : 0;
    j.tiles_x = (int)(L.colsP / (staged ? kT2 : kTileN));
    j.tiles_y = p.dense.Np / (staged ? kT2 : kTileM);
    j.trace = trace_steps > 0 ? trace : nullptr;
    j.trace_steps = trace_steps;
    j.dt_alpha = s.dt * s.noise_alpha;
    j.steps = s.steps;
    j.seed = s.seed;
    j.offset = s.replica_offset;
    return j;
}

// x, y, Phi start values and the per-column coefficients
void launch_dense_setup(const Problem &p, const float *weights, int32_t R, const qaia_schedule &s, void *ws,
                        const WsLayout &L, const DenseJob &j, hipStream_t st) {
    char *b = (char *)ws;
    const int prec = s.precision;
    const bool dsb = s.variant == QAIA_DSB;
    const int colsP = (int)L.colsP, Np = j.Np;
    const size_t total = (size_t)colsP * Np;
    const unsigned ib = (unsigned)((total + kDB - 1) / kDB);
    if (prec == QAIA_FP32)
        hipLaunchKernelGGL(dense_init_kernel<QAIA_FP32>, dim3(ib), dim3(kDB), 0, st, j.xa, j.y, j.pa, Np, p.n,
                           j.cols, colsP, s.seed, s.replica_offset, s.init_amp, dsb);
    else if (prec == QAIA_BF16)
        hipLaunchKernelGGL(dense_init_kernel<QAIA_BF16>, dim3(ib), dim3(kDB), 0, st, j.xa, j.y, j.pa, Np, p.n,
                           j.cols, colsP, s.seed, s.replica_offset, s.init_amp, dsb);
    else
        hipLaunchKernelGGL(dense_init_kernel<QAIA_FP8>, dim3(ib), dim3(kDB), 0, st, j.xa, j.y, j.pa, Np, p.n,
                           j.cols, colsP, s.seed, s.replica_offset, s.init_amp, dsb);
    QAIA_HIP(hipGetLastError());
    const unsigned cb = (unsigned)((colsP * p.m + kDB - 1) / kDB);
    hipLaunchKernelGGL(dense_coef_kernel, dim3(cb), dim3(kDB), 0, st, weights, (const double *)(b + L.c0s), p.m,
                       R, j.cols, colsP, (double)s.dt, p.dense.scales + 8 * prec, (float *)(b + L.coef));
    QAIA_HIP(hipGetLastError());
}

// sgn read-out of the final x and exact cut values
void launch_dense_finish(const Problem &p, int32_t R, const qaia_schedule &s, void *ws, const WsLayout &L,
                         const DenseJob &j, uint64_t *spins, int64_t *obj, hipStream_t st) {
    char *b = (char *)ws;
    const bool dsb = s.variant == QAIA_DSB;
    // after T steps the latest x is xa (discrete SB, in place) or the buffer step T-1 wrote
    const float *xf = dsb ? j.xa : ((s.steps & 1) ? j.xb : j.xa);
    const size_t items = (size_t)j.cols * p.words;
    hipLaunchKernelGGL(dense_readout_kernel, dim3((unsigned)((items + 3) / 4)), dim3(kDB), 0, st, xf, j.Np, p.n,
                       j.cols, R, p.words, (const double *)(b + L.c0s), spins);
    QAIA_HIP(hipGetLastError());
    launch_evaluate(p, spins, j.cols, obj, st);
}

void launch_dense(const Problem &p, const float *weights, int64_t W, int32_t R,
                  const qaia_schedule &s, void *ws, const WsLayout &L, uint64_t *spins, int64_t *obj,
                  float *trace, int32_t trace_steps, bool staged, hipStream_t st) {
    std::string why;
    QAIA_CHECK(dense_supported(p, &why), QAIA_UNSUPPORTED, "dense path: " + why);
    QAIA_CHECK(p.m <= 4, QAIA_UNSUPPORTED, "dense path supports m <= 4");
    const int64_t cols = W * (int64_t)R;
    if (cols == 0) return;
    QAIA_CHECK(L.colsP <= INT32_MAX / 2, QAIA_INVALID_ARGUMENT, "too many replicas for the dense path");
    const DenseJob j = dense_job(p, W, R, s, ws, L, trace, trace_steps, staged);
    launch_dense_setup(p, weights, R, s, ws, L, j, st);
    const dim3 grid(j.tiles_x, j.tiles_y);
    for (int t = 0; t < s.steps; ++t) step_dispatch(s.precision, s.variant == QAIA_DSB, grid, st, j, t);
    QAIA_HIP(hipGetLastError());
    launch_dense_finish(p, R, s, ws, L, j, spins, obj, st);
}

// ---------------------------------------------------------------------------
// field hook

size_t dense_field_ws_bytes(const Problem &p, int prec, int64_t count) {
    const size_t colsP = (size_t)(count + kTileN - 1) / kTileN * kTileN;
    return align256(elem_bytes(prec) * colsP * (size_t)std::max(p.dense.Np, 64));
}

template <int PREC, int M>
static void field_launch(dim3 grid, hipStream_t st, const FieldArgs &a) {
    hipLaunchKernelGGL((dense_field_kernel<PREC, M>), grid, dim3(kDB), 0, st, a);
}

template <int PREC>
static void field_dispatch(int m, dim3 grid, hipStream_t st, const FieldArgs &a) {
    switch (m) {
        case 1: field_launch<PREC, 1>(grid, st, a); break;
        case 2: field_launch<PREC, 2>(grid, st, a); break;
        case 3: field_launch<PREC, 3>(grid, st, a); break;
        case 4: field_launch<PREC, 4>(grid, st, a); break;
        default: throw Error{QAIA_UNSUPPORTED, "dense path supports m <= 4"};
    }
}

void launch_dense_field(const Problem &p, int prec, const float *phi, int64_t count, float *field,
                        void *ws, size_t ws_bytes, hipStream_t st) {
    std::string why;
    QAIA_CHECK(dense_supported(p, &why), QAIA_UNSUPPORTED, "dense path: " + why);
    QAIA_CHECK(p.m <= 4, QAIA_UNSUPPORTED, "dense path supports m <= 4");
    QAIA_CHECK(ws_bytes >= dense_field_ws_bytes(p, prec, count), QAIA_WORKSPACE_TOO_SMALL,
               "field workspace too small");
    if (count == 0) return;
    const int Np = p.dense.Np;
    const int colsP = (int)((count + kTileN - 1) / kTileN * kTileN);
    const size_t total = (size_t)colsP * Np;
    const unsigned ib = (unsigned)((total + kDB - 1) / kDB);
    if (prec == QAIA_FP32)
        hipLaunchKernelGGL(dense_phi_kernel<QAIA_FP32>, dim3(ib), dim3(kDB), 0, st, phi, ws, Np, p.n, (int)count, colsP);
    else if (prec == QAIA_BF16)
        hipLaunchKernelGGL(dense_phi_kernel<QAIA_BF16>, dim3(ib), dim3(kDB), 0, st, phi, ws, Np, p.n, (int)count, colsP);
    else
        hipLaunchKernelGGL(dense_phi_kernel<QAIA_FP8>, dim3(ib), dim3(kDB), 0, st, phi, ws, Np, p.n, (int)count, colsP);
    QAIA_HIP(hipGetLastError());
    FieldArgs a{};
    a.J = dense_J(p, prec);
    a.phi = ws;
    a.Np = Np;
    a.N = p.n;
    a.cols = (int)count;
    a.field = field;
    a.jscale = p.dense.scales + 8 * prec;
    const dim3 grid(colsP / kTileN, Np / kTileM);
    if (prec == QAIA_FP32) field_dispatch<QAIA_FP32>(p.m, grid, st, a);
    else if (prec == QAIA_BF16) field_dispatch<QAIA_BF16>(p.m, grid, st, a);
    else field_dispatch<QAIA_FP8>(p.m, grid, st, a);
    QAIA_HIP(hipGetLastError());
}

}  // namespace qaia
