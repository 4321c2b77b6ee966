// Measurement kernels: the machine's own issue and bandwidth ceilings, so
// that roofline fractions can be stated against measured peaks beside the
// datasheet figures.  Every kernel computes a closed-form result, which the
// tests check exactly.
//
//   fma_peak_kernel  : eight independent fp32 FMA chains per lane
//                      (x <- x * a + b), plain VALU FMAs (packed FP32 is
//                      disabled for every device compile of this library).
//   mfma_peak_kernel : four independent 32x32 accumulators per wave, operands
//                      all 1.0 in the instruction's format (fp32 32x32x2,
//                      bf16 32x32x16, e4m3 32x32x64), back-to-back MFMAs.
//   copy_peak_kernel : 16 bytes per lane, grid-stride, nontemporal, HBM to HBM.
//   valu_mix_peak_kernel : the sparse SB update's instruction mix with full
//                      occupancy: per iteration 14 soft spins x, y per lane
//                      take 60 FMAs (own term, ring couplings, x update) and
//                      42 wall operations (compare, select, clamp), the
//                      10 : 7 ratio of the generated kernel's 180 FMAs and
//                      126 wall operations per replica-step on the 42-node
//                      48-edge graph.
#include "internal.hpp"

namespace qaia {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

constexpr int kPB = 256;     // threads per block
constexpr int kChains = 8;   // FMA chains per lane
constexpr int kAccs = 4;     // MFMA accumulators per wave

__global__ __launch_bounds__(kPB) void fma_peak_kernel(float a, float b, int iters, float *out) {
    const int64_t t = (int64_t)blockIdx.x * kPB + threadIdx.x;
    float x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = (float)((t + c) & 7);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) x[c] = __builtin_fmaf(x[c], a, b);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c];
    out[t] = s;
}

// PREC: 0 fp32, 1 bf16, 2 e4m3; `one` holds 1.0 in the operand format
// (fp32 bits, bf16 bits in the low half, e4m3 bits in the low byte).
template <int PREC>
__global__ __launch_bounds__(kPB) void mfma_peak_kernel(uint32_t one, int iters, float *out) {
    f16v acc[kAccs];
#pragma unroll
    for (int j = 0; j < kAccs; ++j)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[j][i] = 0.0f;
    if constexpr (PREC == QAIA_FP32) {
        const float a = __builtin_bit_cast(float, one);
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int j = 0; j < kAccs; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, a, acc[j], 0, 0, 0);
        }
    } else if constexpr (PREC == QAIA_BF16) {
        const short h = (short)(one & 0xFFFFu);
        const s16x8 bits = {h, h, h, h, h, h, h, h};
        const bf16x8 a = __builtin_bit_cast(bf16x8, bits);
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int j = 0; j < kAccs; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, a, acc[j], 0, 0, 0);
        }
    } else {
        const uint32_t q = (one & 0xFFu) * 0x01010101u;
        const int w = (int)q;
        const i32x8 a = {w, w, w, w, w, w, w, w};
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int j = 0; j < kAccs; ++j)
                acc[j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, a, acc[j], 0, 0, 0, 127, 0, 127);
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < kAccs; ++j) s += acc[j][0];
    out[(int64_t)blockIdx.x * kPB + threadIdx.x] = s;
}

constexpr int kMixSpins = 14;

// Per iteration and spin i: y_i += k x_i, y_i += k x_(i+-1) (ring), spins
// 0..3 also y_i += k x_(i+7), then x_i += k y_i and the wall (|x| > 1 zeroes
// y and clamps x).  With k = 0 every FMA returns its addend exactly and no
// spin reaches the wall (|x| <= 0.5), so the state never changes: the closed
// form is the sum of the start values.  k is a kernel argument, so the
// compiler cannot drop the work.
__global__ __launch_bounds__(kPB) void valu_mix_peak_kernel(float k, int iters, float *out) {
    const int64_t t = (int64_t)blockIdx.x * kPB + threadIdx.x;
    float x[kMixSpins], y[kMixSpins];
#pragma unroll
    for (int i = 0; i < kMixSpins; ++i) {
        x[i] = (float)((t + i) & 7) * 0.125f - 0.5f;
        y[i] = (float)((t + 3 * i) & 3) * 0.25f;
    }
    for (int it = 0; it < iters; ++it) {
        float yn[kMixSpins];
#pragma unroll
        for (int i = 0; i < kMixSpins; ++i) {
            float a = __builtin_fmaf(k, x[i], y[i]);
            a = __builtin_fmaf(k, x[(i + 1) % kMixSpins], a);
            a = __builtin_fmaf(k, x[(i + kMixSpins - 1) % kMixSpins], a);
            if (i < 4) a = __builtin_fmaf(k, x[i + 7], a);
            yn[i] = a;
        }
#pragma unroll
        for (int i = 0; i < kMixSpins; ++i) {
            float xi = __builtin_fmaf(k, yn[i], x[i]);
            y[i] = __builtin_fabsf(xi) > 1.0f ? 0.0f : yn[i];
            x[i] = __builtin_fminf(__builtin_fmaxf(xi, -1.0f), 1.0f);
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < kMixSpins; ++i) s += x[i] + y[i];
    out[t] = s;
}

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// nontemporal 16-byte loads and stores (the data are touched once); a sweep
// of block counts and per-lane unrolling peaked at about 1024 blocks, one
// item per lane per iteration
__global__ __launch_bounds__(kPB) void copy_peak_kernel(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst,
                                                        size_t n16) {
    const size_t stride = (size_t)gridDim.x * kPB;
    for (size_t i = (size_t)blockIdx.x * kPB + threadIdx.x; i < n16; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

void launch_peak_fma(int64_t blocks, int32_t iters, float a, float b, float *out, hipStream_t st) {
    hipLaunchKernelGGL(fma_peak_kernel, dim3((unsigned)blocks), dim3(kPB), 0, st, a, b, iters, out);
    QAIA_HIP(hipGetLastError());
}

void launch_peak_mfma(int32_t precision, int64_t blocks, int32_t iters, float *out, hipStream_t st) {
    const dim3 grid((unsigned)blocks);
    if (precision == QAIA_FP32)
        hipLaunchKernelGGL(mfma_peak_kernel<QAIA_FP32>, grid, dim3(kPB), 0, st, 0x3F800000u, iters, out);
    else if (precision == QAIA_BF16)
        hipLaunchKernelGGL(mfma_peak_kernel<QAIA_BF16>, grid, dim3(kPB), 0, st, 0x3F80u, iters, out);
    else
        hipLaunchKernelGGL(mfma_peak_kernel<QAIA_FP8>, grid, dim3(kPB), 0, st, 0x38u, iters, out);
    QAIA_HIP(hipGetLastError());
}

void launch_peak_valu(int64_t blocks, int32_t iters, float k, float *out, hipStream_t st) {
    hipLaunchKernelGGL(valu_mix_peak_kernel, dim3((unsigned)blocks), dim3(kPB), 0, st, k, iters, out);
    QAIA_HIP(hipGetLastError());
}

void launch_peak_copy(const void *src, void *dst, size_t bytes, hipStream_t st) {
    const size_t n16 = bytes / 16;
    if (n16 == 0) return;
    // four blocks per CU of a 256-CU part, or fewer for small copies
    const size_t want = (n16 + kPB - 1) / kPB;
    const unsigned blocks = (unsigned)(want < 1024 ? want : 1024);
    hipLaunchKernelGGL(copy_peak_kernel, dim3(blocks), dim3(kPB), 0, st, (const u32x4 *)src, (u32x4 *)dst, n16);
    QAIA_HIP(hipGetLastError());
}

}  // namespace qaia
