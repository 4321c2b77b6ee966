// Device helpers shared by the ahead-of-time kernels of libqaia.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qaia {

// Counter-based SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the value
// for counter idx is the (idx+1)-th output of the stream whose state starts
// at seed (state += golden gamma, then the variant-13 finaliser).
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t idx) {
    uint64_t z = seed + (idx + 1ull) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Initial soft spin / momentum: 24-bit uniform u, v = 2u - 1 (exact in
// float32), value = float32(amp * v).
__device__ __forceinline__ float init_value(uint64_t seed, uint64_t idx, float amp) {
    uint64_t bits = splitmix64(seed, idx);
    float u = (float)(uint32_t)(bits >> 40) * 0x1p-24f;
    float v = 2.0f * u - 1.0f;
    return amp * v;
}

// Counter of the initial draw of spin i of global replica g (x: 0, y: 1).
__device__ __forceinline__ uint64_t init_counter(uint64_t g, int n, int i, int comp) {
    return ((g * (uint64_t)n + (uint64_t)i) << 1) | (uint64_t)comp;
}

// Standard normal for noise injection (Eq. 10): Box-Muller on two 24-bit
// uniforms of one draw from the keyed stream.
constexpr uint64_t kNoiseKey = 0xd1b54a32d192ed03ull;
__device__ __forceinline__ float noise_value(uint64_t seed, uint64_t idx) {
    uint64_t bits = splitmix64(seed ^ kNoiseKey, idx);
    float u1 = (float)((uint32_t)(bits >> 40) + 1u) * 0x1p-24f;
    float u2 = (float)(uint32_t)(bits & 0xffffffu) * 0x1p-24f;
    return sqrtf(-2.0f * logf(u1)) * cosf(6.2831853071795864769f * u2);
}

// sgn with sgn(0) = +1 (x is never -0 in these dynamics).
__device__ __forceinline__ float sgn1(float x) { return x >= 0.0f ? 1.0f : -1.0f; }

// Inelastic wall: |x| > 1 -> x = sgn x, y = 0.
__device__ __forceinline__ void wall(float &x, float &y) {
    if (fabsf(x) > 1.0f) {
        x = x > 0.0f ? 1.0f : -1.0f;
        y = 0.0f;
    }
}

}  // namespace qaia
