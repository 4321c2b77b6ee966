// Scratch memory of the allocation-free sampling entry point: a static device
// array that stands in for the caller's workspace, so that qaia_sample_noalloc
// needs no hipMalloc.  Each GPU the library runs on holds its own copy of the
// array until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device (the array's name in host
// code is not a device address).
#include <climits>

#include "internal.hpp"

namespace qaia {

constexpr size_t kNoallocScratchBytes = QAIA_NOALLOC_SCRATCH_BYTES;
static_assert(kNoallocScratchBytes % 256 == 0, "scratch size must keep the workspace alignment");

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

__global__ void noalloc_bad_row_kernel(const WsHeader *h, int64_t *out) {
    if (threadIdx.x == 0) *out = h->bad_row == INT64_MAX ? -1 : h->bad_row;
}

}  // namespace

// Address of `device`'s copy of the scratch array, looked up once per device
// with that device current.
void *noalloc_scratch(int device) {
    int count = 0;
    QAIA_HIP(hipGetDeviceCount(&count));
    QAIA_CHECK(device >= 0 && device < count && device < kMaxDevices, QAIA_INVALID_ARGUMENT,
               "device out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device] == nullptr) {
        DeviceGuard g(device);
        void *ptr = nullptr;
        QAIA_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        QAIA_CHECK(ptr != nullptr, QAIA_DEVICE_ERROR, "scratch array has no device address");
        g_scratch_ptr[device] = ptr;
    }
    return g_scratch_ptr[device];
}

size_t noalloc_scratch_bytes() { return kNoallocScratchBytes; }

// `scratch` is a device address from noalloc_scratch(); the workspace header
// sits at its start.
void launch_noalloc_bad_row(const void *scratch_dev, int64_t *bad_row, hipStream_t st) {
    hipLaunchKernelGGL(noalloc_bad_row_kernel, dim3(1), dim3(64), 0, st, (const WsHeader *)scratch_dev,
                       bad_row);
    QAIA_HIP(hipGetLastError());
}

}  // namespace qaia
