// cf_keygen.hip -- seeded synthetic keys on the device (include/cf_keygen.h).
// Key c of stream `seed` is output c of SplitMix64 started at state `seed`.
#include <hip/hip_runtime.h>

#include "cf_device.hpp"
#include "cf_keygen.h"

namespace {

constexpr int kKeyBlock = 256;

__global__ __launch_bounds__(kKeyBlock) void keygen_kernel(uint64_t *__restrict__ out, uint64_t n,
                                                           uint64_t seed, uint64_t start) {
    const uint64_t stride = uint64_t(gridDim.x) * kKeyBlock;
    for (uint64_t i = uint64_t(blockIdx.x) * kKeyBlock + threadIdx.x; i < n; i += stride)
        __builtin_nontemporal_store(cfk::splitmix_at(seed, start + i), out + i);
}

__global__ __launch_bounds__(kKeyBlock) void keygen_at_kernel(uint64_t *__restrict__ out,
                                                              const uint64_t *__restrict__ ctr,
                                                              uint64_t n, uint64_t seed) {
    const uint64_t stride = uint64_t(gridDim.x) * kKeyBlock;
    for (uint64_t i = uint64_t(blockIdx.x) * kKeyBlock + threadIdx.x; i < n; i += stride)
        out[i] = cfk::splitmix_at(seed, ctr[i]);
}

int keygen_grid(uint64_t n) {
    const uint64_t want = (n + kKeyBlock - 1) / kKeyBlock;
    return int(want < 8192 ? (want ? want : 1) : 8192);
}

}  // namespace

extern "C" cf_status cf_keygen(uint64_t *d_out, uint64_t n, uint64_t seed, uint64_t start,
                               void *stream) {
    if (n == 0) return CF_OK;
    if (!d_out || (reinterpret_cast<uintptr_t>(d_out) & 7u)) return CF_EINVAL;
    keygen_kernel<<<keygen_grid(n), kKeyBlock, 0, static_cast<hipStream_t>(stream)>>>(d_out, n,
                                                                                      seed, start);
    return hipGetLastError() == hipSuccess ? CF_OK : CF_EDEVICE;
}

extern "C" cf_status cf_keygen_at(uint64_t *d_out, const uint64_t *d_counters, uint64_t n,
                                  uint64_t seed, void *stream) {
    if (n == 0) return CF_OK;
    if (!d_out || !d_counters) return CF_EINVAL;
    keygen_at_kernel<<<keygen_grid(n), kKeyBlock, 0, static_cast<hipStream_t>(stream)>>>(
        d_out, d_counters, n, seed);
    return hipGetLastError() == hipSuccess ? CF_OK : CF_EDEVICE;
}
