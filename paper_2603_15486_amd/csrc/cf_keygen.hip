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

// One read of W bytes per thread at the start of a random line; the values
// are summed so the loads stay, and the sum reaches memory only in the
// (practically never taken) case that it equals a fixed constant.
template <int W>
__global__ __launch_bounds__(kKeyBlock) void probe_lines_kernel(const uint8_t *__restrict__ buf,
                                                                uint64_t mask, uint32_t shift,
                                                                uint64_t n, uint64_t seed,
                                                                unsigned long long *sink) {
    const uint64_t stride = uint64_t(gridDim.x) * kKeyBlock;
    uint64_t acc = 0;
    for (uint64_t i = uint64_t(blockIdx.x) * kKeyBlock + threadIdx.x; i < n; i += stride) {
        const uint8_t *p = buf + ((cfk::splitmix_at(seed, i) & mask) << shift);
        if constexpr (W == 16) {
            const ulonglong2 v = *reinterpret_cast<const ulonglong2 *>(p);
            acc += v.x ^ v.y;
        } else {
            acc += *reinterpret_cast<const unsigned long long *>(p);
        }
    }
    if (acc == 0x9e3779b97f4a7c15ull) atomicAdd(sink, 1ull);
}

// One device-scope 64-bit CAS per thread on the first word of a random
// line, as a bucket update does it: READ = 1 loads the word first and swaps
// it for a changed value (the CAS succeeds unless another thread got there
// first); READ = 0 issues the CAS blind, expecting 0.  The returned values
// are summed so that no CAS can be dropped.
template <int READ>
__global__ __launch_bounds__(kKeyBlock) void probe_atomics_kernel(unsigned long long *__restrict__ buf,
                                                                  uint64_t mask, uint32_t shift,
                                                                  uint64_t n, uint64_t seed,
                                                                  unsigned long long *sink) {
    const uint64_t stride = uint64_t(gridDim.x) * kKeyBlock;
    uint64_t acc = 0;
    for (uint64_t i = uint64_t(blockIdx.x) * kKeyBlock + threadIdx.x; i < n; i += stride) {
        const uint64_t r = cfk::splitmix_at(seed, i);
        unsigned long long *w = buf + (((r & mask) << shift) >> 3);
        const unsigned long long expect = READ ? *w : 0ull;
        acc += atomicCAS(w, expect, expect ^ (r | 1ull));
    }
    if (acc == 0x9e3779b97f4a7c15ull) atomicAdd(sink, 1ull);
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

extern "C" cf_status cf_probe_lines(const void *d_buf, uint64_t n_lines, uint32_t line_bytes,
                                    uint32_t width, uint64_t n_reads, uint64_t seed,
                                    uint64_t *d_sink, void *stream) {
    auto pow2 = [](uint64_t x) { return x && !(x & (x - 1)); };
    if (!d_buf || !d_sink || (reinterpret_cast<uintptr_t>(d_buf) & 15u) ||
        (reinterpret_cast<uintptr_t>(d_sink) & 7u) || !pow2(n_lines) ||
        !pow2(line_bytes) || (width != 8 && width != 16) || line_bytes < width)
        return CF_EINVAL;
    if (n_reads == 0) return CF_OK;
    uint32_t shift = 0;
    while ((1u << shift) < line_bytes) ++shift;
    const uint64_t want = (n_reads + kKeyBlock - 1) / kKeyBlock;
    const int grid = int(want < (1u << 18) ? want : (1u << 18));  // one read per thread
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint8_t *buf = static_cast<const uint8_t *>(d_buf);
    auto *sink = reinterpret_cast<unsigned long long *>(d_sink);
    if (width == 16)
        probe_lines_kernel<16><<<grid, kKeyBlock, 0, st>>>(buf, n_lines - 1, shift, n_reads, seed,
                                                           sink);
    else
        probe_lines_kernel<8><<<grid, kKeyBlock, 0, st>>>(buf, n_lines - 1, shift, n_reads, seed,
                                                          sink);
    return hipGetLastError() == hipSuccess ? CF_OK : CF_EDEVICE;
}

extern "C" cf_status cf_probe_atomics(void *d_buf, uint64_t n_lines, uint32_t line_bytes,
                                      uint32_t read_first, uint64_t n_ops, uint64_t seed,
                                      uint64_t *d_sink, void *stream) {
    auto pow2 = [](uint64_t x) { return x && !(x & (x - 1)); };
    if (!d_buf || !d_sink || (reinterpret_cast<uintptr_t>(d_buf) & 7u) ||
        (reinterpret_cast<uintptr_t>(d_sink) & 7u) || !pow2(n_lines) || !pow2(line_bytes) ||
        line_bytes < 8 || read_first > 1)
        return CF_EINVAL;
    if (n_ops == 0) return CF_OK;
    uint32_t shift = 0;
    while ((1u << shift) < line_bytes) ++shift;
    const uint64_t want = (n_ops + kKeyBlock - 1) / kKeyBlock;
    const int grid = int(want < (1u << 18) ? want : (1u << 18));  // one CAS per thread
    hipStream_t st = static_cast<hipStream_t>(stream);
    auto *buf = static_cast<unsigned long long *>(d_buf);
    auto *sink = reinterpret_cast<unsigned long long *>(d_sink);
    if (read_first)
        probe_atomics_kernel<1><<<grid, kKeyBlock, 0, st>>>(buf, n_lines - 1, shift, n_ops, seed,
                                                            sink);
    else
        probe_atomics_kernel<0><<<grid, kKeyBlock, 0, st>>>(buf, n_lines - 1, shift, n_ops, seed,
                                                            sink);
    return hipGetLastError() == hipSuccess ? CF_OK : CF_EDEVICE;
}
