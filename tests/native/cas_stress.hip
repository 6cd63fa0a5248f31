// cas_stress.hip -- test infrastructure: a device-wide compare-and-swap
// stress.  Every thread of a grid that fills all compute units (and so all
// XCDs) increments pseudo-random 64-bit counters `iters` times with a CAS
// loop, reading the expected value first with a plain 8-byte load (mode 0),
// with a 16-byte vector load of the aligned pair holding the counter as the
// filter's bucket loads do (mode 1), or with the hardware atomic add (mode
// 2).  The counters must sum to exactly blocks * 256 * iters: the insert,
// delete and eviction kernels rely on device-scope CAS being exact across
// XCDs while the same lines are also read with plain loads.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace {

__device__ uint64_t mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void stress_kernel(unsigned long long *c, uint32_t ncnt,
                                                     int iters, int mode,
                                                     unsigned long long *gave_up) {
    const uint64_t tid = uint64_t(blockIdx.x) * 256 + threadIdx.x;
    for (int it = 0; it < iters; ++it) {
        const uint32_t idx = uint32_t(mix(tid * 1315423911ull + uint64_t(it)) % ncnt);
        unsigned long long *p = c + idx;
        if (mode == 2) {
            atomicAdd(p, 1ull);
            continue;
        }
        unsigned long long old;
        if (mode == 1) {
            const ulonglong2 v = *reinterpret_cast<const ulonglong2 *>(c + (idx & ~1u));
            old = (idx & 1u) ? v.y : v.x;
        } else {
            old = *p;
        }
        for (int guard = 0;; ++guard) {  // bounded: gives up after 2^20 failed CAS
            const unsigned long long prev = atomicCAS(p, old, old + 1);
            if (prev == old) break;
            old = prev;
            if (guard == (1 << 20)) {
                atomicAdd(gave_up, 1ull);
                break;
            }
        }
    }
}

}  // namespace

// Runs the stress on the current device; *sum receives the counters' total
// and *gave_up the increments abandoned by the retry bound.  ncnt must be
// even and >= 2.  Returns 0, or a HIP error code.
extern "C" int cas_stress(uint32_t ncnt, int blocks, int iters, int mode, uint64_t *sum,
                          uint64_t *gave_up) {
    if (ncnt < 2 || (ncnt & 1u) || blocks < 1 || iters < 1 || mode < 0 || mode > 2) return -1;
    unsigned long long *c = nullptr, *g = nullptr;
    hipError_t e = hipMalloc(&c, ncnt * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc(&g, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemset(c, 0, ncnt * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemset(g, 0, sizeof(unsigned long long));
    if (e == hipSuccess) {
        stress_kernel<<<blocks, 256>>>(c, ncnt, iters, mode, g);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    std::vector<unsigned long long> h(ncnt);
    unsigned long long hg = 0;
    if (e == hipSuccess)
        e = hipMemcpy(h.data(), c, ncnt * sizeof(unsigned long long), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&hg, g, sizeof(hg), hipMemcpyDeviceToHost);
    if (c) (void)hipFree(c);
    if (g) (void)hipFree(g);
    if (e != hipSuccess) return int(e);
    uint64_t s = 0;
    for (unsigned long long v : h) s += v;
    *sum = s;
    *gave_up = hg;
    return 0;
}
