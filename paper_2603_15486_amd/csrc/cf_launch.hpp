// cf_launch.hpp -- host-side launchers of the single-filter kernels for one
// (f, b, hash, eviction policy) instantiation, shared by the translation
// units of libcf.so.  The instantiations live in cf_api.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cf.h"
#include "cf_kernels.hpp"

namespace cfl {

struct Launchers {
    void (*query)(const void *table, uint32_t mmask, const uint64_t *keys, uint64_t n,
                  uint8_t *found, int grid, hipStream_t s);
    void (*del)(void *table, uint32_t mmask, const uint64_t *keys, uint64_t n, uint8_t *okv,
                cfk::Counters *ctr, int grid, hipStream_t s);
    void (*ins)(void *table, uint32_t mmask, const uint64_t *keys, uint64_t n, uint8_t *okv,
                uint32_t *kicks, cfk::Counters *ctr, uint32_t *queue, uint64_t seg,
                cfk::LostLog log, uint32_t max_evict, uint64_t seed, int grid, hipStream_t s);
    void (*recount)(const void *table, uint64_t nwords, cfk::Counters *ctr, int grid,
                    hipStream_t s);
    uint64_t words_per_bucket;  // in units of the geometry's word type
    uint64_t word_bytes;
};

// Launchers for p's geometry, hash and eviction policy; false if unsupported.
bool pick_launchers(const cf_params &p, Launchers &out);

// Queue entries an insert launch of `len` keys needs with `grid` blocks, and
// the per-block segment length.
inline uint64_t insert_segment(uint64_t len, int grid) {
    const uint64_t per = uint64_t(grid) * cfk::kBlock;
    return ((len + per - 1) / per) * cfk::kBlock;
}

}  // namespace cfl
