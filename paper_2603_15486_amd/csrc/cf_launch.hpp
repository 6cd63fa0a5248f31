// cf_launch.hpp -- host-side launchers of the single-filter kernels for one
// (f, b, hash, eviction policy, placement) instantiation, shared by the
// translation units of libcf.so.  The instantiations live in cf_inst_f*.hip,
// one translation unit per fingerprint width so that they compile in
// parallel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cf.h"
#include "cf_kernels.hpp"

namespace cfl {

struct Launchers {
    void (*query)(const void *table, const cfk::Place &pl, const uint64_t *keys, uint64_t n,
                  uint8_t *found, int grid, hipStream_t s);
    void (*del)(void *table, const cfk::Place &pl, const uint64_t *keys, uint64_t n,
                uint8_t *okv, cfk::Counters *ctr, int grid, hipStream_t s);
    void (*ins)(void *table, const cfk::Place &pl, const uint64_t *keys, uint64_t n,
                uint8_t *okv, uint32_t *kicks, cfk::Counters *ctr, uint32_t *queue, uint64_t seg,
                cfk::LostLog log, uint32_t max_evict, uint64_t seed, int grid, hipStream_t s);
    void (*recount)(const void *table, uint64_t nwords, cfk::Counters *ctr, int grid,
                    hipStream_t s);
    uint64_t words_per_bucket;  // in units of the geometry's word type
    uint64_t word_bytes;
};

// Launchers for p's geometry, hash, eviction policy and placement; false if
// unsupported.  pick_launchers dispatches on f to the per-width tables
// (pick_launchers_f*: query, delete, recount; pick_insert_f*: insert).
bool pick_launchers(const cf_params &p, Launchers &out);
bool pick_launchers_f8(const cf_params &p, Launchers &out);
bool pick_launchers_f16(const cf_params &p, Launchers &out);
bool pick_launchers_f32(const cf_params &p, Launchers &out);
bool pick_insert_f8(const cf_params &p, Launchers &out);
bool pick_insert_f16(const cf_params &p, Launchers &out);
bool pick_insert_f32(const cf_params &p, Launchers &out);

// Checks every field of p (what cf_create documents); on failure records
// the message, prefixed by `who` when it is not empty, and returns the
// status.
cf_status check_params(const cf_params &p, const char *who);

// The kernels' view of p's placement (p already checked).
inline cfk::Place make_place(const cf_params &p) {
    cfk::Place pl{};
    if (p.placement == CF_PLACE_OFFSET) {
        pl.m = uint32_t(p.num_buckets);
        pl.m1 = pl.m - 1;
        pl.mdiv = cfk::fastmod_constant(pl.m);
        pl.m1div = pl.m1 ? cfk::fastmod_constant(pl.m1) : 0;
    } else {
        pl.mmask = uint32_t(p.num_buckets - 1);
    }
    return pl;
}

// Queue entries an insert launch of `len` keys needs with `grid` blocks, and
// the per-block segment length.
inline uint64_t insert_segment(uint64_t len, int grid) {
    const uint64_t per = uint64_t(grid) * cfk::kBlock;
    return ((len + per - 1) / per) * cfk::kBlock;
}

}  // namespace cfl
