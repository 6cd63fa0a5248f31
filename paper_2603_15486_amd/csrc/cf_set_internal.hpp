// cf_set_internal.hpp -- what other translation units of the library may
// ask of a filter set beyond its C ABI (include/cf_set.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cf_set.h"

namespace cfs {

// Number of filters the set was created with (0 for NULL).
uint32_t filter_count(const cf_set *set);

// Scratch lanes.  A batch uses the chunk scratch (sorted indices, bin
// offsets, eviction queue) of one lane; batches on different lanes may be
// in flight at once and overlap on the device, as long as they touch
// disjoint filters (the caller orders batches that share a filter).  Lane 0
// is the set's own scratch, which cf_set_execute, graphs and cf_set_apply
// use.  reserve_lanes makes lanes 1 .. n-1 (synchronous; set-up only).
uint32_t lane_count(const cf_set *set);
cf_status reserve_lanes(cf_set *set, uint32_t n);

// cf_set_execute on one lane, always in the class-kernel form with every
// class chain on `stream` (never the persistent form, whose cooperative
// grid takes the whole device, and never the set's side streams, which the
// lanes share).
cf_status execute_lane(cf_set *set, uint32_t lane, const uint8_t *ops, const uint32_t *fids,
                       const uint64_t *keys, uint64_t n, uint8_t *results, hipStream_t stream);

// cf_set_apply on one lane.
cf_status apply_lane(cf_set *set, uint32_t lane, uint32_t fid, uint32_t op, const uint64_t *keys,
                     uint64_t n, uint8_t *results, hipStream_t stream);

}  // namespace cfs
