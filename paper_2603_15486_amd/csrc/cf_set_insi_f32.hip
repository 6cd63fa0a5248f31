// cf_set_insi_f32.hip -- filter-set insert kernels for 32-bit fingerprints
// (built at -O1, see the build script).
#include "cf_set_kernels.hpp"

bool cfs::pick_class_insert_f32(uint32_t b, uint32_t hash, uint32_t placement,
                                 ClassLaunch &out) {
    return pick_class_b<32, true>(b, hash, placement, out);
}
