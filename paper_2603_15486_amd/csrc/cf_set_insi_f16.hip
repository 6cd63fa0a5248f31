// cf_set_insi_f16.hip -- filter-set insert kernels for 16-bit fingerprints
// (built at -O1, see the build script).
#include "cf_set_kernels.hpp"

bool cfs::pick_class_insert_f16(uint32_t b, uint32_t hash, uint32_t placement,
                                 ClassLaunch &out) {
    return pick_class_b<16, true>(b, hash, placement, out);
}
