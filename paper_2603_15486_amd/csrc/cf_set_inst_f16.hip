// cf_set_inst_f16.hip -- filter-set query, delete and recount kernels for
// 16-bit fingerprints.
#include "cf_set_kernels.hpp"

bool cfs::pick_class_f16(uint32_t b, uint32_t hash, uint32_t placement, ClassLaunch &out) {
    return pick_class_b<16, false>(b, hash, placement, out);
}
