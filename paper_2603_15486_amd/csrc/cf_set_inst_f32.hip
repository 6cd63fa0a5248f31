// cf_set_inst_f32.hip -- filter-set query, delete and recount kernels for
// 32-bit fingerprints.
#include "cf_set_kernels.hpp"

bool cfs::pick_class_f32(uint32_t b, uint32_t hash, uint32_t placement, ClassLaunch &out) {
    return pick_class_b<32, false>(b, hash, placement, out);
}
