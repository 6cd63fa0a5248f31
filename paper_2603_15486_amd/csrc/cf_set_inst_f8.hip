// cf_set_inst_f8.hip -- filter-set query, delete and recount kernels for
// 8-bit fingerprints: the class kernels and the query and delete phase
// kernels.
#include "cf_set_persist.hpp"

bool cfs::pick_class_f8(uint32_t b, uint32_t hash, uint32_t placement, ClassLaunch &out) {
    return pick_class_b<8, false>(b, hash, placement, out);
}

bool cfs::pick_phase_f8(uint32_t hash, uint32_t placement, uint32_t bmax, PhaseLaunch &out) {
    return pick_phase_f<8, false>(hash, placement, bmax, out);
}
