// cf_set_persist_insi_f16.hip -- the persistent batch kernel and the insert
// phase kernel for 16-bit fingerprints (built at -O1: they hold insert code,
// see the build script).
#include "cf_set_persist.hpp"

bool cfs::pick_persist_f16(uint32_t hash, uint32_t placement, uint32_t bmax,
                           PersistLaunch &out) {
    return pick_persist_f<16>(hash, placement, bmax, out);
}

bool cfs::pick_phase_insert_f16(uint32_t hash, uint32_t placement, uint32_t bmax,
                                PhaseLaunch &out) {
    return pick_phase_f<16, true>(hash, placement, bmax, out);
}
