// cf_set_persist_insi_f8.hip -- the persistent batch kernel and the insert
// phase kernel for 8-bit fingerprints (built at -O1: they hold insert code,
// see the build script).
#include "cf_set_persist.hpp"

bool cfs::pick_persist_f8(uint32_t hash, uint32_t placement, uint32_t bmax,
                           PersistLaunch &out) {
    return pick_persist_f<8>(hash, placement, bmax, out);
}

bool cfs::pick_phase_insert_f8(uint32_t hash, uint32_t placement, uint32_t bmax,
                                PhaseLaunch &out) {
    return pick_phase_f<8, true>(hash, placement, bmax, out);
}
