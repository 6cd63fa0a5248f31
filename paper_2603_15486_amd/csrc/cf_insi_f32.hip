// cf_insi_f32.hip -- single-filter insert kernels for 32-bit fingerprints
// (built at -O1, see the build script).
#include "cf_inst.hpp"

bool cfl::pick_insert_f32(const cf_params &p, Launchers &out) {
    return inst::pick_b<32, true>(p, out);
}
