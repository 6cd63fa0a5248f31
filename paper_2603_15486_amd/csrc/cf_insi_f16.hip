// cf_insi_f16.hip -- single-filter insert kernels for 16-bit fingerprints
// (built at -O1, see the build script).
#include "cf_inst.hpp"

bool cfl::pick_insert_f16(const cf_params &p, Launchers &out) {
    return inst::pick_b<16, true>(p, out);
}
