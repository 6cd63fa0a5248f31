// cf_insi_f8.hip -- single-filter insert kernels for 8-bit fingerprints
// (built at -O1, see the build script).
#include "cf_inst.hpp"

bool cfl::pick_insert_f8(const cf_params &p, Launchers &out) {
    return inst::pick_b<8, true>(p, out);
}
