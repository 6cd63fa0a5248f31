// cf_inst_f16.hip -- single-filter query, delete and recount kernels for
// 16-bit fingerprints.
#include "cf_inst.hpp"

bool cfl::pick_launchers_f16(const cf_params &p, Launchers &out) {
    return inst::pick_b<16, false>(p, out);
}
