// cf_inst_f32.hip -- single-filter query, delete and recount kernels for
// 32-bit fingerprints.
#include "cf_inst.hpp"

bool cfl::pick_launchers_f32(const cf_params &p, Launchers &out) {
    return inst::pick_b<32, false>(p, out);
}
