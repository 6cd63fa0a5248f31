// cf_inst_f8.hip -- single-filter query, delete and recount kernels for
// 8-bit fingerprints.
#include "cf_inst.hpp"

bool cfl::pick_launchers_f8(const cf_params &p, Launchers &out) {
    return inst::pick_b<8, false>(p, out);
}
