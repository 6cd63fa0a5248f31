// cf_inst.hpp -- the single-filter kernel instantiations behind
// cfl::Launchers.  Included only by the cf_inst_f*.hip translation units,
// each of which instantiates one fingerprint width.
#pragma once

#include "cf_launch.hpp"

namespace cfl {
namespace inst {

using cfk::Counters;
using cfk::kBlock;

template <int F, int B, int HASH, int EVICT, int POL>
struct Inst {
    using G = cfk::Geom<F, B>;
    using W = typename G::W;
    static void query(const void *t, const cfk::Place &pl, const uint64_t *k, uint64_t n,
                      uint8_t *o, int grid, hipStream_t s) {
        cfk::query_kernel<G, HASH, POL>
            <<<grid, kBlock, 0, s>>>(static_cast<const W *>(t), pl, k, n, o);
    }
    static void del(void *t, const cfk::Place &pl, const uint64_t *k, uint64_t n, uint8_t *o,
                    Counters *c, int grid, hipStream_t s) {
        cfk::delete_kernel<G, HASH, POL>
            <<<grid, kBlock, 0, s>>>(static_cast<W *>(t), pl, k, n, o, c);
    }
    static void ins(void *t, const cfk::Place &pl, const uint64_t *k, uint64_t n, uint8_t *o,
                    uint32_t *kk, Counters *c, uint32_t *q, uint64_t seg, cfk::LostLog log,
                    uint32_t me, uint64_t seed, int grid, hipStream_t s) {
        cfk::insert_kernel<G, HASH, EVICT, POL><<<grid, kBlock, 0, s>>>(
            static_cast<W *>(t), pl, k, n, o, kk, c, q, seg, log, me, seed);
    }
    static void recount(const void *t, uint64_t nw, Counters *c, int grid, hipStream_t s) {
        cfk::recount_kernel<G><<<grid, kBlock, 0, s>>>(static_cast<const W *>(t), nw, c);
    }
    static constexpr Launchers table() {
        return Launchers{&query, &del, &ins, &recount, uint64_t(G::WPB), uint64_t(sizeof(W))};
    }
};

template <int F, int B, int POL>
constexpr Launchers pick_he(int hash, int evict) {
    return hash == 0
               ? (evict == 0 ? Inst<F, B, 0, 0, POL>::table() : Inst<F, B, 0, 1, POL>::table())
               : (evict == 0 ? Inst<F, B, 1, 0, POL>::table() : Inst<F, B, 1, 1, POL>::table());
}

template <int F, int B>
constexpr Launchers pick_p(const cf_params &p) {
    return p.placement == CF_PLACE_OFFSET ? pick_he<F, B, 1>(p.hash, p.evict)
                                          : pick_he<F, B, 0>(p.hash, p.evict);
}

template <int F>
bool pick_b(const cf_params &p, Launchers &out) {
    switch (p.slots_per_bucket) {
        case 4: out = pick_p<F, 4>(p); return true;
        case 8: out = pick_p<F, 8>(p); return true;
        case 16: out = pick_p<F, 16>(p); return true;
        case 32: out = pick_p<F, 32>(p); return true;
        default: return false;
    }
}

}  // namespace inst
}  // namespace cfl
