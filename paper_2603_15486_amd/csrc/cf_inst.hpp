// cf_inst.hpp -- the single-filter kernel instantiations behind
// cfl::Launchers.  Included only by the cf_inst_f*.hip (query, delete,
// recount) and cf_insi_f*.hip (insert) translation units, each of which
// instantiates one fingerprint width; the insert units are built at -O1
// (see the build script).
#pragma once

#include <type_traits>

#include "cf_launch.hpp"

namespace cfl {
namespace inst {

using cfk::Counters;
using cfk::kBlock;

// Query, delete and recount: independent of the eviction policy.
template <int F, int B, int HASH, int POL>
struct InstQD {
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
    static void recount(const void *t, uint64_t nw, Counters *c, int grid, hipStream_t s) {
        cfk::recount_kernel<G><<<grid, kBlock, 0, s>>>(static_cast<const W *>(t), nw, c);
    }
    static void fill(Launchers &L) {
        L.query = &query;
        L.del = &del;
        L.recount = &recount;
        L.words_per_bucket = uint64_t(G::WPB);
        L.word_bytes = uint64_t(sizeof(W));
    }
};

// Insert, per eviction policy and breadth-first probe width.
template <int F, int B, int HASH, int EVICT, int POL, int PW>
struct InstI {
    using G = cfk::Geom<F, B>;
    using W = typename G::W;
    static void ins(void *t, const cfk::Place &pl, const uint64_t *k, uint64_t n, uint8_t *o,
                    uint32_t *kk, Counters *c, uint32_t *q, uint64_t seg, cfk::LostLog log,
                    uint32_t me, uint64_t seed, int grid, hipStream_t s) {
        cfk::insert_kernel<G, HASH, EVICT, POL, PW><<<grid, kBlock, 0, s>>>(
            static_cast<W *>(t), pl, k, n, o, kk, c, q, seg, log, me, seed);
    }
};

// Tables of at most this many bytes get a breadth-first search that loads
// each group of candidates' other buckets together (cfk::probe_width); the
// rest probe candidate by candidate.  Measured on one-launch fills at load
// 0.95: 2 MiB 6.6 -> 7.25 Gops/s and 8 MiB 13.8 -> 14.3-14.7 grouped.  The
// 64 MiB eviction-stress table (4-byte buckets, to load 0.98) was 2-5%
// slower grouped, and the 512 MiB and 4 GiB tables, whose probes are HBM
// requests, 3% (the 4 GiB step's inserts 15%).
constexpr uint64_t kGroupedProbeBytes = uint64_t(16) << 20;

template <int F, int B, int POL>
void fill_qd(int hash, Launchers &L) {
    if (hash == 0) InstQD<F, B, 0, POL>::fill(L);
    else InstQD<F, B, 1, POL>::fill(L);
}

template <int F, int B, int POL>
void fill_ins(int hash, int evict, bool grouped, Launchers &L) {
    constexpr int PW = cfk::probe_width<cfk::Geom<F, B>>();
    if (evict == 0 && grouped)
        L.ins = hash == 0 ? &InstI<F, B, 0, 0, POL, PW>::ins : &InstI<F, B, 1, 0, POL, PW>::ins;
    else
        L.ins = hash == 0
                    ? (evict == 0 ? &InstI<F, B, 0, 0, POL, 1>::ins : &InstI<F, B, 0, 1, POL, 1>::ins)
                    : (evict == 0 ? &InstI<F, B, 1, 0, POL, 1>::ins : &InstI<F, B, 1, 1, POL, 1>::ins);
}

// Fills the query/delete/recount part (INSERT = false) or the insert part
// (INSERT = true) of L for p's bucket size; false if unsupported.
template <int F, bool INSERT>
bool pick_b(const cf_params &p, Launchers &L) {
    auto one = [&](auto bconst) {
        constexpr int B = decltype(bconst)::value;
        const bool off = p.placement == CF_PLACE_OFFSET;
        if constexpr (INSERT) {
            const bool grouped = p.num_buckets * uint64_t(B) * uint64_t(F) / 8 <= kGroupedProbeBytes;
            if (off) fill_ins<F, B, 1>(p.hash, p.evict, grouped, L);
            else fill_ins<F, B, 0>(p.hash, p.evict, grouped, L);
        } else {
            if (off) fill_qd<F, B, 1>(p.hash, L);
            else fill_qd<F, B, 0>(p.hash, L);
        }
        return true;
    };
    switch (p.slots_per_bucket) {
        case 4: return one(std::integral_constant<int, 4>{});
        case 8: return one(std::integral_constant<int, 8>{});
        case 16: return one(std::integral_constant<int, 16>{});
        case 32: return one(std::integral_constant<int, 32>{});
        default: return false;
    }
}

}  // namespace inst
}  // namespace cfl
