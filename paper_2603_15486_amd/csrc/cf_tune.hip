// cf_tune.hip -- geometry and launch-shape tuning (include/cf_tune.h).
//
// Both tuners drive the library's own entry points: the geometry tuner
// times standalone filters (cf_create / cf_insert / cf_query / cf_delete)
// on probe tables, the shape tuner times cf_set_execute under each
// candidate launch shape and undoes every trial with a second batch built
// on the device from the trial's results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "cf.h"
#include "cf_error.hpp"
#include "cf_keygen.h"
#include "cf_set.h"
#include "cf_set_internal.hpp"
#include "cf_tune.h"

using cferr::fail;

namespace cft {

constexpr uint32_t kFps[] = {8, 16, 32};
constexpr uint32_t kSlots[] = {4, 8, 16, 32};
constexpr uint64_t kQueryKeys = 1ull << 22;
constexpr uint64_t kFillChunk = 1ull << 24;
constexpr uint64_t kNegativeBase = 1ull << 63;  // key counters never used for stored keys

uint64_t next_pow2(uint64_t x) {
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Eq. (4): 1 - (1 - 2^-f)^(2 b alpha), evaluated without cancellation.
double fpr_eq4(uint32_t f, uint32_t b, double alpha) {
    return -std::expm1(2.0 * b * alpha * std::log1p(-std::ldexp(1.0, -int(f))));
}

// The offset placement compares f - 1 fingerprint bits in the b slots of
// each bucket and the choice bit besides, so a negative key meets b*alpha
// occupied slots in expectation that can match, each with chance
// 2^-(f-1): 1 - (1 - 2^-(f-1))^(b alpha), to first order Eq. (4)'s rate.
double fpr_offset(uint32_t f, uint32_t b, double alpha) {
    return -std::expm1(double(b) * alpha * std::log1p(-std::ldexp(1.0, 1 - int(f))));
}

struct ProbeResult {
    double rate[3] = {0, 0, 0};  // query, delete, insert
    uint32_t failures = 0;
};

using ProbeKey = std::tuple<int, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t,
                            uint64_t, uint64_t, uint64_t, uint64_t, uint64_t>;
std::mutex g_mu;
std::map<ProbeKey, ProbeResult> g_cache;

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    bool alloc(size_t bytes) { return hipMalloc(&p, bytes ? bytes : 1) == hipSuccess; }
};

struct Events {
    hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
    ~Events() {
        for (hipEvent_t x : e)
            if (x) (void)hipEventDestroy(x);
    }
    bool create() {
        for (hipEvent_t &x : e)
            if (hipEventCreate(&x) != hipSuccess) return false;
        return true;
    }
};

double median3(double a, double b, double c) {
    return std::max(std::min(a, b), std::min(std::max(a, b), c));
}

// Fill a filter of the candidate geometry (m_probe buckets) to fill_lo keys,
// then three times: insert `band` more keys, query kQueryKeys keys (npos of
// them stored), delete the band again.  Rates are medians of the three.
cf_status probe(const cf_params &cand, uint64_t m_probe, uint64_t fill_lo, uint64_t band,
                uint64_t npos, uint64_t seed, hipStream_t st, ProbeResult &out) {
    cf_params p = cand;
    p.num_buckets = m_probe;
    cf_filter *flt = nullptr;
    cf_status rc = cf_create(&p, &flt);
    if (rc != CF_OK) return rc;
    struct Guard {
        cf_filter *f;
        ~Guard() { cf_destroy(f); }
    } guard{flt};
    const uint64_t fill_step = std::min(kFillChunk, std::max<uint64_t>(fill_lo, 1));
    const uint64_t res_n = std::max({fill_step, band, kQueryKeys});
    DevBuf kfill, kband, kq, res;
    if (!kfill.alloc(fill_step * 8) || !kband.alloc(band * 8) || !kq.alloc(kQueryKeys * 8) ||
        !res.alloc(res_n))
        return fail(CF_ENOMEM, "cannot allocate probe buffers");
    if ((rc = cf_reserve(flt, std::max(fill_step, band))) != CF_OK) return rc;
    auto *kf = static_cast<uint64_t *>(kfill.p);
    auto *kb = static_cast<uint64_t *>(kband.p);
    auto *kk = static_cast<uint64_t *>(kq.p);
    auto *r = static_cast<uint8_t *>(res.p);
    for (uint64_t off = 0; off < fill_lo; off += fill_step) {
        const uint64_t k = std::min(fill_step, fill_lo - off);
        if ((rc = cf_keygen(kf, k, seed, off, st)) != CF_OK) return rc;
        if ((rc = cf_insert(flt, kf, k, nullptr, nullptr, st)) != CF_OK) return rc;
    }
    if ((rc = cf_keygen(kb, band, seed, fill_lo, st)) != CF_OK) return rc;
    // Positive queries cycle over the stored keys; negatives use counters no
    // stored key has.
    const uint64_t stored = std::max<uint64_t>(fill_lo, 1);
    for (uint64_t off = 0; off < npos; off += stored) {
        const uint64_t k = std::min(stored, npos - off);
        if ((rc = cf_keygen(kk + off, k, seed, 0, st)) != CF_OK) return rc;
    }
    if (npos < kQueryKeys &&
        (rc = cf_keygen(kk + npos, kQueryKeys - npos, seed, kNegativeBase, st)) != CF_OK)
        return rc;
    Events ev;
    if (!ev.create()) return fail(CF_EDEVICE, "cannot create events");
    double ms[3][3];
    for (int rep = 0; rep < 3; ++rep) {
        (void)hipEventRecord(ev.e[0], st);
        if ((rc = cf_insert(flt, kb, band, nullptr, nullptr, st)) != CF_OK) return rc;
        (void)hipEventRecord(ev.e[1], st);
        if ((rc = cf_query(flt, kk, kQueryKeys, r, st)) != CF_OK) return rc;
        (void)hipEventRecord(ev.e[2], st);
        if ((rc = cf_delete(flt, kb, band, nullptr, st)) != CF_OK) return rc;
        (void)hipEventRecord(ev.e[3], st);
        if (hipEventSynchronize(ev.e[3]) != hipSuccess) return fail(CF_EDEVICE, "probe failed");
        float t[3];
        for (int k = 0; k < 3; ++k) (void)hipEventElapsedTime(&t[k], ev.e[k], ev.e[k + 1]);
        ms[2][rep] = t[0];  // insert
        ms[0][rep] = t[1];  // query
        ms[1][rep] = t[2];  // delete
    }
    const double cnt[3] = {double(kQueryKeys), double(band), double(band)};
    for (int k = 0; k < 3; ++k) {
        const double m = median3(ms[k][0], ms[k][1], ms[k][2]);
        out.rate[k] = m > 0 ? cnt[k] / (m * 1e-3) : 0.0;
    }
    uint64_t fails = 0;
    if ((rc = cf_failures(flt, &fails, st)) != CF_OK) return rc;
    if (hipStreamSynchronize(st) != hipSuccess) return fail(CF_EDEVICE, "probe failed");
    out.failures = uint32_t(std::min<uint64_t>(fails, 0xFFFFFFFFu));
    return CF_OK;
}

// Undo of one executed mixed batch: stored inserts become deletes, removing
// deletes become inserts, everything else is made invalid (ignored).
__global__ __launch_bounds__(256) void undo_ops_kernel(const uint8_t *__restrict__ ops,
                                                       const uint8_t *__restrict__ res,
                                                       uint64_t n, uint8_t *__restrict__ undo) {
    const uint64_t stride = uint64_t(gridDim.x) * 256;
    for (uint64_t j = uint64_t(blockIdx.x) * 256 + threadIdx.x; j < n; j += stride) {
        const uint8_t op = ops[j];
        uint8_t u = 0xFF;
        if (res[j] == 1) u = op == CF_OP_INSERT ? CF_OP_DELETE : (op == CF_OP_DELETE ? CF_OP_INSERT : 0xFF);
        undo[j] = u;
    }
}

// The keys of one tuning execution: each insert's key replaced by a fresh
// one mixed from it and the execution's salt (SplitMix64's output function,
// a bijection of 64-bit words), every other operation's key kept.  An undo
// removes exactly the keys the execution stored, so without fresh keys the
// next execution would re-insert them into the very slots the undo just
// emptied and never need an eviction search.
__global__ __launch_bounds__(256) void fresh_insert_keys_kernel(const uint8_t *__restrict__ ops,
                                                                const uint64_t *__restrict__ keys,
                                                                uint64_t n, uint64_t salt,
                                                                uint64_t *__restrict__ out) {
    const uint64_t stride = uint64_t(gridDim.x) * 256;
    for (uint64_t j = uint64_t(blockIdx.x) * 256 + threadIdx.x; j < n; j += stride) {
        uint64_t k = keys[j];
        if (ops[j] == CF_OP_INSERT) {
            k += salt;
            k = (k ^ (k >> 30)) * 0xbf58476d1ce4e5b9ull;
            k = (k ^ (k >> 27)) * 0x94d049bb133111ebull;
            k ^= k >> 31;
        }
        out[j] = k;
    }
}

}  // namespace cft

extern "C" {

cf_status cf_tune_geometry(const cf_tune_goal *goal, cf_tune_candidate *cands, uint32_t cap,
                           uint32_t *n_out, cf_params *best, void *stream) {
    using namespace cft;
    if (!goal || !n_out) return fail(CF_EINVAL, "NULL argument");
    const double max_load = goal->max_load == 0.0 ? 0.95 : goal->max_load;
    if (goal->capacity == 0 || !(max_load > 0.0 && max_load <= 1.0) || goal->max_fpr < 0.0 ||
        !(goal->positive_share >= 0.0 && goal->positive_share <= 1.0) || goal->measure > 1 ||
        goal->mix[0] < 0 || goal->mix[1] < 0 || goal->mix[2] < 0 ||
        goal->hash > CF_HASH_XXH64 || goal->evict > CF_EVICT_DFS || goal->placements > 3 ||
        goal->tie_permille > 1000)
        return fail(CF_EINVAL, "bad tuning goal");
    double w[3] = {goal->mix[0], goal->mix[1], goal->mix[2]};
    if (w[0] + w[1] + w[2] == 0.0) w[0] = w[1] = w[2] = 1.0;
    const double wsum = w[0] + w[1] + w[2];
    const uint32_t max_evict =
        goal->max_evict ? goal->max_evict : (goal->evict == CF_EVICT_DFS ? 500u : 128u);
    const uint64_t probe_bytes = goal->probe_bytes ? goal->probe_bytes : (1ull << 30);
    const uint64_t need = uint64_t(std::ceil(double(goal->capacity) / max_load));

    const uint32_t places = goal->placements ? goal->placements : 3u;
    std::vector<cf_tune_candidate> all;
    for (uint32_t pl = 0; pl < 2; ++pl) {
        if (!(places & (1u << pl))) continue;
        for (uint32_t f : kFps)
            for (uint32_t b : kSlots) {
                // XOR needs a power of two (Eq. (3)); the offset policy takes
                // the exact bucket count (Sec. 4.6.2)
                const uint64_t exact = (need + b - 1) / b;
                const uint64_t m = pl == CF_PLACE_XOR ? next_pow2(exact) : exact;
                if (m > (pl == CF_PLACE_XOR ? (1ull << 32) : (1ull << 32) - 1)) continue;
                cf_tune_candidate c{};
                c.params = cf_params{m, b, f, goal->hash, goal->evict, max_evict, 0, goal->seed,
                                     pl, 0};
                c.bytes = cf_table_bytes(&c.params);
                if (!c.bytes) continue;  // not compiled
                c.load = double(goal->capacity) / (double(m) * b);
                c.fpr = pl == CF_PLACE_XOR ? fpr_eq4(f, b, c.load) : fpr_offset(f, b, c.load);
                c.feasible = (goal->max_fpr == 0.0 || c.fpr <= goal->max_fpr) &&
                             (goal->max_bytes == 0 || c.bytes <= goal->max_bytes);
                all.push_back(c);
            }
    }

    if (goal->measure) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return fail(CF_EDEVICE, "no current HIP device");
        hipStream_t st = static_cast<hipStream_t>(stream);
        for (cf_tune_candidate &c : all) {
            if (!c.feasible) continue;
            const uint32_t b = c.params.slots_per_bucket;
            uint64_t mp = c.params.num_buckets;
            while (mp > 1024) {
                cf_params q = c.params;
                q.num_buckets = mp;
                if (cf_table_bytes(&q) <= probe_bytes) break;
                mp >>= 1;
            }
            const uint64_t slots = mp * b;
            uint64_t hi = uint64_t(c.load * double(slots));
            uint64_t band = std::max<uint64_t>(uint64_t(0.02 * double(slots)), 1);
            if (hi < band) hi = band;
            const uint64_t lo = hi - band;
            const uint64_t npos =
                lo ? uint64_t(std::llround(goal->positive_share * double(kQueryKeys))) : 0;
            const ProbeKey key{dev, c.params.fp_bits, b, c.params.hash, c.params.evict,
                               c.params.max_evict, c.params.placement, mp, lo, band, npos,
                               goal->seed};
            ProbeResult pr;
            bool hit = false;
            {
                std::lock_guard<std::mutex> lk(g_mu);
                auto it = g_cache.find(key);
                if (it != g_cache.end()) {
                    pr = it->second;
                    hit = true;
                }
            }
            if (!hit) {
                cf_status rc = probe(c.params, mp, lo, band, npos, goal->seed, st, pr);
                if (rc != CF_OK) return rc;
                std::lock_guard<std::mutex> lk(g_mu);
                g_cache[key] = pr;
            }
            c.probe_buckets = mp;
            c.probe_failures = pr.failures;
            // a geometry whose probe failed insertions cannot hold the
            // capacity at this load
            if (pr.failures) c.feasible = 0;
            double t = 0;
            for (int k = 0; k < 3; ++k) {
                c.rate[k] = pr.rate[k];
                if (w[k] > 0) t += w[k] * (pr.rate[k] > 0 ? 1e9 / pr.rate[k] : 1e30);
            }
            c.ns_per_op = t / wsum;
        }
    }

    // Measured times within the tolerance of the fastest feasible candidate
    // count as equal (run-to-run noise is a few per cent); among those the
    // smallest table wins.
    const bool measured = goal->measure != 0;
    double best_ns = 0;
    for (const cf_tune_candidate &c : all)
        if (c.feasible && c.ns_per_op > 0 && (best_ns == 0 || c.ns_per_op < best_ns))
            best_ns = c.ns_per_op;
    const double tol = (goal->tie_permille ? goal->tie_permille : 50u) / 1000.0;
    const double thr = best_ns * (1.0 + tol);
    std::stable_sort(all.begin(), all.end(),
                     [measured, thr](const cf_tune_candidate &x, const cf_tune_candidate &y) {
                         if (x.feasible != y.feasible) return x.feasible > y.feasible;
                         if (measured) {
                             const bool wx = x.ns_per_op > 0 && x.ns_per_op <= thr;
                             const bool wy = y.ns_per_op > 0 && y.ns_per_op <= thr;
                             if (wx != wy) return wx;
                             if (!wx && x.ns_per_op != y.ns_per_op)
                                 return x.ns_per_op < y.ns_per_op;
                         }
                         if (x.bytes != y.bytes) return x.bytes < y.bytes;
                         if (measured && x.ns_per_op != y.ns_per_op)
                             return x.ns_per_op < y.ns_per_op;
                         if (x.params.slots_per_bucket != y.params.slots_per_bucket)
                             return x.params.slots_per_bucket > y.params.slots_per_bucket;
                         if (x.params.fp_bits != y.params.fp_bits)
                             return x.params.fp_bits < y.params.fp_bits;
                         return x.params.placement < y.params.placement;
                     });
    *n_out = uint32_t(all.size());
    if (cands)
        for (uint32_t k = 0; k < std::min<uint32_t>(cap, uint32_t(all.size())); ++k)
            cands[k] = all[k];
    if (all.empty() || !all[0].feasible) return fail(CF_EINVAL, "no compiled geometry meets the goal");
    if (best) *best = all[0].params;
    return CF_OK;
}

cf_status cf_set_tune(cf_set *set, const uint8_t *d_ops, const uint32_t *d_fids,
                      const uint64_t *d_keys, uint64_t n, const cf_set_shape *shapes,
                      uint32_t nshapes, uint32_t reps, uint32_t flags, cf_set_trial *trials,
                      uint32_t trials_cap, uint32_t *ntrials_out, cf_set_shape *out,
                      uint64_t *failures_out, void *stream) {
    using namespace cft;
    if (!set || (n && (!d_ops || !d_fids || !d_keys))) return fail(CF_EINVAL, "NULL argument");
    if (flags & ~uint32_t(CF_SET_TUNE_EAGER)) return fail(CF_EINVAL, "unknown flags");
    const bool eager = (flags & CF_SET_TUNE_EAGER) != 0 || n == 0;
    cf_set_shape keep{};
    (void)cf_set_get_shape(set, &keep);
    std::vector<cf_set_shape> cand;
    if (shapes) {
        cand.assign(shapes, shapes + nshapes);
    } else {
        // the class chains on one stream and on the set's current streams
        std::vector<uint32_t> streams{1u};
        if (keep.streams != 1) streams.push_back(keep.streams);
        for (uint32_t l : streams)
            for (uint32_t w : {0u, 1u})
                for (uint32_t c : {512u, 1024u, 2048u, 4096u})
                    cand.push_back(cf_set_shape{c, l, 0, 0, 0, w, 0});
        // one launch per phase: available exactly when the persistent form is
        if (cf_set_persistent_capacity(set, 256) > 0)
            for (uint32_t w : {0u, 1u})
                for (uint32_t c : {512u, 1024u, 2048u, 4096u})
                    cand.push_back(cf_set_shape{c, keep.streams, 0, 0, 0, w, 1});
        for (uint32_t blk : {256u, 512u}) {
            const uint32_t fit = cf_set_persistent_capacity(set, blk);
            std::vector<uint32_t> per;
            for (uint32_t k : {1u, 2u, fit})
                if (k >= 1 && k <= fit && std::find(per.begin(), per.end(), k) == per.end())
                    per.push_back(k);
            for (uint32_t w : {0u, 1u})
                for (uint32_t k : per)
                    for (uint32_t c : {1024u, 2048u, 4096u})
                        cand.push_back(cf_set_shape{c, keep.streams, 1, blk, k, w, 0});
        }
    }
    if (cand.empty()) return fail(CF_EINVAL, "no candidate shapes");
    if (reps == 0) reps = 3;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint32_t nf = cfs::filter_count(set);
    std::vector<uint64_t> f0(nf), f1(nf);
    cf_status rc = cf_set_failures(set, f0.data(), stream);
    if (rc != CF_OK) return rc;
    if (hipStreamSynchronize(st) != hipSuccess) return fail(CF_EDEVICE, "stream failed");
    DevBuf res, undo, fresh, dn;
    if (!res.alloc(n) || !undo.alloc(n) || !fresh.alloc(n * sizeof(uint64_t)) ||
        !dn.alloc(sizeof(uint64_t)))
        return fail(CF_ENOMEM, "cannot allocate tuning buffers");
    if (hipMemcpy(dn.p, &n, sizeof(n), hipMemcpyHostToDevice) != hipSuccess)
        return fail(CF_EDEVICE, "tuning buffer copy failed");
    auto *r = static_cast<uint8_t *>(res.p);
    auto *u = static_cast<uint8_t *>(undo.p);
    auto *fk = static_cast<uint64_t *>(fresh.p);
    Events ev;
    if (!ev.create()) return fail(CF_EDEVICE, "cannot create events");
    const int grid = int(std::clamp<uint64_t>((n + 255) / 256, 1, 4096));
    uint64_t executions = 0;
    cf_graph *graph = nullptr;  // the candidate's captured batch (graph timing)
    // One execution and its undo; timed = the execution alone, as a launch of
    // the candidate's captured graph or (eager) as cf_set_execute.  Every
    // execution inserts fresh keys (fresh_insert_keys_kernel, a new salt each
    // time), so each one meets the tables as the batch's own new keys would.
    auto trial = [&](float *ms) -> cf_status {
        if (n) {
            const uint64_t salt = (++executions) * 0x9e3779b97f4a7c15ull;
            fresh_insert_keys_kernel<<<grid, 256, 0, st>>>(d_ops, d_keys, n, salt, fk);
            if (hipGetLastError() != hipSuccess) return fail(CF_EDEVICE, "key launch failed");
        }
        (void)hipEventRecord(ev.e[0], st);
        cf_status s = graph ? cf_graph_launch(graph, stream)
                            : cf_set_execute(set, d_ops, d_fids, fk, n, r, stream);
        if (s != CF_OK) return s;
        (void)hipEventRecord(ev.e[1], st);
        if (n) {
            undo_ops_kernel<<<grid, 256, 0, st>>>(d_ops, r, n, u);
            if (hipGetLastError() != hipSuccess) return fail(CF_EDEVICE, "undo launch failed");
            // The undo's results overwrite r; the execution's are no longer needed.
            if ((s = cf_set_execute(set, u, d_fids, fk, n, r, stream)) != CF_OK) return s;
        }
        if (hipEventSynchronize(ev.e[1]) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
            return fail(CF_EDEVICE, "tuning batch failed");
        (void)hipEventElapsedTime(ms, ev.e[0], ev.e[1]);
        return CF_OK;
    };
    // After a failure: the caller's shape back, and the error of the failure.
    auto bail = [&](cf_status s) {
        const std::string msg = cf_last_error();
        if (graph) (void)cf_graph_destroy(graph);
        graph = nullptr;
        (void)cf_set_set_shape(set, &keep);
        return fail(s, "%s", msg.c_str());
    };
    size_t best = 0;
    double best_ms = 1e300;
    for (size_t k = 0; k < cand.size(); ++k) {
        if ((rc = cf_set_set_shape(set, &cand[k])) != CF_OK) return bail(rc);
        if (!eager &&
            (rc = cf_set_graph_create(set, d_ops, d_fids, fk, static_cast<uint64_t *>(dn.p), r,
                                      &graph)) != CF_OK)
            return bail(rc);
        float warm = 0;
        if ((rc = trial(&warm)) != CF_OK) return bail(rc);  // first-launch costs out of the way
        std::vector<float> t(reps);
        for (uint32_t i = 0; i < reps; ++i)
            if ((rc = trial(&t[i])) != CF_OK) return bail(rc);
        if (graph) {
            (void)cf_graph_destroy(graph);
            graph = nullptr;
        }
        uint32_t abandoned = 0;
        if ((rc = cf_set_status(set, &abandoned)) != CF_OK) return bail(rc);
        if (abandoned)
            return bail(fail(CF_EDEVICE, "a persistent trial abandoned its batch (%u-thread "
                             "blocks, %u per compute unit)", cand[k].block,
                             cand[k].blocks_per_cu));
        std::sort(t.begin(), t.end());
        const double med = t[reps / 2];
        if (trials && k < trials_cap) {
            cf_set_shape got{};
            (void)cf_set_get_shape(set, &got);
            trials[k] = cf_set_trial{got, med};
        }
        if (med < best_ms) {
            best_ms = med;
            best = k;
        }
    }
    if (ntrials_out) *ntrials_out = uint32_t(cand.size());
    if ((rc = cf_set_set_shape(set, &cand[best])) != CF_OK) return rc;
    if (out) (void)cf_set_get_shape(set, out);
    if ((rc = cf_set_failures(set, f1.data(), stream)) != CF_OK) return rc;
    if (hipStreamSynchronize(st) != hipSuccess) return fail(CF_EDEVICE, "stream failed");
    if (failures_out) {
        uint64_t d = 0;
        for (uint32_t f = 0; f < nf; ++f) d += f1[f] - f0[f];
        *failures_out = d;
    }
    return CF_OK;
}

}  // extern "C"
