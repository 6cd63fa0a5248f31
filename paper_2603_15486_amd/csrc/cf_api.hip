// cf_api.hip -- host side of libcf.so: the C ABI declared in include/cf.h.
//
// Runtime parameters (f, b, hash, eviction policy) select one of a closed set
// of compiled kernel instantiations, in the spirit of Sec. 4.7's single
// compile-time configuration structure: every geometry gets fully unrolled
// bucket code, the caller still picks it at run time.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "cf.h"
#include "cf_error.hpp"
#include "cf_kernels.hpp"
#include "cf_launch.hpp"

using cfk::Counters;
using cfk::kBlock;

namespace {
thread_local std::string g_err;
}  // namespace

namespace cferr {
cf_status fail(cf_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}
}  // namespace cferr

namespace {

using cferr::fail;

cf_status ok() { return CF_OK; }

cf_status check_launch(const char *what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CF_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    return CF_OK;
}

// Batches are processed in chunks whose key indices fit the 32-bit
// eviction queue entries.
constexpr uint64_t kChunk = 1ull << 31;
constexpr uint64_t kDefaultLost = 1ull << 16;

using cfl::Launchers;

bool pick(const cf_params &p, Launchers &out) { return cfl::pick_launchers(p, out); }

bool is_pow2(uint64_t x) { return x && !(x & (x - 1)); }

cf_status validate(const cf_params *p) {
    if (!p) return fail(CF_EINVAL, "params is NULL");
    return cfl::check_params(*p, "");
}

uint64_t table_bytes_of(const cf_params &p) {
    const uint64_t bits = p.num_buckets * uint64_t(p.slots_per_bucket) * p.fp_bits;
    return ((bits + 63) / 64) * 8;
}

// Switch to the filter's device for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool switched = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
            switched = hipSetDevice(dev) == hipSuccess;
        }
    }
    ~DeviceGuard() {
        if (switched) (void)hipSetDevice(prev);
    }
};

}  // namespace

bool cfl::pick_launchers(const cf_params &p, Launchers &out) {
    switch (p.fp_bits) {
        case 8: return pick_launchers_f8(p, out) && pick_insert_f8(p, out);
        case 16: return pick_launchers_f16(p, out) && pick_insert_f16(p, out);
        case 32: return pick_launchers_f32(p, out) && pick_insert_f32(p, out);
        default: return false;
    }
}

cf_status cfl::check_params(const cf_params &p, const char *who) {
    const std::string pre = who && *who ? std::string(who) + ": " : std::string();
    if (p.placement == CF_PLACE_XOR) {
        if (!is_pow2(p.num_buckets) || p.num_buckets > (1ull << 32))
            return fail(CF_EINVAL, "%snum_buckets must be a power of two in [1, 2^32] under "
                        "the XOR placement, got %llu", pre.c_str(),
                        (unsigned long long)p.num_buckets);
    } else if (p.placement == CF_PLACE_OFFSET) {
        if (p.num_buckets == 0 || p.num_buckets >= (1ull << 32))
            return fail(CF_EINVAL, "%snum_buckets must be in [1, 2^32) under the offset "
                        "placement, got %llu", pre.c_str(), (unsigned long long)p.num_buckets);
    } else {
        return fail(CF_EINVAL, "%sunknown placement %u", pre.c_str(), p.placement);
    }
    if (p.hash > CF_HASH_XXH64) return fail(CF_EINVAL, "%sunknown hash %u", pre.c_str(), p.hash);
    if (p.evict > CF_EVICT_DFS)
        return fail(CF_EINVAL, "%sunknown eviction policy %u", pre.c_str(), p.evict);
    const uint32_t b = p.slots_per_bucket, f = p.fp_bits;
    if (!(b == 4 || b == 8 || b == 16 || b == 32))
        return fail(CF_EUNSUPPORTED, "%sslots_per_bucket must be 4, 8, 16 or 32, got %u",
                    pre.c_str(), b);
    if (!(f == 8 || f == 16 || f == 32))
        return fail(CF_EUNSUPPORTED, "%sfp_bits must be 8, 16 or 32, got %u", pre.c_str(), f);
    return CF_OK;
}

struct cf_filter {
    cf_params p;
    int device;
    cfk::Place place;
    uint64_t table_bytes;
    uint64_t nwords;  // words of the geometry's word type covering m buckets
    void *table;
    Counters *ctr;
    unsigned long long *lost_bucket;
    uint32_t *lost_tag;
    uint64_t lost_cap;
    uint32_t *queue;     // eviction queue, one segment per block of the insert grid
    uint64_t queue_cap;
    Launchers L;
    int grid_cap;         // blocks of the query, delete and whole-table launches
    int insert_grid_cap;  // blocks of an insert launch
    bool owns_table;     // false for a table in caller memory (cf_create_in)
};

namespace {

int grid_capped(uint64_t n, int cap) {
    const uint64_t want = (n + kBlock - 1) / kBlock;
    const uint64_t g = want < uint64_t(cap) ? want : uint64_t(cap);
    return int(g ? g : 1);
}
int grid_for(const cf_filter *f, uint64_t n) { return grid_capped(n, f->grid_cap); }
int insert_grid_for(const cf_filter *f, uint64_t n) { return grid_capped(n, f->insert_grid_cap); }

cf_status check_batch(const cf_filter *f, const uint64_t *keys, uint64_t n, const void *out,
                      bool out_required) {
    if (!f) return fail(CF_EINVAL, "filter is NULL");
    if (n == 0) return CF_OK;
    if (!keys) return fail(CF_EINVAL, "keys is NULL with n = %llu", (unsigned long long)n);
    if (reinterpret_cast<uintptr_t>(keys) & 7u) return fail(CF_EINVAL, "keys not 8-byte aligned");
    if (out_required && !out) return fail(CF_EINVAL, "output buffer is NULL");
    return CF_OK;
}

// Queue entries needed for a batch of n keys: one segment per block, each as
// long as the keys the block can see in its grid-stride loop.
uint64_t queue_need(const cf_filter *f, uint64_t len) {
    const uint64_t grid = uint64_t(insert_grid_for(f, len));
    const uint64_t per = grid * kBlock;
    return grid * (((len + per - 1) / per) * kBlock);
}

cf_status grow_queue(cf_filter *f, uint64_t n, hipStream_t s) {
    const uint64_t want = queue_need(f, n < kChunk ? n : kChunk);
    if (want <= f->queue_cap) return CF_OK;
    if (s) (void)hipStreamSynchronize(s);
    (void)hipDeviceSynchronize();
    if (f->queue) (void)hipFree(f->queue);
    f->queue = nullptr;
    f->queue_cap = 0;
    if (hipMalloc(&f->queue, want * sizeof(uint32_t)) != hipSuccess) {
        (void)hipGetLastError();
        f->queue = nullptr;
        return fail(CF_ENOMEM, "cannot allocate eviction queue of %llu entries",
                    (unsigned long long)want);
    }
    f->queue_cap = want;
    return CF_OK;
}

// Eviction queue of cf_insert_noalloc: a fixed array that the library keeps
// on every GPU it runs on for the life of the process, so that call needs no
// allocation.  In host code the name is only a stand-in for the symbol: every
// launch gets the per-device address that noalloc_queue looks up.
constexpr uint64_t kNoallocQueue = CF_NOALLOC_MAX_KEYS;
constexpr int kNoallocDevices = 64;
static __device__ __align__(256) uint32_t scratch[kNoallocQueue];

// Address of this device's copy of `scratch`, looked up once per device with
// that device current (the caller's DeviceGuard); nullptr if the lookup fails.
uint32_t *noalloc_queue(int device) {
    static std::mutex mu;
    static uint32_t *addr[kNoallocDevices] = {};
    if (device < 0 || device >= kNoallocDevices) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        addr[device] = static_cast<uint32_t *>(p);
    }
    return addr[device];
}

}  // namespace

extern "C" {

uint64_t cf_table_bytes(const cf_params *params) {
    if (validate(params) != CF_OK) return 0;
    return table_bytes_of(*params);
}

// cf_create and cf_create_in: the table is allocated here when table is
// NULL, else it is the caller's buffer.
static cf_status create_impl(const cf_params *params, void *table, cf_filter **out) {
    cf_filter *f = new (std::nothrow) cf_filter();
    if (!f) return fail(CF_ENOMEM, "host allocation failed");
    f->p = *params;
    if (!pick(f->p, f->L)) {
        delete f;
        return fail(CF_EUNSUPPORTED, "no kernels for f=%u b=%u", params->fp_bits,
                    params->slots_per_bucket);
    }
    if (hipGetDevice(&f->device) != hipSuccess) {
        delete f;
        return fail(CF_EDEVICE, "no current HIP device");
    }
    f->place = cfl::make_place(*params);
    f->table_bytes = table_bytes_of(*params);
    f->nwords = params->num_buckets * f->L.words_per_bucket;
    f->lost_cap = params->lost_capacity ? params->lost_capacity : kDefaultLost;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, f->device) !=
            hipSuccess ||
        cus <= 0)
        cus = 256;
    // Launch shape, measured on the 4 GiB filter at load 0.94-0.95: query and
    // delete launches are fastest with one key per thread (up to 1024 blocks
    // per compute unit, then grid-stride), inserts with 128 blocks per
    // compute unit (fewer keys per block shorten each block's eviction tail;
    // still fewer leave too few keys to overlap it with).
    f->grid_cap = cus * 1024;
    f->insert_grid_cap = cus * 128;
    if (const char *env = getenv("CF_GRID_PER_CU")) {
        const int v = atoi(env);
        if (v > 0 && v <= 1024) f->grid_cap = f->insert_grid_cap = cus * v;
    }
    f->owns_table = table == nullptr;
    f->table = table;
    bool okall = (table || hipMalloc(&f->table, f->table_bytes) == hipSuccess) &&
                 hipMalloc(&f->ctr, sizeof(Counters)) == hipSuccess &&
                 hipMalloc(&f->lost_bucket, f->lost_cap * sizeof(unsigned long long)) ==
                     hipSuccess &&
                 hipMalloc(&f->lost_tag, f->lost_cap * sizeof(uint32_t)) == hipSuccess;
    if (okall)
        okall = hipMemset(f->table, 0, f->table_bytes) == hipSuccess &&
                hipMemset(f->ctr, 0, sizeof(Counters)) == hipSuccess &&
                hipDeviceSynchronize() == hipSuccess;
    if (!okall) {
        (void)hipGetLastError();
        cf_destroy(f);
        return fail(CF_ENOMEM, "cannot allocate a %llu-byte table",
                    (unsigned long long)table_bytes_of(*params));
    }
    *out = f;
    return ok();
}

cf_status cf_create(const cf_params *params, cf_filter **out) {
    if (!out) return fail(CF_EINVAL, "out is NULL");
    *out = nullptr;
    cf_status st = validate(params);
    if (st != CF_OK) return st;
    return create_impl(params, nullptr, out);
}

cf_status cf_create_in(const cf_params *params, void *d_table, uint64_t nbytes,
                       cf_filter **out) {
    if (!out) return fail(CF_EINVAL, "out is NULL");
    *out = nullptr;
    cf_status st = validate(params);
    if (st != CF_OK) return st;
    if (!d_table) return fail(CF_EINVAL, "table buffer is NULL");
    if (reinterpret_cast<uintptr_t>(d_table) & 15u)
        return fail(CF_EINVAL, "table buffer not 16-byte aligned");
    if (nbytes < table_bytes_of(*params))
        return fail(CF_EINVAL, "table buffer of %llu bytes, %llu needed",
                    (unsigned long long)nbytes, (unsigned long long)table_bytes_of(*params));
    return create_impl(params, d_table, out);
}

cf_status cf_destroy(cf_filter *f) {
    if (!f) return CF_OK;
    DeviceGuard g(f->device);
    (void)hipDeviceSynchronize();
    if (f->table && f->owns_table) (void)hipFree(f->table);
    if (f->ctr) (void)hipFree(f->ctr);
    if (f->lost_bucket) (void)hipFree(f->lost_bucket);
    if (f->lost_tag) (void)hipFree(f->lost_tag);
    if (f->queue) (void)hipFree(f->queue);
    delete f;
    return CF_OK;
}

cf_status cf_reserve(cf_filter *f, uint64_t max_batch) {
    if (!f) return fail(CF_EINVAL, "filter is NULL");
    DeviceGuard g(f->device);
    return grow_queue(f, max_batch, nullptr);
}

cf_status cf_insert(cf_filter *f, const uint64_t *keys, uint64_t n, uint8_t *okv,
                    uint32_t *kicks, void *stream) {
    cf_status st = check_batch(f, keys, n, nullptr, false);
    if (st != CF_OK || n == 0) return st;
    DeviceGuard g(f->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    st = grow_queue(f, n, s);
    if (st != CF_OK) return st;
    const cfk::LostLog log{f->lost_bucket, f->lost_tag, f->lost_cap};
    for (uint64_t off = 0; off < n; off += kChunk) {
        const uint64_t len = (n - off) < kChunk ? (n - off) : kChunk;
        const int grid = insert_grid_for(f, len);
        const uint64_t per = uint64_t(grid) * kBlock;
        const uint64_t seg = ((len + per - 1) / per) * kBlock;
        f->L.ins(f->table, f->place, keys + off, len, okv ? okv + off : nullptr,
                 kicks ? kicks + off : nullptr, f->ctr, f->queue, seg, log, f->p.max_evict,
                 f->p.seed, grid, s);
        st = check_launch("insert");
        if (st != CF_OK) return st;
    }
    return ok();
}

// cf_insert with the fixed queue above in place of the filter's own, which
// cf_insert may have to grow: no device allocation, one launch.
cf_status cf_insert_noalloc(cf_filter *f, const uint64_t *keys, uint64_t n, uint8_t *okv,
                            uint32_t *kicks, void *stream) {
    cf_status st = check_batch(f, keys, n, nullptr, false);
    if (st != CF_OK || n == 0) return st;
    if (n > kNoallocQueue)
        return fail(CF_EINVAL, "cf_insert_noalloc: n = %llu keys exceeds its limit of %llu",
                    (unsigned long long)n, (unsigned long long)kNoallocQueue);
    DeviceGuard g(f->device);
    const uint64_t need = queue_need(f, n);
    if (need > kNoallocQueue)
        return fail(CF_EINVAL,
                    "cf_insert_noalloc: the launch shape needs %llu queue entries, the fixed "
                    "queue holds %llu",
                    (unsigned long long)need, (unsigned long long)kNoallocQueue);
    uint32_t *q = noalloc_queue(f->device);
    if (!q)
        return fail(CF_EDEVICE, "cf_insert_noalloc: no address for the fixed queue on device %d",
                    f->device);
    const int grid = insert_grid_for(f, n);
    const uint64_t per = uint64_t(grid) * kBlock;
    const uint64_t seg = ((n + per - 1) / per) * kBlock;
    const cfk::LostLog log{f->lost_bucket, f->lost_tag, f->lost_cap};
    f->L.ins(f->table, f->place, keys, n, okv, kicks, f->ctr, q, seg, log, f->p.max_evict,
             f->p.seed, grid, static_cast<hipStream_t>(stream));
    return check_launch("insert (fixed queue)");
}

cf_status cf_query(cf_filter *f, const uint64_t *keys, uint64_t n, uint8_t *found,
                   void *stream) {
    cf_status st = check_batch(f, keys, n, found, true);
    if (st != CF_OK || n == 0) return st;
    DeviceGuard g(f->device);
    f->L.query(f->table, f->place, keys, n, found, grid_for(f, n),
               static_cast<hipStream_t>(stream));
    return check_launch("query");
}

cf_status cf_delete(cf_filter *f, const uint64_t *keys, uint64_t n, uint8_t *okv,
                    void *stream) {
    cf_status st = check_batch(f, keys, n, nullptr, false);
    if (st != CF_OK || n == 0) return st;
    DeviceGuard g(f->device);
    f->L.del(f->table, f->place, keys, n, okv, f->ctr, grid_for(f, n),
             static_cast<hipStream_t>(stream));
    return check_launch("delete");
}

cf_status cf_count(cf_filter *f, uint64_t *out, void *stream) {
    if (!f || !out) return fail(CF_EINVAL, "NULL argument");
    DeviceGuard g(f->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    cfk::sum_counts_kernel<<<1, 64, 0, s>>>(f->ctr);
    cf_status st = check_launch("count");
    if (st != CF_OK) return st;
    if (hipMemcpyAsync(out, &f->ctr->total, sizeof(uint64_t), hipMemcpyDefault, s) !=
        hipSuccess)
        return fail(CF_EDEVICE, "count copy: %s", hipGetErrorString(hipGetLastError()));
    return ok();
}

cf_status cf_failures(cf_filter *f, uint64_t *out, void *stream) {
    if (!f || !out) return fail(CF_EINVAL, "NULL argument");
    DeviceGuard g(f->device);
    if (hipMemcpyAsync(out, &f->ctr->failures, sizeof(uint64_t), hipMemcpyDefault,
                       static_cast<hipStream_t>(stream)) != hipSuccess)
        return fail(CF_EDEVICE, "failures copy: %s", hipGetErrorString(hipGetLastError()));
    return ok();
}

cf_status cf_lost(cf_filter *f, uint64_t *buckets, uint32_t *tags, uint64_t cap,
                  uint64_t *n_out) {
    if (!f || !n_out || (cap && (!buckets || !tags))) return fail(CF_EINVAL, "NULL argument");
    DeviceGuard g(f->device);
    if (hipDeviceSynchronize() != hipSuccess)
        return fail(CF_EDEVICE, "synchronise: %s", hipGetErrorString(hipGetLastError()));
    unsigned long long total = 0;
    if (hipMemcpy(&total, &f->ctr->failures, sizeof(total), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(CF_EDEVICE, "lost count copy failed");
    uint64_t n = total < f->lost_cap ? total : f->lost_cap;
    if (n > cap) n = cap;
    if (n) {
        if (hipMemcpy(buckets, f->lost_bucket, n * sizeof(uint64_t), hipMemcpyDeviceToHost) !=
                hipSuccess ||
            hipMemcpy(tags, f->lost_tag, n * sizeof(uint32_t), hipMemcpyDeviceToHost) !=
                hipSuccess)
            return fail(CF_EDEVICE, "lost log copy failed");
    }
    *n_out = n;
    return ok();
}

cf_status cf_export(cf_filter *f, void *dst, uint64_t nbytes, void *stream) {
    if (!f || !dst) return fail(CF_EINVAL, "NULL argument");
    if (nbytes != f->table_bytes)
        return fail(CF_EINVAL, "nbytes %llu != table bytes %llu", (unsigned long long)nbytes,
                    (unsigned long long)f->table_bytes);
    DeviceGuard g(f->device);
    if (hipMemcpyAsync(dst, f->table, nbytes, hipMemcpyDefault,
                       static_cast<hipStream_t>(stream)) != hipSuccess)
        return fail(CF_EDEVICE, "export copy: %s", hipGetErrorString(hipGetLastError()));
    return ok();
}

cf_status cf_import(cf_filter *f, const void *src, uint64_t nbytes, void *stream) {
    if (!f || !src) return fail(CF_EINVAL, "NULL argument");
    if (nbytes != f->table_bytes)
        return fail(CF_EINVAL, "nbytes %llu != table bytes %llu", (unsigned long long)nbytes,
                    (unsigned long long)f->table_bytes);
    DeviceGuard g(f->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(f->table, src, nbytes, hipMemcpyDefault, s) != hipSuccess)
        return fail(CF_EDEVICE, "import copy: %s", hipGetErrorString(hipGetLastError()));
    cfk::clear_counters_kernel<<<1, 64, 0, s>>>(f->ctr);
    cf_status st = check_launch("import (clear)");
    if (st != CF_OK) return st;
    f->L.recount(f->table, f->nwords, f->ctr, grid_for(f, f->nwords), s);
    return check_launch("import (recount)");
}

cf_status cf_reset(cf_filter *f, void *stream) {
    if (!f) return fail(CF_EINVAL, "filter is NULL");
    DeviceGuard g(f->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const uint64_t n64 = f->table_bytes / 8;
    cfk::zero_words_kernel<<<grid_for(f, n64), kBlock, 0, s>>>(static_cast<uint64_t *>(f->table),
                                                               n64);
    cf_status st = check_launch("reset (table)");
    if (st != CF_OK) return st;
    cfk::clear_counters_kernel<<<1, 64, 0, s>>>(f->ctr);
    return check_launch("reset (counters)");
}

cf_status cf_get_params(const cf_filter *f, cf_params *out) {
    if (!f || !out) return fail(CF_EINVAL, "NULL argument");
    *out = f->p;
    return CF_OK;
}

const char *cf_last_error(void) { return g_err.c_str(); }

}  // extern "C"
