// Plan cache of the MPK library: plans keyed by the sparsity pattern of their
// matrix (a 128-bit hash of n, the row pointers and the column indices) and by
// the options that shape the plan.  The paper amortises its preprocessing (BFS
// levels, level groups) over many calls on one pattern (Sec. 6); here a
// request for a pattern already planned returns that plan, and new values of
// the same pattern only refill and re-upload the matrix values.  The cache
// owns its plans and their device buffers (one allocation per plan, made when
// a pattern is first planned), within a byte budget; plans not in use are
// evicted least recently used first.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"
#include "planner.h"

namespace {

struct Entry {
    uint64_t key[2] = {0, 0};
    uint64_t vals[2] = {0, 0};  // hash of the values last uploaded
    int32_t n = 0;
    int64_t nnz = 0;
    mpk_options opt{};
    mpk_plan_t plan = nullptr;
    void* dev = nullptr;
    size_t bytes = 0;
    int32_t users = 0;  // gets not yet released
    uint64_t stamp = 0;
};

void value_hash(int64_t nnz, const double* val, uint64_t out[2]) {
    uint64_t a = 0x452821E638D01377ull, b = 0xBE5466CF34E90C6Cull;
    for (int64_t e = 0; e < nnz; ++e) {
        uint64_t w;
        std::memcpy(&w, val + e, 8);
        a = (a ^ w) * 0x9E3779B97F4A7C15ull;
        a ^= a >> 29;
        b = (b + w) * 0xBF58476D1CE4E5B9ull;
        b ^= b >> 31;
    }
    out[0] = a;
    out[1] = b;
}

}  // namespace

struct mpk_plan_cache_s {
    int device = 0;
    size_t budget = 0, used = 0;
    uint64_t clock = 0;
    std::vector<Entry> entries;
    std::mutex mu;
    int64_t hits = 0, value_updates = 0, misses = 0;
};

MPK_API mpk_status mpk_plan_cache_create(size_t device_bytes, mpk_plan_cache_t* out) {
    if (!out) return mpk::set_error(MPK_ERR_ARG, "out is null");
    *out = nullptr;
    auto* c = new (std::nothrow) mpk_plan_cache_s;
    if (!c) return mpk::set_error(MPK_ERR_NOMEM, "out of host memory");
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return mpk::set_error(MPK_ERR_HIP, "no current device");
    }
    c->budget = device_bytes;
    *out = c;
    return MPK_OK;
}

MPK_API mpk_status mpk_plan_cache_get(mpk_plan_cache_t c, int32_t n, const int32_t* rowptr, const int32_t* col,
                                      const double* val, const mpk_options* opt, void* stream, mpk_plan_t* plan,
                                      int32_t* outcome) {
    if (!c || !plan) return mpk::set_error(MPK_ERR_ARG, "null argument");
    *plan = nullptr;
    if (outcome) *outcome = -1;
    if (n < 0 || !rowptr || (n > 0 && rowptr[n] > 0 && (!col || !val)))
        return mpk::set_error(MPK_ERR_ARG, "bad CSR arguments");
    std::string why = mpk::validate_csr(n, rowptr, col);
    if (!why.empty()) return mpk::set_error(MPK_ERR_CSR, "%s", why.c_str());
    mpk_options o{};
    if (opt) o = *opt;
    const int64_t nnz = n > 0 ? rowptr[n] : 0;
    uint64_t key[2], vh[2];
    mpk::pattern_hash(n, rowptr, col, key);
    value_hash(nnz, val, vh);
    std::lock_guard<std::mutex> lk(c->mu);
    for (auto& e : c->entries)
        if (e.key[0] == key[0] && e.key[1] == key[1] && e.n == n && e.nnz == nnz &&
            std::memcmp(&e.opt, &o, sizeof o) == 0) {
            int32_t how = 0;
            if (e.vals[0] != vh[0] || e.vals[1] != vh[1]) {
                if (e.users > 0)
                    return mpk::set_error(MPK_ERR_STATE,
                                          "the cached plan of this pattern is in use with other values");
                mpk_status s = mpk_update_values(e.plan, n, rowptr, col, val, stream);
                if (s != MPK_OK) return s;
                e.vals[0] = vh[0];
                e.vals[1] = vh[1];
                how = 1;
                ++c->value_updates;
            } else {
                ++c->hits;
            }
            ++e.users;
            e.stamp = ++c->clock;
            *plan = e.plan;
            if (outcome) *outcome = how;
            return MPK_OK;
        }
    // a new pattern: plan, make room (least recently used plans not in use), upload
    mpk_plan_t p = nullptr;
    size_t bytes = 0;
    mpk_status s = mpk_build_levels(n, rowptr, col, val, &o, &p, &bytes);
    if (s != MPK_OK) return s;
    bytes = std::max<size_t>(bytes, 256);
    if (bytes > c->budget) {
        mpk_destroy(p);
        return mpk::set_error(MPK_ERR_NOMEM, "the plan needs %zu device bytes, the cache holds %zu", bytes,
                              c->budget);
    }
    while (c->used + bytes > c->budget) {
        int victim = -1;
        for (int i = 0; i < (int)c->entries.size(); ++i)
            if (c->entries[i].users == 0 && (victim < 0 || c->entries[i].stamp < c->entries[victim].stamp))
                victim = i;
        if (victim < 0) {
            mpk_destroy(p);
            return mpk::set_error(MPK_ERR_NOMEM, "the cache is full of plans in use");
        }
        Entry& v = c->entries[victim];
        mpk_destroy(v.plan);
        hipFree(v.dev);
        c->used -= v.bytes;
        c->entries.erase(c->entries.begin() + victim);
    }
    Entry e;
    hipError_t he = hipSetDevice(c->device);
    if (he == hipSuccess) he = hipMalloc(&e.dev, bytes);
    if (he != hipSuccess) {
        mpk_destroy(p);
        return mpk::set_error(MPK_ERR_HIP, "plan memory: %s", hipGetErrorString(he));
    }
    s = mpk_upload(p, e.dev, bytes, stream);
    if (s != MPK_OK) {
        mpk_destroy(p);
        hipFree(e.dev);
        return s;
    }
    std::memcpy(e.key, key, sizeof key);
    std::memcpy(e.vals, vh, sizeof vh);
    e.n = n;
    e.nnz = nnz;
    e.opt = o;
    e.plan = p;
    e.bytes = bytes;
    e.users = 1;
    e.stamp = ++c->clock;
    c->entries.push_back(e);
    c->used += bytes;
    ++c->misses;
    *plan = p;
    if (outcome) *outcome = 2;
    return MPK_OK;
}

MPK_API mpk_status mpk_plan_cache_release(mpk_plan_cache_t c, mpk_plan_t plan) {
    if (!c || !plan) return mpk::set_error(MPK_ERR_ARG, "null argument");
    std::lock_guard<std::mutex> lk(c->mu);
    for (auto& e : c->entries)
        if (e.plan == plan) {
            if (e.users <= 0) return mpk::set_error(MPK_ERR_STATE, "the plan was not taken from the cache");
            --e.users;
            return MPK_OK;
        }
    return mpk::set_error(MPK_ERR_ARG, "the plan does not belong to this cache");
}

MPK_API mpk_status mpk_plan_cache_stats(mpk_plan_cache_t c, int32_t* plans, size_t* bytes_used, int64_t* hits,
                                        int64_t* value_updates, int64_t* misses) {
    if (!c) return mpk::set_error(MPK_ERR_ARG, "null cache");
    std::lock_guard<std::mutex> lk(c->mu);
    if (plans) *plans = (int32_t)c->entries.size();
    if (bytes_used) *bytes_used = c->used;
    if (hits) *hits = c->hits;
    if (value_updates) *value_updates = c->value_updates;
    if (misses) *misses = c->misses;
    return MPK_OK;
}

MPK_API void mpk_plan_cache_destroy(mpk_plan_cache_t c) {
    if (!c) return;
    hipSetDevice(c->device);
    for (auto& e : c->entries) {
        mpk_destroy(e.plan);
        hipFree(e.dev);
    }
    delete c;
}
