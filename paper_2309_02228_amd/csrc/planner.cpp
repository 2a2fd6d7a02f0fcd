// Host planner: level structure (Sec. 3), level-order permutation, SELL-64
// layout, chunk partition over the XCDs and the dependency lists that drive
// the blocked kernel.
#include "planner.h"

#include <algorithm>
#include <atomic>
#include <climits>
#include <cstdio>
#include <numeric>
#include <thread>

namespace mpk {

namespace {

// Threads for building host tables: the machine's hardware threads, at most 16.
constexpr int64_t kRowGrain = 1 << 16;  // rows per thread at least

int host_threads() {
    const unsigned h = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(h, 16u));
}

// Runs fn(i0, i1) over [0, n) cut into contiguous ranges whose bounds are
// multiples of `align`, one per thread and at least `grain` items each.  The
// ranges must write disjoint memory; results do not depend on the thread count.
template <typename Fn>
void parallel_ranges(int64_t n, int64_t align, int64_t grain, Fn fn) {
    const int nt = (int)std::min<int64_t>(host_threads(), std::max<int64_t>(1, n / grain));
    const int64_t per = ((n + nt - 1) / nt + align - 1) / align * align;
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t) {
        const int64_t i0 = std::min(n, t * per), i1 = std::min(n, (t + 1) * per);
        if (i0 < i1) pool.emplace_back(fn, t, i0, i1);
    }
    fn(0, (int64_t)0, std::min(n, per));
    for (auto& th : pool) th.join();
}

// A team of threads running one function together, with a barrier for
// lock-step phases (the levels of a breadth-first search).
class Team {
public:
    explicit Team(int nt) : nt_(nt) {}
    int size() const { return nt_; }
    template <typename Fn>
    void run(Fn fn) {  // fn(thread index)
        std::vector<std::thread> pool;
        for (int t = 1; t < nt_; ++t) pool.emplace_back(fn, t);
        fn(0);
        for (auto& th : pool) th.join();
    }
    void barrier() {
        const int g = gen_.load(std::memory_order_acquire);
        if (count_.fetch_add(1, std::memory_order_acq_rel) == nt_ - 1) {
            count_.store(0, std::memory_order_relaxed);
            gen_.fetch_add(1, std::memory_order_release);
        } else {
            for (int spin = 0; gen_.load(std::memory_order_acquire) == g; ++spin)
                if (spin >= 4096) std::this_thread::yield();
        }
    }

private:
    int nt_;
    std::atomic<int> count_{0}, gen_{0};
};

}  // namespace

std::string validate_csr(int32_t n, const int32_t* rowptr, const int32_t* col) {
    char buf[160];
    if (rowptr[0] != 0) return "rowptr[0] must be 0";
    // the first offending row, as a row-by-row scan would find it: the first row
    // whose pointer decreases bounds the rows whose columns can be read, and the
    // smallest row with a bad column below it is described instead if there is one
    int32_t nrows = n;
    for (int32_t i = 0; i < n; ++i)
        if (rowptr[i + 1] < rowptr[i]) {
            nrows = i;
            break;
        }
    std::atomic<int64_t> bad{INT64_MAX};
    parallel_ranges(nrows, 1, kRowGrain, [&](int, int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1 && i < bad.load(std::memory_order_relaxed); ++i)
            for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
                if (col[e] < 0 || col[e] >= n || (e > rowptr[i] && col[e] <= col[e - 1])) {
                    int64_t cur = bad.load();
                    while (i < cur && !bad.compare_exchange_weak(cur, i)) {
                    }
                    return;
                }
    });
    if (bad.load() == INT64_MAX) {
        if (nrows == n) return "";
        snprintf(buf, sizeof buf, "rowptr decreases at row %d", nrows);
        return buf;
    }
    const int32_t i = (int32_t)bad.load();
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
        if (col[e] < 0 || col[e] >= n) {
            snprintf(buf, sizeof buf, "column %d out of range in row %d", col[e], i);
            return buf;
        }
        if (e > rowptr[i] && col[e] <= col[e - 1]) {
            snprintf(buf, sizeof buf, "columns not strictly ascending in row %d", i);
            return buf;
        }
    }
    return "";
}

namespace {

// Large index arrays that are written in full right after they are sized.
using Ints = std::vector<int32_t, NoInit<int32_t>>;

// Per-thread output list, on its own cache lines (its size field is written at
// every append).
struct alignas(64) Local {
    std::vector<int32_t> v;
};

// Undirected graph of pattern(A) + pattern(A^T), self-loops dropped, each
// neighbour list sorted and free of duplicates.  The counts and the scatter of
// both directions use atomic slots, so the unsorted order inside a row depends
// on the threads; sorting each row makes the result independent of them.
void symmetric_pattern(int32_t n, const int32_t* rowptr, const int32_t* col,
                       std::vector<int64_t>& ptr, Ints& adj) {
    // a structurally symmetric pattern is its own union with the transpose: the
    // rows without their diagonal entries, already sorted (columns ascend)
    std::atomic<bool> sym{true};
    parallel_ranges(n, 1, kRowGrain, [&](int, int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1 && sym.load(std::memory_order_relaxed); ++i)
            for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
                const int32_t j = col[e];
                if (!std::binary_search(col + rowptr[j], col + rowptr[j + 1], (int32_t)i)) {
                    sym.store(false, std::memory_order_relaxed);
                    break;
                }
            }
    });
    if (sym.load()) {
        ptr.assign(n + 1, 0);
        parallel_ranges(n, 1, kRowGrain, [&](int, int64_t i0, int64_t i1) {
            for (int64_t i = i0; i < i1; ++i) {
                int64_t k = 0;
                for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) k += col[e] != i;
                ptr[i + 1] = k;
            }
        });
        for (int32_t i = 0; i < n; ++i) ptr[i + 1] += ptr[i];
        adj.resize(ptr[n]);
        parallel_ranges(n, 1, kRowGrain, [&](int, int64_t i0, int64_t i1) {
            for (int64_t i = i0; i < i1; ++i) {
                int64_t k = ptr[i];
                for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
                    if (col[e] != i) adj[k++] = col[e];
            }
        });
        return;
    }
    std::vector<int64_t> cnt(n + 1, 0);
    parallel_ranges(n, 1, kRowGrain, [&](int, int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) {
            int64_t own = 0;
            for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
                if (col[e] != i) {
                    ++own;
                    __atomic_fetch_add(&cnt[col[e] + 1], 1, __ATOMIC_RELAXED);
                }
            __atomic_fetch_add(&cnt[i + 1], own, __ATOMIC_RELAXED);
        }
    });
    for (int32_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    Ints tmp(cnt[n]);  // every entry is written by the scatter
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    parallel_ranges(n, 1, kRowGrain, [&](int, int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i)
            for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
                if (col[e] != i) {
                    tmp[__atomic_fetch_add(&fill[i], 1, __ATOMIC_RELAXED)] = col[e];
                    tmp[__atomic_fetch_add(&fill[col[e]], 1, __ATOMIC_RELAXED)] = (int32_t)i;
                }
    });
    // each row's neighbours sorted and without repeats, then packed
    ptr.assign(n + 1, 0);
    parallel_ranges(n, 1, kRowGrain, [&](int, int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) {
            auto b = tmp.begin() + cnt[i], e = tmp.begin() + cnt[i + 1];
            std::sort(b, e);
            ptr[i + 1] = std::unique(b, e) - b;
        }
    });
    for (int32_t i = 0; i < n; ++i) ptr[i + 1] += ptr[i];
    adj.resize(ptr[n]);
    parallel_ranges(n, 1, kRowGrain, [&](int, int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i)
            std::copy(tmp.begin() + cnt[i], tmp.begin() + cnt[i] + (ptr[i + 1] - ptr[i]), adj.begin() + ptr[i]);
    });
}

// Visited marks of a breadth-first search, one byte per vertex; `claim` is the
// atomic test-and-set of the threaded search.  (A bit per vertex puts 512
// vertices on a cache line, and the threads then contend for the lines.)
struct Marks {
    std::vector<uint8_t> w;
    explicit Marks(int32_t n) : w(n, 0) {}
    bool test(int32_t v) const { return w[v] != 0; }
    void set(int32_t v) { w[v] = 1; }
    bool claim(int32_t v) {
        if (__atomic_load_n(&w[v], __ATOMIC_RELAXED)) return false;
        return __atomic_exchange_n(&w[v], (uint8_t)1, __ATOMIC_RELAXED) == 0;
    }
    void clear(int32_t v) { w[v] = 0; }
};

// Breadth-first search from `root`.  Marks every reached vertex (the caller
// clears them afterwards via `order`), returns the visit order and the start
// of each distance layer inside it.  Layers are expanded by one thread while
// they are small and by a team of threads once a layer holds more than
// kTeamLayer vertices; the layers as sets do not depend on that (only the
// order inside a layer does).
struct Bfs {
    std::vector<int32_t> order;       // vertices by nondecreasing distance
    std::vector<int32_t> layer_ptr;   // layer d = order[layer_ptr[d] .. layer_ptr[d+1])
};

constexpr int64_t kTeamLayer = 4096;

void bfs(const std::vector<int64_t>& ptr, const Ints& adj, int32_t root,
         Marks& seen, Bfs& out) {
    out.order.clear();
    out.layer_ptr.clear();
    out.order.push_back(root);
    seen.set(root);
    out.layer_ptr.push_back(0);
    int64_t f0 = 0, f1 = 1;  // the current layer in `order`
    // one thread while layers are small
    while (f0 < f1 && (f1 - f0 <= kTeamLayer || host_threads() == 1)) {
        for (int64_t t = f0; t < f1; ++t) {
            const int32_t u = out.order[t];
            for (int64_t e = ptr[u]; e < ptr[u + 1]; ++e) {
                const int32_t v = adj[e];
                if (!seen.test(v)) {
                    seen.set(v);
                    out.order.push_back(v);
                }
            }
        }
        f0 = f1;
        f1 = (int64_t)out.order.size();
        out.layer_ptr.push_back((int32_t)f0);
    }
    if (f0 < f1) {  // a team for the rest: each thread expands a slice of the layer
        Team team(host_threads());
        const int nt = team.size();
        std::vector<Local> found(nt);
        team.run([&](int t) {
            for (;;) {
                const int64_t b = f0, e = f1;  // read between barriers
                if (b == e) break;
                auto& mine = found[t].v;
                mine.clear();
                for (int64_t i = b + (e - b) * t / nt; i < b + (e - b) * (t + 1) / nt; ++i) {
                    const int32_t u = out.order[i];
                    for (int64_t k = ptr[u]; k < ptr[u + 1]; ++k) {
                        const int32_t v = adj[k];
                        if (seen.claim(v)) mine.push_back(v);
                    }
                }
                team.barrier();
                if (t == 0) {  // append the next layer
                    for (auto& f : found) out.order.insert(out.order.end(), f.v.begin(), f.v.end());
                    f0 = e;
                    f1 = (int64_t)out.order.size();
                    out.layer_ptr.push_back((int32_t)f0);
                }
                team.barrier();
            }
        });
    }
}

void reset(Marks& seen, const Bfs& b) {
    parallel_ranges((int64_t)b.order.size(), 1, kRowGrain, [&](int, int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) seen.clear(b.order[i]);
    });
}

// George-Liu pseudo-peripheral node of the component containing `start`.
// `br` holds the search from `start` on entry and the search from the
// returned node on exit.
int32_t pseudo_peripheral(const std::vector<int64_t>& ptr, const Ints& adj,
                          int32_t start, Marks& seen, Bfs& br) {
    Bfs bx;
    int32_t r = start;
    for (;;) {
        const int32_t lb = br.layer_ptr[br.layer_ptr.size() - 2];
        const int32_t le = br.layer_ptr.back();
        int32_t x = -1;
        int64_t best = -1;
        for (int32_t t = lb; t < le; ++t) {
            int32_t v = br.order[t];
            int64_t deg = ptr[v + 1] - ptr[v];
            if (x < 0 || deg < best || (deg == best && v < x)) {
                x = v;
                best = deg;
            }
        }
        bfs(ptr, adj, x, seen, bx);
        reset(seen, bx);
        if (bx.layer_ptr.size() > br.layer_ptr.size()) {  // eccentricity grew
            r = x;
            std::swap(br, bx);
            continue;
        }
        return r;
    }
}

// The SELL-64 slots of every permuted row: its entries sorted by permuted
// column.  With `pattern`, the columns (and the GS2 masks) are written too;
// otherwise only the values (a plan of the same pattern with new values).
void fill_sell(HostPlan& P, const int32_t* rowptr, const int32_t* col, const double* val, bool pattern) {
    // rows write disjoint slots: threads take contiguous ranges of chunks and
    // write every slot of them, padding included (0.0 and column -1), so the
    // arrays need no initialisation of their own
    parallel_ranges((int64_t)P.nchunks * kChunkRows, kChunkRows, kRowGrain, [&](int, int64_t i0, int64_t i1) {
        for (int64_t c = i0 / kChunkRows; c < i1 / kChunkRows; ++c) {
            std::fill(P.sell_val.begin() + P.chunk_off[c], P.sell_val.begin() + P.chunk_off[c + 1], 0.0);
            if (pattern)
                std::fill(P.sell_col.begin() + P.chunk_off[c], P.sell_col.begin() + P.chunk_off[c + 1], -1);
        }
        std::vector<std::pair<int32_t, double>> row;
        for (int32_t i = (int32_t)i0; i < (int32_t)std::min<int64_t>(i1, P.n); ++i) {
            int32_t o = P.perm[i];
            row.clear();
            for (int32_t e = rowptr[o]; e < rowptr[o + 1]; ++e)
                row.emplace_back(P.iperm[col[e]], val[e]);
            // columns are distinct, so the order is unique; short rows (the usual
            // case) by insertion, long ones by std::sort
            if (row.size() <= 32) {
                for (size_t j = 1; j < row.size(); ++j) {
                    const auto x = row[j];
                    size_t k = j;
                    for (; k > 0 && row[k - 1].first > x.first; --k) row[k] = row[k - 1];
                    row[k] = x;
                }
            } else {
                std::sort(row.begin(), row.end(),
                          [](const std::pair<int32_t, double>& a, const std::pair<int32_t, double>& b) {
                              return a.first < b.first;
                          });
            }
            const int32_t c = i / kChunkRows, lane = i % kChunkRows;
            for (size_t j = 0; j < row.size(); ++j) {
                int64_t s = P.chunk_off[c] + (int64_t)j * kChunkRows + lane;
                P.sell_val[s] = row[j].second;
                if (!pattern) continue;
                P.sell_col[s] = row[j].first;
                if (P.split_lower) {
                    if (P.perm[row[j].first] < o) P.lmask[i] |= 1u << j;
                    if (row[j].first == i) P.dslot[i] = (int32_t)j;
                }
            }
        }
    });
}

}  // namespace

void refill_values(HostPlan& P, const int32_t* rowptr, const int32_t* col, const double* val) {
    fill_sell(P, rowptr, col, val, false);
}

void pattern_hash(int32_t n, const int32_t* rowptr, const int32_t* col, uint64_t out[2]) {
    // two 64-bit multiply-xorshift chains with different odd multipliers (a
    // 128-bit key): each block of 2^20 words (row pointers, then column indices)
    // is hashed from a seed that depends on its index, and the block keys are
    // then chained in order, so the key does not depend on the thread count
    struct Chain {
        uint64_t a, b;
        void mix(uint64_t w) {
            a = (a ^ w) * 0x9E3779B97F4A7C15ull;
            a ^= a >> 29;
            b = (b + w) * 0xBF58476D1CE4E5B9ull;
            b ^= b >> 31;
        }
    };
    constexpr int64_t kBlock = 1 << 20;
    const int64_t nnz = n > 0 ? rowptr[n] : 0;
    const int64_t words = (int64_t)n + 1 + nnz;
    const int64_t nblocks = (words + kBlock - 1) / kBlock;
    std::vector<Chain> part(nblocks);
    parallel_ranges(nblocks, 1, 4, [&](int, int64_t b0, int64_t b1) {
        for (int64_t k = b0; k < b1; ++k) {
            Chain h{0x243F6A8885A308D3ull ^ (uint64_t)k, 0x13198A2E03707344ull + (uint64_t)k};
            for (int64_t w = k * kBlock; w < std::min(words, (k + 1) * kBlock); ++w)
                h.mix(w <= n ? (uint64_t)(uint32_t)rowptr[w]
                             : 0x5555555555555555ull ^ (uint64_t)(uint32_t)col[w - n - 1]);
            part[k] = h;
        }
    });
    Chain h{0x243F6A8885A308D3ull ^ (uint64_t)n, 0x13198A2E03707344ull + (uint64_t)n};
    for (const Chain& c : part) {
        h.mix(c.a);
        h.mix(c.b);
    }
    out[0] = h.a;
    out[1] = h.b;
}

// Units of G consecutive chunks of each partition's sequence, carried together
// by one worker, and the smallest deadlock-free worker count per block size q
// (D3): bmin[u] = smallest first chunk among units within h unit hops of u; the
// condition for W workers holds iff W > max over unit positions j of
// (j - first position whose first chunk is >= bmin[unit j]), per partition.
static void build_units(const HostPlan& P, int32_t G, Units& U) {
    U.group = G;
    U.ptr.assign(kParts + 1, 0);
    std::vector<int32_t>& unit_ptr = U.ptr;
    std::vector<int32_t> first, unit_of(P.nchunks);
    for (int x = 0; x < kParts; ++x) {
        const int32_t len = P.seq_ptr[x + 1] - P.seq_ptr[x];
        for (int32_t j = 0; j < len; j += G) {
            for (int32_t t = j; t < std::min(len, j + G); ++t)
                unit_of[P.seq[P.seq_ptr[x] + t]] = (int32_t)first.size();
            first.push_back(P.seq[P.seq_ptr[x] + j]);
        }
        unit_ptr[x + 1] = (int32_t)first.size();
    }
    const int32_t nunits = (int32_t)first.size();
    // one record per unit, read by the blocked kernel in a single scalar load
    U.stride = G <= 1 ? 8 : (G == 2 ? 16 : 32);
    U.rec.assign((size_t)nunits * U.stride, 0);
    for (int x = 0; x < kParts; ++x) {
        const int32_t len = P.seq_ptr[x + 1] - P.seq_ptr[x];
        for (int32_t u = unit_ptr[x]; u < unit_ptr[x + 1]; ++u) {
            int32_t* r = U.rec.data() + (size_t)u * U.stride;
            for (int32_t g = 0; g < G; ++g) {
                const int32_t t = (u - unit_ptr[x]) * G + g;
                if (t >= len) {
                    r[5 * g] = -1;
                    continue;
                }
                const int32_t c = P.seq[P.seq_ptr[x] + t];
                r[5 * g + 0] = c;
                r[5 * g + 1] = (int32_t)(P.chunk_off[c] / kChunkRows);
                r[5 * g + 2] = (int32_t)((P.chunk_off[c + 1] - P.chunk_off[c]) / kChunkRows);
            }
        }
    }
    // the units each unit's rows read (its own excluded); the dependency range
    // of the record and the completion words polled come from these lists
    std::vector<int32_t>& udep_ptr = U.dep_ptr;
    udep_ptr.assign(nunits + 1, 0);
    std::vector<int32_t> udep;
    {
        std::vector<int32_t> stamp(nunits, -1), list;
        for (int x = 0; x < kParts; ++x)
            for (int32_t u = unit_ptr[x]; u < unit_ptr[x + 1]; ++u) {
                list.clear();
                stamp[u] = u;
                const int32_t j0 = (u - unit_ptr[x]) * G;
                const int32_t len = P.seq_ptr[x + 1] - P.seq_ptr[x];
                for (int32_t t = j0; t < std::min(len, j0 + G); ++t) {
                    const int32_t c = P.seq[P.seq_ptr[x] + t];
                    for (int32_t e = P.dep_ptr[c]; e < P.dep_ptr[c + 1]; ++e) {
                        const int32_t v = unit_of[P.dep_idx[e]];
                        if (stamp[v] != u) {
                            stamp[v] = u;
                            list.push_back(v);
                        }
                    }
                }
                udep.insert(udep.end(), list.begin(), list.end());
                udep_ptr[u + 1] = (int32_t)udep.size();
            }
    }
    U.dep_idx.resize(udep.size());
    for (size_t e = 0; e < udep.size(); ++e) U.dep_idx[e] = first[udep[e]];
    for (int32_t u = 0; u < nunits; ++u) {
        U.rec[(size_t)u * U.stride + 3] = udep_ptr[u];
        U.rec[(size_t)u * U.stride + 4] = udep_ptr[u + 1];
    }
    U.min_workers.assign(P.p_block + 1, 1);
    std::vector<int32_t> bmin(first), nb(nunits);
    for (int32_t q = 1; q <= P.p_block; ++q) {
        if (q >= 2) {  // one more hop
            for (int32_t u = 0; u < nunits; ++u) {
                int32_t m = bmin[u];
                for (int32_t e = udep_ptr[u]; e < udep_ptr[u + 1]; ++e) m = std::min(m, bmin[udep[e]]);
                nb[u] = m;
            }
            bmin.swap(nb);
        }
        int32_t need = 1;
        for (int x = 0; x < kParts; ++x) {
            const int32_t* f = first.data() + unit_ptr[x];
            const int32_t len = unit_ptr[x + 1] - unit_ptr[x];
            for (int32_t j = 0; j < len; ++j) {
                int32_t lo = (int32_t)(std::lower_bound(f, f + j + 1, bmin[unit_ptr[x] + j]) - f);
                need = std::max(need, j - lo + 1);
            }
        }
        U.min_workers[q] = need;
    }
}

void build_plan(HostPlan& P, int32_t n, const int32_t* rowptr, const int32_t* col,
                const double* val) {
    P.n = n;
    pattern_hash(n, rowptr, col, P.pattern_key);
    P.nnz = n ? rowptr[n] : 0;

    // ---- levels (readings R1-R3) ------------------------------------------
    std::vector<int64_t> ptr;
    Ints adj;
    symmetric_pattern(n, rowptr, col, ptr, adj);
    Marks marks(n);
    P.level_of_row.assign(n, -1);
    P.roots.clear();
    std::vector<char> seen(n, 0);
    Bfs comp, lv;
    int32_t base = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (seen[v]) continue;
        bfs(ptr, adj, v, marks, comp);  // the component of the lowest unvisited row
        bool has_root = P.root_mode == 1 && marks.test(P.root);
        reset(marks, comp);
        int32_t r;
        if (has_root) {
            r = P.root;
            bfs(ptr, adj, r, marks, lv);
            reset(marks, lv);
        } else {  // the component's search is the first step of the root search
            std::swap(lv, comp);
            r = pseudo_peripheral(ptr, adj, v, marks, lv);
        }
        parallel_ranges((int64_t)lv.order.size(), 1, kRowGrain, [&](int, int64_t t0, int64_t t1) {
            int32_t d = (int32_t)(std::upper_bound(lv.layer_ptr.begin(), lv.layer_ptr.end(), (int32_t)t0) -
                                  lv.layer_ptr.begin()) - 1;
            for (int64_t t = t0; t < t1; ++t) {
                while (t >= lv.layer_ptr[d + 1]) ++d;
                P.level_of_row[lv.order[t]] = base + d;
                seen[lv.order[t]] = 1;
            }
        });
        base += (int32_t)lv.layer_ptr.size() - 1;
        P.roots.push_back(r);
    }
    P.nlevels = base;

    // ---- permutation: rows by (level, original index) (R4) ------------------
    // counting sort by level, stable in the row index: each thread counts the
    // rows of a contiguous range per level, and places its rows behind the rows
    // of the same level from lower ranges (serial when the levels are many)
    P.level_ptr.assign(P.nlevels + 1, 0);
    P.level_nnz.assign(P.nlevels, 0);
    P.perm.assign(n, 0);
    P.iperm.assign(n, 0);
    {
        const int64_t nt = (int64_t)P.nlevels * host_threads() <= n ? host_threads() : 1;
        const int64_t per = (n + nt - 1) / std::max<int64_t>(nt, 1);
        std::vector<std::vector<int64_t>> cnt(nt, std::vector<int64_t>(P.nlevels, 0));
        std::vector<std::vector<int64_t>> ent(nt, std::vector<int64_t>(P.nlevels, 0));
        auto range = [&](int64_t t) { return std::make_pair(std::min<int64_t>(n, t * per), std::min<int64_t>(n, (t + 1) * per)); };
        auto each = [&](auto fn) {
            std::vector<std::thread> pool;
            for (int64_t t = 1; t < nt; ++t) pool.emplace_back(fn, t);
            fn((int64_t)0);
            for (auto& th : pool) th.join();
        };
        each([&](int64_t t) {
            for (int64_t i = range(t).first; i < range(t).second; ++i) {
                ++cnt[t][P.level_of_row[i]];
                ent[t][P.level_of_row[i]] += rowptr[i + 1] - rowptr[i];
            }
        });
        // level_ptr, level_nnz and each range's first position per level
        int64_t at = 0;
        for (int32_t l = 0; l < P.nlevels; ++l) {
            for (int64_t t = 0; t < nt; ++t) {
                const int64_t c = cnt[t][l];
                cnt[t][l] = at;
                at += c;
                P.level_nnz[l] += ent[t][l];
            }
            P.level_ptr[l + 1] = (int32_t)at;
        }
        each([&](int64_t t) {
            auto& pos = cnt[t];
            for (int64_t i = range(t).first; i < range(t).second; ++i) {
                const int32_t k = (int32_t)pos[P.level_of_row[i]]++;
                P.perm[k] = (int32_t)i;
                P.iperm[i] = k;
            }
        });
    }

    // ---- SELL-64 layout of P A P^T ------------------------------------------
    P.nchunks = (n + kChunkRows - 1) / kChunkRows;
    P.chunk_off.assign(P.nchunks + 1, 0);
    P.max_width = 0;
    parallel_ranges(P.nchunks, 1, kRowGrain / kChunkRows, [&](int, int64_t c0, int64_t c1) {
        for (int64_t c = c0; c < c1; ++c) {
            int32_t w = 0;
            for (int32_t i = (int32_t)c * kChunkRows; i < std::min<int64_t>(n, (c + 1) * kChunkRows); ++i) {
                int32_t o = P.perm[i];
                w = std::max(w, rowptr[o + 1] - rowptr[o]);
            }
            P.chunk_off[c + 1] = (int64_t)w * kChunkRows;
        }
    });
    for (int32_t c = 0; c < P.nchunks; ++c) {
        P.max_width = std::max(P.max_width, (int32_t)(P.chunk_off[c + 1] / kChunkRows));
        P.chunk_off[c + 1] += P.chunk_off[c];
    }
    const int64_t slots = P.chunk_off[P.nchunks];
    P.sell_val.resize(slots);  // every slot is written by fill_sell
    P.sell_col.resize(slots);
    if (P.split_lower) {
        P.lmask.assign((size_t)P.nchunks * kChunkRows, 0u);
        P.dslot.assign((size_t)P.nchunks * kChunkRows, 0);
    }
    fill_sell(P, rowptr, col, val, true);
    // register slots: the smallest supported width covering every chunk, capped
    P.reg_slots = P.max_width <= 4 ? 4 : P.max_width <= 7 ? 7 : P.max_width <= 8 ? 8
                : P.max_width <= 16 ? 16 : 32;
    if (P.max_reg > 0) P.reg_slots = std::min(P.reg_slots, P.max_reg);
    // chunks per worker when the caller leaves it open: two (four chunks of
    // FP32 values fit the plain power kernel better, but not the polynomial
    // kernels, and a plan serves both); wide rows leave room for one chunk only
    const bool auto_group = P.group == 0;
    if (P.group == 0) P.group = 2;
    if (P.reg_slots >= 32) P.group = 1;

    // ---- chunk ownership by position inside the level (D2) ------------------
    P.owner.assign(P.nchunks, 0);
    for (int32_t c = 0; c < P.nchunks; ++c) {
        int32_t r0 = c * kChunkRows;
        int32_t l = P.level_of_row[P.perm[r0]];
        int64_t start = P.level_ptr[l], size = P.level_ptr[l + 1] - P.level_ptr[l];
        P.owner[c] = (int32_t)(((int64_t)kParts * (r0 - start)) / size);
    }
    P.seq_ptr.assign(kParts + 1, 0);
    for (int32_t c = 0; c < P.nchunks; ++c) ++P.seq_ptr[P.owner[c] + 1];
    for (int x = 0; x < kParts; ++x) P.seq_ptr[x + 1] += P.seq_ptr[x];
    P.seq.assign(P.nchunks, 0);
    {
        std::vector<int32_t> pos(P.seq_ptr.begin(), P.seq_ptr.end() - 1);
        for (int32_t c = 0; c < P.nchunks; ++c) P.seq[pos[P.owner[c]]++] = c;
    }

    // ---- dependency lists (D3) -----------------------------------------------
    // one pass over contiguous ranges of chunks, each thread with its own marks
    // and its lists in chunk order, then placed behind the prefix sums
    P.dep_ptr.assign(P.nchunks + 1, 0);
    P.dep_idx.clear();
    {
        const int nt = host_threads();
        std::vector<Local> lists(nt);
        std::vector<int64_t> first_chunk(nt, -1);
        parallel_ranges(P.nchunks, 1, kRowGrain / kChunkRows, [&](int t, int64_t c0, int64_t c1) {
            std::vector<int32_t> stamp(P.nchunks, -1);
            auto& out = lists[t].v;
            first_chunk[t] = c0;
            for (int64_t c = c0; c < c1; ++c) {
                const size_t start = out.size();
                stamp[c] = (int32_t)c;  // never list the chunk itself
                for (int32_t i = (int32_t)c * kChunkRows; i < std::min<int64_t>(n, (c + 1) * kChunkRows); ++i) {
                    const int32_t o = P.perm[i];
                    for (int64_t e = ptr[o]; e < ptr[o + 1]; ++e) {
                        const int32_t d = P.iperm[adj[e]] / kChunkRows;
                        if (stamp[d] != c) {
                            stamp[d] = (int32_t)c;
                            out.push_back(d);
                        }
                    }
                }
                std::sort(out.begin() + start, out.end());
                P.dep_ptr[c + 1] = (int32_t)(out.size() - start);
            }
        });
        for (int32_t c = 0; c < P.nchunks; ++c) P.dep_ptr[c + 1] += P.dep_ptr[c];
        P.dep_idx.resize(P.dep_ptr[P.nchunks]);
        parallel_ranges(nt, 1, 1, [&](int, int64_t t0, int64_t t1) {
            for (int64_t t = t0; t < t1; ++t)
                if (first_chunk[t] >= 0)
                    std::copy(lists[t].v.begin(), lists[t].v.end(), P.dep_idx.begin() + P.dep_ptr[first_chunk[t]]);
        });
    }

    // ---- work units and their deadlock bound (D3) ------------------------------
    build_units(P, std::max(1, P.group), P.units);
    // the blocked kernels also have variants carrying three, five and six chunks
    // per worker at rows of up to 8 slots; the upload decides where to use them
    for (int i = 0; i < kWide; ++i) {
        P.wide[i] = Units{};
        if (auto_group && P.group == 2 && P.reg_slots <= 8) build_units(P, kWideGroups[i], P.wide[i]);
    }
}

std::vector<int32_t> group_levels(const HostPlan& P, int32_t q) {
    // greedy and contiguous under the budget floor(C / q) (R14)
    const int64_t budget = P.cache_bytes / std::max(1, q);
    const int64_t vbytes = P.value_type == 1 ? 4 : P.value_type == 2 ? 2 : 8;
    std::vector<int32_t> gp{0};
    int64_t w_group = 0, rows_group = 0;
    for (int32_t l = 0; l < P.nlevels; ++l) {
        const int64_t rows = P.level_ptr[l + 1] - P.level_ptr[l];
        const int64_t w = P.level_nnz[l] * (vbytes + 4) + rows * (4 + 16);
        if (rows_group > 0 && w_group + w > budget && rows_group >= P.min_group_rows) {
            gp.push_back(l);
            w_group = rows_group = 0;
        }
        w_group += w;
        rows_group += rows;
    }
    gp.push_back(P.nlevels);
    return gp;
}

std::vector<StageTask> wavefront_schedule(const HostPlan& P, int32_t q) {
    // task (k, g) on levels shifted down by k - 1, at stage g + k - 1 (R15)
    const std::vector<int32_t> gp = group_levels(P, q);
    const int32_t G = (int32_t)gp.size() - 1, L = P.nlevels;
    std::vector<StageTask> tasks;
    for (int32_t stage = 0; stage < G + q - 1; ++stage)
        for (int32_t k = 1; k <= q; ++k) {
            const int32_t g = stage - (k - 1);
            if (g < 0 || g >= G) continue;
            const int32_t lo = g == 0 ? 0 : std::max(0, gp[g] - (k - 1));
            const int32_t hi = g == G - 1 ? L - 1 : gp[g + 1] - 1 - (k - 1);
            if (hi < lo) continue;
            tasks.push_back({stage, k, P.level_ptr[lo], P.level_ptr[hi + 1]});
        }
    return tasks;
}

}  // namespace mpk
