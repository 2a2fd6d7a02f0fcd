// Host planner: level structure (Sec. 3), level-order permutation, SELL-64
// layout, chunk partition over the XCDs and the dependency lists that drive
// the blocked kernel.
#include "planner.h"

#include <algorithm>
#include <cstdio>
#include <numeric>
#include <thread>

namespace mpk {

std::string validate_csr(int32_t n, const int32_t* rowptr, const int32_t* col) {
    char buf[160];
    if (rowptr[0] != 0) return "rowptr[0] must be 0";
    for (int32_t i = 0; i < n; ++i) {
        if (rowptr[i + 1] < rowptr[i]) {
            snprintf(buf, sizeof buf, "rowptr decreases at row %d", i);
            return buf;
        }
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
    }
    return "";
}

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
        if (i0 < i1) pool.emplace_back(fn, i0, i1);
    }
    fn((int64_t)0, std::min(n, per));
    for (auto& th : pool) th.join();
}

// Undirected graph of pattern(A) + pattern(A^T), self-loops dropped, each
// neighbour list sorted and free of duplicates.
void symmetric_pattern(int32_t n, const int32_t* rowptr, const int32_t* col,
                       std::vector<int64_t>& ptr, std::vector<int32_t>& adj) {
    std::vector<int64_t> cnt(n + 1, 0);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
            if (col[e] != i) {
                ++cnt[i + 1];
                ++cnt[col[e] + 1];
            }
    for (int32_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    std::vector<int32_t> tmp(cnt[n]);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
            if (col[e] != i) {
                tmp[fill[i]++] = col[e];
                tmp[fill[col[e]]++] = i;
            }
    // each row's neighbours sorted and without repeats, then packed
    ptr.assign(n + 1, 0);
    parallel_ranges(n, 1, kRowGrain, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) {
            auto b = tmp.begin() + cnt[i], e = tmp.begin() + cnt[i + 1];
            std::sort(b, e);
            ptr[i + 1] = std::unique(b, e) - b;
        }
    });
    for (int32_t i = 0; i < n; ++i) ptr[i + 1] += ptr[i];
    adj.resize(ptr[n]);
    parallel_ranges(n, 1, kRowGrain, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i)
            std::copy(tmp.begin() + cnt[i], tmp.begin() + cnt[i] + (ptr[i + 1] - ptr[i]), adj.begin() + ptr[i]);
    });
}

// Breadth-first search from `root`.  Fills dist for every reached vertex
// (caller resets them afterwards via `order`), returns the visit order and
// the start of each distance layer inside it.
struct Bfs {
    std::vector<int32_t> order;       // vertices by nondecreasing distance
    std::vector<int32_t> layer_ptr;   // layer d = order[layer_ptr[d] .. layer_ptr[d+1])
};

void bfs(const std::vector<int64_t>& ptr, const std::vector<int32_t>& adj, int32_t root,
         std::vector<int32_t>& dist, Bfs& out) {
    out.order.clear();
    out.layer_ptr.clear();
    out.order.push_back(root);
    dist[root] = 0;
    out.layer_ptr.push_back(0);
    size_t head = 0;
    int32_t cur = 0;
    while (head < out.order.size()) {
        int32_t u = out.order[head];
        if (dist[u] != cur) {  // first vertex of the next layer
            out.layer_ptr.push_back((int32_t)head);
            cur = dist[u];
        }
        ++head;
        for (int64_t e = ptr[u]; e < ptr[u + 1]; ++e) {
            int32_t v = adj[e];
            if (dist[v] < 0) {
                dist[v] = dist[u] + 1;
                out.order.push_back(v);
            }
        }
    }
    out.layer_ptr.push_back((int32_t)out.order.size());
}

void reset(std::vector<int32_t>& dist, const Bfs& b) {
    for (int32_t v : b.order) dist[v] = -1;
}

// George-Liu pseudo-peripheral node of the component containing `start`.
// `br` holds the search from `start` on entry and the search from the
// returned node on exit.
int32_t pseudo_peripheral(const std::vector<int64_t>& ptr, const std::vector<int32_t>& adj,
                          int32_t start, std::vector<int32_t>& dist, Bfs& br) {
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
        bfs(ptr, adj, x, dist, bx);
        reset(dist, bx);
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
    // rows write disjoint slots: threads take contiguous ranges of chunks
    parallel_ranges(P.n, kChunkRows, kRowGrain, [&](int64_t i0, int64_t i1) {
        std::vector<std::pair<int32_t, double>> row;
        for (int32_t i = (int32_t)i0; i < (int32_t)i1; ++i) {
            int32_t o = P.perm[i];
            row.clear();
            for (int32_t e = rowptr[o]; e < rowptr[o + 1]; ++e)
                row.emplace_back(P.iperm[col[e]], val[e]);
            std::sort(row.begin(), row.end(),
                      [](const std::pair<int32_t, double>& a, const std::pair<int32_t, double>& b) {
                          return a.first < b.first;
                      });
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
    std::fill(P.sell_val.begin(), P.sell_val.end(), 0.0);
    fill_sell(P, rowptr, col, val, false);
}

void pattern_hash(int32_t n, const int32_t* rowptr, const int32_t* col, uint64_t out[2]) {
    // two 64-bit multiply-xorshift chains with different odd multipliers over the
    // row pointers and the column indices (a 128-bit key of the pattern)
    uint64_t a = 0x243F6A8885A308D3ull ^ (uint64_t)n, b = 0x13198A2E03707344ull + (uint64_t)n;
    auto mix = [&](uint64_t w) {
        a = (a ^ w) * 0x9E3779B97F4A7C15ull;
        a ^= a >> 29;
        b = (b + w) * 0xBF58476D1CE4E5B9ull;
        b ^= b >> 31;
    };
    for (int32_t i = 0; i <= n; ++i) mix((uint64_t)(uint32_t)rowptr[i]);
    const int64_t nnz = n > 0 ? rowptr[n] : 0;
    for (int64_t e = 0; e < nnz; ++e) mix(0x5555555555555555ull ^ (uint64_t)(uint32_t)col[e]);
    out[0] = a;
    out[1] = b;
}

void build_plan(HostPlan& P, int32_t n, const int32_t* rowptr, const int32_t* col,
                const double* val) {
    P.n = n;
    pattern_hash(n, rowptr, col, P.pattern_key);
    P.nnz = n ? rowptr[n] : 0;

    // ---- levels (readings R1-R3) ------------------------------------------
    std::vector<int64_t> ptr;
    std::vector<int32_t> adj;
    symmetric_pattern(n, rowptr, col, ptr, adj);
    std::vector<int32_t> dist(n, -1);
    P.level_of_row.assign(n, -1);
    P.roots.clear();
    std::vector<char> seen(n, 0);
    Bfs comp, lv;
    int32_t base = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (seen[v]) continue;
        bfs(ptr, adj, v, dist, comp);  // the component of the lowest unvisited row
        bool has_root = P.root_mode == 1 && dist[P.root] >= 0;
        reset(dist, comp);
        int32_t r;
        if (has_root) {
            r = P.root;
            bfs(ptr, adj, r, dist, lv);
            reset(dist, lv);
        } else {  // the component's search is the first step of the root search
            std::swap(lv, comp);
            r = pseudo_peripheral(ptr, adj, v, dist, lv);
        }
        for (size_t d = 0; d + 1 < lv.layer_ptr.size(); ++d)
            for (int32_t t = lv.layer_ptr[d]; t < lv.layer_ptr[d + 1]; ++t)
                P.level_of_row[lv.order[t]] = base + (int32_t)d;
        for (int32_t u : lv.order) seen[u] = 1;
        base += (int32_t)lv.layer_ptr.size() - 1;
        P.roots.push_back(r);
    }
    P.nlevels = base;

    // ---- permutation: rows by (level, original index) (R4) ------------------
    P.level_ptr.assign(P.nlevels + 1, 0);
    for (int32_t i = 0; i < n; ++i) ++P.level_ptr[P.level_of_row[i] + 1];
    for (int32_t l = 0; l < P.nlevels; ++l) P.level_ptr[l + 1] += P.level_ptr[l];
    P.level_nnz.assign(P.nlevels, 0);
    for (int32_t i = 0; i < n; ++i) P.level_nnz[P.level_of_row[i]] += rowptr[i + 1] - rowptr[i];
    P.perm.assign(n, 0);
    P.iperm.assign(n, 0);
    {
        std::vector<int32_t> pos(P.level_ptr.begin(), P.level_ptr.end() - (P.nlevels ? 1 : 0));
        for (int32_t i = 0; i < n; ++i) {
            int32_t k = pos[P.level_of_row[i]]++;
            P.perm[k] = i;
            P.iperm[i] = k;
        }
    }

    // ---- SELL-64 layout of P A P^T ------------------------------------------
    P.nchunks = (n + kChunkRows - 1) / kChunkRows;
    P.chunk_off.assign(P.nchunks + 1, 0);
    P.max_width = 0;
    for (int32_t c = 0; c < P.nchunks; ++c) {
        int32_t w = 0;
        for (int32_t i = c * kChunkRows; i < std::min(n, (c + 1) * kChunkRows); ++i) {
            int32_t o = P.perm[i];
            w = std::max(w, rowptr[o + 1] - rowptr[o]);
        }
        P.max_width = std::max(P.max_width, w);
        P.chunk_off[c + 1] = P.chunk_off[c] + (int64_t)w * kChunkRows;
    }
    const int64_t slots = P.chunk_off[P.nchunks];
    P.sell_val.assign(slots, 0.0);
    P.sell_col.assign(slots, -1);
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
    if (P.group == 0) P.group = 2;
    if (P.reg_slots >= 32) P.group = 1;

    // ---- chunk ownership by position inside the level (R6) ------------------
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

    // ---- dependency lists (R7) -----------------------------------------------
    // two passes over ranges of chunks (lengths, then the sorted lists), each
    // range with its own marks
    P.dep_ptr.assign(P.nchunks + 1, 0);
    P.dep_idx.clear();
    {
        auto chunk_list = [&](int32_t c, std::vector<int32_t>& stamp, std::vector<int32_t>& list) {
            list.clear();
            stamp[c] = c;  // never list the chunk itself
            for (int32_t i = c * kChunkRows; i < std::min(n, (c + 1) * kChunkRows); ++i) {
                int32_t o = P.perm[i];
                for (int64_t e = ptr[o]; e < ptr[o + 1]; ++e) {
                    int32_t d = P.iperm[adj[e]] / kChunkRows;
                    if (stamp[d] != c) {
                        stamp[d] = c;
                        list.push_back(d);
                    }
                }
            }
        };
        parallel_ranges(P.nchunks, 1, kRowGrain / kChunkRows, [&](int64_t c0, int64_t c1) {
            std::vector<int32_t> stamp(P.nchunks, -1), list;
            for (int64_t c = c0; c < c1; ++c) {
                chunk_list((int32_t)c, stamp, list);
                P.dep_ptr[c + 1] = (int32_t)list.size();
            }
        });
        for (int32_t c = 0; c < P.nchunks; ++c) P.dep_ptr[c + 1] += P.dep_ptr[c];
        P.dep_idx.resize(P.dep_ptr[P.nchunks]);
        parallel_ranges(P.nchunks, 1, kRowGrain / kChunkRows, [&](int64_t c0, int64_t c1) {
            std::vector<int32_t> stamp(P.nchunks, -1), list;
            for (int64_t c = c0; c < c1; ++c) {
                chunk_list((int32_t)c, stamp, list);
                std::sort(list.begin(), list.end());
                std::copy(list.begin(), list.end(), P.dep_idx.begin() + P.dep_ptr[c]);
            }
        });
    }

    // ---- smallest deadlock-free worker count per block size q (R7) ----------
    // Units: G consecutive chunks of a partition's sequence, carried together.
    // bmin[u] = smallest first chunk among units within h unit hops of u; the
    // condition for W workers holds iff W > max over unit positions j of
    // (j - first position whose first chunk is >= bmin[unit j]), per partition.
    const int32_t G = std::max(1, P.group);
    P.unit_ptr.assign(kParts + 1, 0);
    std::vector<int32_t>& unit_ptr = P.unit_ptr;
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
    P.unit_stride = G <= 1 ? 8 : (G == 2 ? 16 : 32);
    P.unit_rec.assign((size_t)nunits * P.unit_stride, 0);
    for (int x = 0; x < kParts; ++x) {
        const int32_t len = P.seq_ptr[x + 1] - P.seq_ptr[x];
        for (int32_t u = unit_ptr[x]; u < unit_ptr[x + 1]; ++u) {
            int32_t* r = P.unit_rec.data() + (size_t)u * P.unit_stride;
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
                r[5 * g + 3] = P.dep_ptr[c];
                r[5 * g + 4] = P.dep_ptr[c + 1];
            }
        }
    }
    std::vector<int32_t> udep_ptr(nunits + 1, 0), udep;
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
    P.min_workers.assign(P.p_block + 1, 1);
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
        P.min_workers[q] = need;
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
