// Host-side planner of the MPK library: BFS level structure, level-order
// permutation, SELL-64 layout of the permuted matrix, chunk-to-XCD partition
// and chunk dependency lists.  Plain C++17, no HIP.
#pragma once

#include <cstdint>
#include <memory>
#include <new>
#include <string>
#include <utility>
#include <vector>

namespace mpk {

// Allocator whose value construction leaves memory uninitialised: for large
// arrays that are written in full, in parallel, right after they are sized.
template <typename T>
struct NoInit : std::allocator<T> {
    template <typename U>
    struct rebind {
        using other = NoInit<U>;
    };
    NoInit() = default;
    template <typename U>
    NoInit(const NoInit<U>&) noexcept {}
    template <typename U>
    void construct(U* p) noexcept {
        ::new ((void*)p) U;
    }
    template <typename U, typename... A>
    void construct(U* p, A&&... a) {
        ::new ((void*)p) U(std::forward<A>(a)...);
    }
};

constexpr int kChunkRows = 64;  // rows per chunk = lanes per wavefront
constexpr int kParts = 8;       // XCD partitions of the MI355X
constexpr int kMaxBlock = 15;   // largest p_block (4 bits of the done counters)
constexpr int kWide = 3;                        // extra unit tables of a plan
constexpr int kWideGroups[kWide] = {3, 5, 6};  // their chunks per worker

// Work units of G consecutive chunks of a partition's sequence: units of
// partition x are ptr[x] .. ptr[x + 1] - 1; unit u's record is rec[u * stride +
// 5 g + {0: chunk (-1 past the end), 1: slot offset / 64, 2: width}] for each
// chunk g, and rec[u * stride + {3, 4}] = dep_ptr[u], dep_ptr[u + 1] (the other
// chunks' fields 3 and 4 are 0).  A unit's chunks publish each power together,
// after one wait for all their stores, and only the first chunk's completion
// word is written: dep_idx[dep_ptr[u] ..] lists that word (the chunk id) for
// every other unit that u's rows read.
struct Units {
    int32_t group = 0;                 // G
    std::vector<int32_t> ptr;          // kParts + 1
    std::vector<int32_t> rec;
    std::vector<int32_t> dep_ptr;      // units + 1
    std::vector<int32_t> dep_idx;
    int32_t stride = 0;                // ints per record: 8, 16 or 32 for G = 1, 2, 3..6
    std::vector<int32_t> min_workers;  // index q = 0..p_block (entry 0 unused): the
                                       // smallest deadlock-free worker count (D3)
};

struct HostPlan {
    int32_t n = 0;
    int64_t nnz = 0;
    // options
    int32_t root_mode = 0, root = 0, p_block = 4, workers_req = 0, watchdog = 0;
    int32_t group = 2;  // chunks a worker carries together (G); 0 = chosen by the planner
    int32_t value_type = 0;  // 0: FP64 values on the device, 1: FP32, 2: BF16 with a row scale
    int32_t max_reg = 0;     // cap on register slots (0 = automatic)
    int64_t cache_bytes = 256ll << 20;  // C of the level groups (R14)
    int32_t min_group_rows = 0;         // row floor of a level group (R14)
    int32_t split_lower = 0;            // also record the strictly lower slots of each row
    uint64_t pattern_key[2] = {0, 0};   // pattern_hash of the CSR the plan was built from

    // Sec. 3 level structure
    int32_t nlevels = 0;
    std::vector<int32_t> level_ptr;     // nlevels + 1, permuted row offsets
    std::vector<int32_t> level_of_row;  // n, by original row
    std::vector<int32_t> perm, iperm;   // perm[new] = old, iperm[old] = new
    std::vector<int32_t> roots;         // BFS root of each component
    std::vector<int64_t> level_nnz;     // nlevels: stored entries of each level's rows

    // SELL-64 layout of P A P^T
    int32_t nchunks = 0;
    std::vector<int64_t> chunk_off;  // nchunks + 1, slot offsets (multiples of 64)
    std::vector<double, NoInit<double>> sell_val;    // slots
    std::vector<int32_t, NoInit<int32_t>> sell_col;  // slots, -1 = padding
    int32_t max_width = 0;
    int32_t reg_slots = 8;  // slots per row the blocked kernel keeps in registers
    // with split_lower (rows of at most 32 slots): per permuted row, bit s of lmask is
    // set when slot s holds a column that precedes the row in the original numbering
    // (the strictly lower triangle L of A), and dslot is the slot of the diagonal entry
    std::vector<uint32_t> lmask;        // nchunks * 64
    std::vector<int32_t> dslot;         // nchunks * 64

    // partition and dependencies
    std::vector<int32_t> owner;          // nchunks
    std::vector<int32_t> seq, seq_ptr;   // chunks of each partition, ascending; kParts + 1
    std::vector<int32_t> dep_ptr;        // nchunks + 1
    std::vector<int32_t> dep_idx;        // dependency chunk ids
    Units units;   // G = group: every blocked kernel
    // G = kWideGroups[i] (group 0 when absent), built when the caller left the group to
    // the planner and rows fit 8 register slots
    Units wide[kWide];
};

// One task of the wavefront schedule (R15): power k (1..q) of a block on the
// permuted rows [row_begin, row_end), run at `stage`.
struct StageTask {
    int32_t stage, k, row_begin, row_end;
};

// Level groups under floor(C / q) bytes (R14): group g holds levels
// group_ptr[g] .. group_ptr[g + 1] - 1.
std::vector<int32_t> group_levels(const HostPlan& P, int32_t q);

// The tasks of one block of q powers in stage order, then k (R15).
std::vector<StageTask> wavefront_schedule(const HostPlan& P, int32_t q);

// Rewrites the SELL values of a plan from new values of the CSR pattern it was
// built from (columns, levels and tables unchanged).
void refill_values(HostPlan& P, const int32_t* rowptr, const int32_t* col, const double* val);

// 128-bit key of a CSR pattern (n, row pointers, column indices).
void pattern_hash(int32_t n, const int32_t* rowptr, const int32_t* col, uint64_t out[2]);

// Validates the CSR input; returns an empty string or an error message.
std::string validate_csr(int32_t n, const int32_t* rowptr, const int32_t* col);

// Builds every host table of the plan.  Input must be valid (validate_csr).
void build_plan(HostPlan& P, int32_t n, const int32_t* rowptr, const int32_t* col,
                const double* val);

}  // namespace mpk
