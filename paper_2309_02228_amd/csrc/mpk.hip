// MI355X (gfx950) kernels and C ABI of the matrix power kernel library.
//
// Device layout of a plan (one caller-owned buffer, 256-byte aligned pieces):
//   SELL-64 values (f64) and columns (i32, -1 = padding) of P A P^T,
//   chunk slot offsets (i64), perm / iperm (i32), per-XCD chunk sequences,
//   work-unit tables with their dependency lists, completion words (u32,
//   one per chunk, written for the first chunk of each unit) and a status
//   block.
//
// Two kernels compute powers:
//   * spmv_kernel: one launch per power (Alg. 1), waves stride over the
//     chunks of their XCD partition.  It is the plain comparator.
//   * mpk_block_kernel: one persistent launch per block of q powers.  Each
//     wave takes a unit of G chunks, keeps their SELL slots in registers and
//     advances them through the q powers; before power k it waits until
//     every unit its rows read has published power k-1.  The matrix
//     therefore streams from HBM once per block instead of once per power
//     (Sec. 3, temporal blocking along the level structure).
// Vectors written inside the blocked kernel use device-coherent (sc1)
// stores and loads: the L2 of one XCD is not kept coherent with plain
// write-back stores of another XCD, and agent-scope fences cost far more
// than the work they would guard.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mpk.h"
#include "internal.h"
#include "planner.h"


namespace {

using mpk::kChunkRows;
using mpk::kParts;

constexpr int kWaves = 4;                 // waves per workgroup
constexpr int kBlockThreads = kWaves * 64;
constexpr int kMaxQ = mpk::kMaxBlock;      // powers per blocked launch
constexpr int kSpinLimit = 1 << 20;        // watchdog polls per dependency wait
constexpr uint32_t kEpochLimit = 1u << 27; // done words hold epoch * 16 + power
// Completion words sit one per 128-byte line: neighbouring chunks publish from
// different waves (and XCDs); sharing a line makes every write-through
// invalidate the line under the other chunks' pollers.
constexpr int kFlagStride = 32;
constexpr int kStatusSlots = 64;  // per plan: one per calling stream (least recently used reused)

// KIND_JCHAIN: the Jacobi-preconditioned chain w_j = w_{j-1} + c (B - I)^k w_{j-1}
// (c = -(-1)^k) as one sequence of sub-powers u = (B - I) u_prev; every k-th
// sub-power closes a link with w_j = fma(c, u, w_{j-1}), which is stored both in the
// ring (the next sub-power's input) and as output column j.
// KIND_GS2: the GS2-preconditioned chain, gl = gamma + 2 sub-powers per power: r = 0
// gives g_0 = D^{-1} w_{j-1}, r = 1..gamma the sweeps g_r = g_0 - D^{-1} L g_{r-1}, and
// r = gamma + 1 closes the power with w_j = A g_gamma (also stored as output column j).
// KIND_SMOOTH: the pre-smoother of an AMG cycle followed by its residual, gamma + 1
// sub-powers per outer GS2 sweep on A z = b and a final sub-power b - A z (see
// smooth_value); it reads the same lower masks and diagonal slots as KIND_GS2.
enum Kind { KIND_MONO = 0, KIND_NEWTON = 1, KIND_CHEB = 2, KIND_JCHAIN = 3, KIND_GS2 = 4, KIND_SMOOTH = 5 };
constexpr int kKinds = 6;
// kinds whose rows keep the diagonal entry and the strictly lower mask (split plans)
constexpr bool split_kind(int k) { return k == KIND_GS2 || k == KIND_SMOOTH; }

// ------------------------------------------------------------------ device
struct DevPlan {
    const void* val;           // SELL values: double, float (FP32) or BF16 bits
    const float* rowscale;     // per permuted row (BF16 storage only)
    const int32_t* col;
    const int64_t* off;
    const int32_t* seq;
    const int32_t* seq_ptr;
    const int32_t* unit_ptr;  // kParts + 1
    const int32_t* unit_rec;  // one record of unit_stride ints per unit
    int32_t ndeps;            // length of dep_idx
    const int32_t* dep_idx;   // the unit table's dependency lists (completion-word chunk ids)
    uint32_t* done;
    uint32_t* tickets;  // [4 launch slots][kParts], one per 128-byte line
    const uint32_t* lmask;  // per permuted row: slots of the strictly lower triangle (split plans)
    const int32_t* dslot;   // per permuted row: slot of the diagonal entry (split plans)
    int32_t n;
};

// Per-launch operator coefficients, indexed by the local power 0..q-1.
struct Coefs {
    double lam[kMaxQ];  // Newton shift
    double sig[kMaxQ];  // Newton column scaling
    double c[kMaxQ];    // polynomial coefficient of the power
    double theta, delta;
    int jk;             // KIND_JCHAIN: sub-powers per link; KIND_GS2: sub-powers per power
    double jc;          // KIND_JCHAIN: coefficient of (B - I)^k at the end of a link
    int pinv;           // KIND_GS2: 1 = the chain applies P^{-1} only (a power closes with g_gamma)
    int chain_len;      // KIND_SMOOTH: sub-powers of the whole chain (the last is the residual)
};

// GS2 sub-power r of a power from the row's full sum sA = (A g)_i, its strictly lower
// part sL = (L g)_i, its own previous value, g_0, the diagonal entry d and the power's
// input w0.  A power closes with (A g_gamma - lam w0) / sig (lam = 0, sig = 1: A g_gamma;
// Newton shifts of an s-step basis otherwise), or with g_gamma itself when pinv is set.
__device__ __forceinline__ double gs2_value(double sA, double sL, double prev, double g0, double d, double w0, int r,
                                            int gl, int pinv, double lam, double sig) {
    if (r == 0) return prev / d;
    if (r < gl - 1 || pinv) return g0 - sL / d;
    if (lam == 0.0 && sig == 1.0) return sA;
    return fma(-lam, w0, sA) / sig;
}

// Sub-power r of an outer sweep of the GS2 pre-smoother (non-compact form, gl = gamma + 1
// sub-powers per sweep) from the row's full sum sA = (A v)_i and strictly lower part
// sL = (L v)_i of the previous sub-power's vector v, the sweep's start value z, the
// diagonal entry d and b_i: r = 0 gives g_0 = (b - A z)_i / d (kept in g0), r >= 1 the
// inner sweeps g_r = g_0 - (L g_{r-1})_i / d, and the sweep's last sub-power stores
// z + g_gamma, the start of the next sweep.  The chain's final sub-power is the residual
// b - A z of the smoothed vector.
__device__ __forceinline__ double smooth_value(double sA, double sL, double z, double& g0, double d, double b, int r,
                                               int gl, bool final) {
    if (final) return b - sA;
    const double g = r == 0 ? (b - sA) / d : g0 - sL / d;
    if (r == 0) g0 = g;
    return r == gl - 1 ? z + g : g;
}

// Gathers of vector entries by 32-bit row index through a structured buffer
// resource (8-byte records, n of them): an index past the end (the column -1
// of padding slots) reads 0.0 instead of faulting, so no lane mask is needed.
typedef int gi32x4 __attribute__((ext_vector_type(4)));
typedef int gi32x2 __attribute__((ext_vector_type(2)));
__device__ gi32x2 struct_buffer_load_b64(gi32x4 rsrc, int vindex, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.struct.buffer.load.v2i32");
__device__ __forceinline__ gi32x4 vec_rsrc(const double* base, int n) {
    const uint64_t b = (uint64_t)base;
    gi32x4 r;
    r.x = (int)(uint32_t)b;
    r.y = (int)(((uint32_t)(b >> 32) & 0xffffu) | (8u << 16));  // stride 8 bytes
    r.z = n;
    r.w = 0x00020000;
    return r;
}
// AUX 16: a device-coherent read (sc1), for powers written in the same launch
template <int AUX>
__device__ __forceinline__ double gather(gi32x4 r, int i) {
    return __builtin_bit_cast(double, struct_buffer_load_b64(r, i, 0, 0, AUX));
}

__device__ __forceinline__ double load_coherent(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_coherent(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t load_word(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Operator kind applied to s = (A y_{k-1})_i with the row's own y_{k-1}, y_{k-2}.
// `link0` is the chain's value at the start of the current link (KIND_JCHAIN).
template <int KIND>
__device__ __forceinline__ double finish(double s, double prev, double prev2, double link0, int gk, int kl,
                                         const Coefs& C) {
    if (KIND == KIND_MONO) return s;
    if (KIND == KIND_NEWTON) return fma(-C.lam[kl], prev, s) / C.sig[kl];
    if (KIND == KIND_JCHAIN) {
        const double u = s - prev;
        if (gk % C.jk != 0) return u;
        const double w = fma(C.jc, u, link0);  // w_j = A P^{-1} w_{j-1}
        // a Newton shift of an s-step basis: (A P^{-1} - lam) w_{j-1} / sig
        return (C.lam[kl] == 0.0 && C.sig[kl] == 1.0) ? w : fma(-C.lam[kl], link0, w) / C.sig[kl];
    }
    const double t = fma(-C.theta, prev, s);
    return gk == 1 ? t / C.delta : (2.0 * t) / C.delta - prev2;
}

// ---- plain comparator: one power per launch --------------------------------
struct SpmvArgs {
    DevPlan P;
    const double* in;     // y_{k-1}
    const double* prev2;  // y_{k-2} (Chebyshev), may be null
    double* out;          // y_k
    const double* acc_in; // polynomial accumulator before this power (null: c0 * x)
    double* acc_out;      // polynomial accumulator after this power (null: none)
    double c0;
    int gk;               // global power index of this launch
    const double* link_in;  // KIND_JCHAIN: the chain's value at the start of the link
    const double* pow_in;   // KIND_GS2: the input w0 of the power (KIND_SMOOTH: b)
    double* link_out;       // KIND_JCHAIN: output column j - 1 receives w_j
    int64_t link_ld;
    double* z_io;           // KIND_SMOOTH: the current sweep's start z, rewritten as a sweep closes
    double* res_out;        // KIND_SMOOTH: receives the residual of the final sub-power
    Coefs C;              // entry 0 describes this power
};

// Row sum over the chunk's slots j = 0..width-1, in this order, as one FMA
// chain.  Slots are fetched in batches of 8 (columns and values first, then
// the gathers) so that a batch costs two memory round trips.
// A stored value as FP64.  BF16 storage (VT = uint16_t) holds q with the
// row's FP32 scale s; s * q has at most 8 + 24 significant bits, so the FP64
// product is exact.
template <typename VT>
__device__ __forceinline__ double decode(VT v, float scale) {
    if constexpr (sizeof(VT) == 2)
        return (double)scale * (double)__uint_as_float((uint32_t)v << 16);
    else
        return (double)v;
}

template <typename VT>
__device__ __forceinline__ float row_scale(const DevPlan& P, int row) {
    if constexpr (sizeof(VT) == 2)
        return P.rowscale[row];
    else
        return 1.0f;
}

template <typename VT>
__device__ __forceinline__ double row_sum_mem(const DevPlan& P, const double* in, int64_t off,
                                              int width, int lane, int row) {
    const VT* val = (const VT*)P.val;
    const float sc = row_scale<VT>(P, row);
    double s = 0.0;
    for (int j0 = 0; j0 < width; j0 += 8) {
        int cj[8];
        double vj[8], xj[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            cj[t] = -1;
            vj[t] = 0.0;
            if (j0 + t < width) {
                const int64_t slot = off + (int64_t)(j0 + t) * kChunkRows + lane;
                cj[t] = __builtin_nontemporal_load(P.col + slot);
                vj[t] = decode<VT>(__builtin_nontemporal_load(val + slot), sc);
            }
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) xj[t] = cj[t] >= 0 ? in[cj[t]] : 0.0;
#pragma unroll
        for (int t = 0; t < 8; ++t)
            if (cj[t] >= 0) s = fma(vj[t], xj[t], s);
    }
    return s;
}

// Both sums of a GS2 row in slot order: sA over all slots, sL over the strictly lower
// ones (lm), and the diagonal entry (slot ds).
template <typename VT>
__device__ __forceinline__ void row_sums_gs2(const DevPlan& P, const double* in, int64_t off, int width,
                                             int lane, int row, double& sA, double& sL, double& d) {
    const VT* val = (const VT*)P.val;
    const float sc = row_scale<VT>(P, row);
    const uint32_t lm = row < P.n ? P.lmask[row] : 0u;
    const int ds = row < P.n ? P.dslot[row] : -1;
    sA = 0.0;
    sL = 0.0;
    d = 1.0;
    for (int j = 0; j < width; ++j) {
        const int64_t slot = off + (int64_t)j * kChunkRows + lane;
        const int cj = P.col[slot];
        if (cj < 0) continue;
        const double v = decode<VT>(val[slot], sc);
        const double x = in[cj];
        sA = fma(v, x, sA);
        if ((lm >> j) & 1u) sL = fma(v, x, sL);
        if (j == ds) d = v;
    }
}

// Waves take chunks c = wave, wave + W, ... (a streaming pass; the matrix is
// not reused within a launch, so no XCD partition is needed).
template <int KIND, bool POLY, typename VT>
__global__ __launch_bounds__(kBlockThreads) void spmv_kernel(SpmvArgs a) {
    const int lane = threadIdx.x & 63;
    const int W = gridDim.x * kWaves;
    const int nchunks = (a.P.n + kChunkRows - 1) / kChunkRows;
    for (int c = blockIdx.x * kWaves + (threadIdx.x >> 6); c < nchunks; c += W) {
        const int row = c * kChunkRows + lane;
        const int64_t off = a.P.off[c];
        const int width = (int)((a.P.off[c + 1] - off) / kChunkRows);
        if constexpr (split_kind(KIND)) {
            const int r = (a.gk - 1) % a.C.jk;
            double sA = 0.0, sL = 0.0, d = 1.0;
            if (r == 0 && KIND == KIND_GS2) {  // g_0 = D^{-1} w: row-local, only the diagonal entry is read
                if (row < a.P.n)
                    d = decode<VT>(((const VT*)a.P.val)[off + (int64_t)a.P.dslot[row] * kChunkRows + lane],
                                   row_scale<VT>(a.P, row));
            } else {
                row_sums_gs2<VT>(a.P, a.in, off, width, lane, row, sA, sL, d);
            }
            if (row < a.P.n) {
                if constexpr (KIND == KIND_SMOOTH) {
                    const bool fin = a.gk == a.C.chain_len;
                    double g0 = a.link_in[row];
                    const double y = smooth_value(sA, sL, a.z_io[row], g0, d, a.pow_in[row], r, a.C.jk, fin);
                    a.out[row] = y;
                    if (fin) a.res_out[row] = y;
                    else if (r == a.C.jk - 1) a.z_io[row] = y;
                } else {
                    const double y = gs2_value(sA, sL, a.in[row], a.link_in[row], d, a.pow_in[row], r, a.C.jk,
                                               a.C.pinv, a.C.lam[0], a.C.sig[0]);
                    a.out[row] = y;
                    if (r == a.C.jk - 1) a.link_out[(int64_t)((a.gk - 1) / a.C.jk) * a.link_ld + row] = y;
                }
            }
            continue;
        }
        const double s = row_sum_mem<VT>(a.P, a.in, off, width, lane, row);
        if (row < a.P.n) {
            const double prev = (KIND != KIND_MONO || POLY) ? a.in[row] : 0.0;
            const double prev2 = (KIND == KIND_CHEB && a.prev2) ? a.prev2[row] : 0.0;
            const double link0 = KIND == KIND_JCHAIN ? a.link_in[row] : 0.0;
            const double y = finish<KIND>(s, prev, prev2, link0, a.gk, 0, a.C);
            a.out[row] = y;
            if (KIND == KIND_JCHAIN && a.gk % a.C.jk == 0)
                a.link_out[(int64_t)(a.gk / a.C.jk - 1) * a.link_ld + row] = y;
            if (POLY) {
                const double acc = a.acc_in ? a.acc_in[row] : a.c0 * prev;
                a.acc_out[row] = fma(a.C.c[0], y, acc);
            }
        }
    }
}

// ---- blocked kernel: q powers per persistent launch -------------------------
struct BlockArgs {
    DevPlan P;
    const double* in;     // y_base (block input; written before the launch)
    const double* prev2;  // y_{base-1} (Chebyshev only), may be null
    double* out0;         // destination of y_{base+1}
    int64_t out_ld;       // distance between consecutive destinations
    int out_mod;          // destinations cycle every out_mod powers (ring), else large
    int base_slot;        // slot of y_{base+1} inside the cycle
    double* copy0;        // if set: copy0[row] = in[row] (basis column 0)
    const double* acc_in; // polynomial accumulator before the block (null: c0 * x)
    double* acc_out;      // polynomial accumulator after the block (null: none)
    double c0;
    int base;             // powers finished before this launch
    int q;                // powers in this launch
    int workers;          // waves per partition
    int spin_limit;       // watchdog polls; negative: give up at once
    int plain_gather;     // 1: powers written in this launch may be read with plain loads
    uint32_t epoch;
    int32_t* status;      // the calling stream's status slot: [0] code, [1] chunk, [2] power
    const double* link_in;  // KIND_JCHAIN: the chain's value at the start of the link of y_{base+1}
    const double* pow_in;   // KIND_GS2: the input w0 of the power of y_{base+1} (KIND_SMOOTH: b)
    double* link_out;       // KIND_JCHAIN: output column j - 1 receives w_j
    int64_t link_ld;
    double* z_io;           // KIND_SMOOTH: the current sweep's start z, rewritten as a sweep closes
    double* res_out;        // KIND_SMOOTH: receives the residual of the final sub-power
    Coefs C;
};

__device__ __forceinline__ double* dest(const BlockArgs& a, int kl) {
    return a.out0 + (int64_t)((a.base_slot + kl) % a.out_mod) * a.out_ld;
}

// Raises the device status (first failure wins) and returns false.
__device__ bool give_up(const BlockArgs& a, int c, int kl) {
    if ((threadIdx.x & 63) == 0 && atomicCAS(a.status, 0, (int)MPK_ERR_DEVICE) == 0) {
        __hip_atomic_store(a.status + 1, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(a.status + 2, a.base + kl + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return false;
}

// Polls completion words until each lane's word has reached `target`.
// `wo` are byte offsets into the completion-word array `done` (buffer
// resource `dr`), read with device-coherent loads.  Returns false if the
// watchdog fired or another wave already gave up.
template <int G>
__device__ bool poll_until(const BlockArgs& a, __amdgpu_buffer_rsrc_t dr, const uint32_t (&wo)[G],
                           bool (&ok)[G], uint32_t target, int c_report, int kl) {
    for (int spin = 0;; ++spin) {
        bool all = true;
        if (a.spin_limit >= 0) {
            // chunk by chunk, only lanes still waiting (issuing the loads of all
            // chunks before waiting on any measured slower)
#pragma unroll
            for (int g = 0; g < G; ++g)
                if (!ok[g])
                    ok[g] = (int32_t)((uint32_t)__builtin_amdgcn_raw_buffer_load_b32(dr, (int)wo[g], 0, 16) -
                                      target) >= 0;
        }
#pragma unroll
        for (int g = 0; g < G; ++g) all = all && ok[g];
        if (__all(all)) return true;
        if ((spin & 255) == 255 || a.spin_limit < 0) {
            if (__hip_atomic_load(a.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
                return false;
            if (spin >= a.spin_limit) return give_up(a, c_report, kl);
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Unit = G consecutive chunks of a partition's sequence, carried together
// through the q powers of a block; its SELL slots stay in registers.
template <int REG, int G, int KIND, bool POLY, typename VT>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(G == 6 ? 2 : 1, 8)))
void mpk_block_kernel(BlockArgs a) {
    const VT* val = (const VT*)a.P.val;
    const int lane = threadIdx.x & 63;
    const int part = blockIdx.x % kParts;
    // plan tables are constant during the launch: reading them through the
    // constant address space turns the wave-uniform reads into scalar loads
    typedef const int32_t __attribute__((address_space(4))) kint;
    kint* unit_ptr = (kint*)a.P.unit_ptr;
    const int ub = unit_ptr[part];
    const int nunits = unit_ptr[part + 1] - ub;
    constexpr int kStride = G <= 1 ? 8 : (G == 2 ? 16 : 32);
    const int nchunks = (a.P.n + kChunkRows - 1) / kChunkRows;
    const __amdgpu_buffer_rsrc_t dr =
        __builtin_amdgcn_make_buffer_rsrc((void*)a.P.done, 0, nchunks * 4 * kFlagStride, 0x00020000);
    const __amdgpu_buffer_rsrc_t depr =
        __builtin_amdgcn_make_buffer_rsrc((void*)a.P.dep_idx, 0, a.P.ndeps * 4, 0x00020000);
    // Units are handed out in sequence order from a per-partition counter, so
    // only waves that are actually resident take work.  This launch uses slot
    // epoch % 4 and clears the slot of the launch after next.
    uint32_t* tick = a.P.tickets + ((a.epoch & 3u) * kParts + part) * kFlagStride;
    if (blockIdx.x < kParts && threadIdx.x == 0)
        a.P.tickets[(((a.epoch + 2u) & 3u) * kParts + blockIdx.x) * kFlagStride] = 0u;
    for (;;) {
        uint32_t t = 0;
        if (lane == 0) t = atomicAdd(tick, 1u);
        const int u = (int)__builtin_amdgcn_readfirstlane(t);
        if (u >= nunits) break;
        // the unit's record: chunk, slot offset / 64 and width of each of its
        // chunks and the range of its dependency list, in one scalar load
        kint* rec = (kint*)a.P.unit_rec + (int64_t)(ub + u) * kStride;
        int c[G], width[G], row[G];
        int64_t off[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            c[g] = rec[5 * g];
            off[g] = (int64_t)rec[5 * g + 1] * kChunkRows;
            width[g] = rec[5 * g + 2];
            row[g] = c[g] * kChunkRows + lane;
        }
        // the other units its rows read, each by the completion word of its first
        // chunk: one lane per unit in the first batch; lanes past the list read
        // out of range and get 0
        const int d0 = rec[3], d1 = rec[4];
        const int di = d0 + lane;
        const bool need = di < d1;
        const uint32_t wo[1] = {(uint32_t)__builtin_amdgcn_raw_buffer_load_b32(depr, need ? di * 4 : -1, 0, 0) *
                                (4u * kFlagStride)};
        const bool long_list = d1 - d0 > 64;
        VT rv[G][REG];
        int rc[G][REG];
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int j = 0; j < REG; ++j) {
                rc[g][j] = -1;
                rv[g][j] = (VT)0;
                if (j < width[g]) {
                    const int64_t slot = off[g] + (int64_t)j * kChunkRows + lane;
                    rc[g][j] = __builtin_nontemporal_load(a.P.col + slot);
                    rv[g][j] = __builtin_nontemporal_load(val + slot);
                }
            }
        float rsc[G];  // row scales (BF16 storage)
#pragma unroll
        for (int g = 0; g < G; ++g) rsc[g] = row_scale<VT>(a.P, c[g] >= 0 ? row[g] : 0);
        // the row's own previous value is needed by the shifted kinds, the
        // polynomial accumulator and the basis copy only
        const bool need_prev = KIND != KIND_MONO || POLY || a.copy0 != nullptr;
        double prev[G], prev2[G], acc[G], link0[G], w0[G];
        uint32_t lm[G];  // KIND_GS2: strictly lower slots of the row
        double dg[G];    // KIND_GS2: the row's diagonal entry
        double zr[G];    // KIND_SMOOTH: the current sweep's start value
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const bool act = c[g] >= 0 && row[g] < a.P.n;
            prev[g] = (act && need_prev) ? a.in[row[g]] : 0.0;
            link0[g] = ((KIND == KIND_JCHAIN || split_kind(KIND)) && act) ? a.link_in[row[g]] : 0.0;
            w0[g] = (split_kind(KIND) && act) ? a.pow_in[row[g]] : 0.0;
            lm[g] = 0u;
            dg[g] = 1.0;
            zr[g] = (KIND == KIND_SMOOTH && act) ? a.z_io[row[g]] : 0.0;
            if (split_kind(KIND) && act) {
                lm[g] = a.P.lmask[row[g]];
                dg[g] = decode<VT>(val[off[g] + (int64_t)a.P.dslot[row[g]] * kChunkRows + lane], rsc[g]);
            }
            prev2[g] = (KIND == KIND_CHEB && act && a.prev2) ? a.prev2[row[g]] : 0.0;
            if (a.copy0 && act) a.copy0[row[g]] = prev[g];
            acc[g] = 0.0;
            if (POLY && act) acc[g] = a.acc_in ? a.acc_in[row[g]] : a.c0 * prev[g];
        }
        for (int kl = 0; kl < a.q; ++kl) {
            const double* src = kl == 0 ? a.in : dest(a, kl - 1);
            // the first sub-power of a GS2 power (g_0 = D^{-1} w) is row-local: no
            // dependency wait and no gather
            const bool local = KIND == KIND_GS2 && (a.base + kl) % a.C.jk == 0;
            if (kl > 0 && !local) {
                const uint32_t target = a.epoch * 16u + (uint32_t)kl;
                bool ok[1] = {!need};
                if (!poll_until<1>(a, dr, wo, ok, target, c[0], kl)) return;
                if (long_list) {  // dependency lists longer than one wave
                    for (int b = d0 + 64; b < d1; b += 64) {
                        const int i = b + lane;
                        const uint32_t wx[1] = {(uint32_t)(i < d1 ? a.P.dep_idx[i] : 0) * (4u * kFlagStride)};
                        bool okx[1] = {!(i < d1)};
                        if (!poll_until<1>(a, dr, wx, okx, target, c[0], kl)) return;
                    }
                }
                asm volatile("" ::: "memory");
            }
            double s[G], sl[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                s[g] = 0.0;
                sl[g] = 0.0;
                if (local) continue;
                // gathers by 32-bit row index through a buffer resource (no 64-bit
                // addresses to keep across the powers); padding slots (column -1,
                // value 0) gather 0.0 and add an exact +0 to a sum that starts at +0
                const gi32x4 xr = vec_rsrc(src, a.P.n);
                double xv[REG];
                if (kl == 0 || a.plain_gather) {
#pragma unroll
                    for (int j = 0; j < REG; ++j) xv[j] = gather<0>(xr, rc[g][j]);
                } else {
#pragma unroll
                    for (int j = 0; j < REG; ++j) xv[j] = gather<16>(xr, rc[g][j]);
                }
#pragma unroll
                for (int j = 0; j < REG; ++j) {
                    VT r = rv[g][j];
                    // keep narrow values narrow in registers: convert at each use
                    // instead of letting the compiler hoist a widened copy
                    if constexpr (sizeof(VT) < 8) asm volatile("" : "+v"(r));
                    s[g] = fma(decode<VT>(r, rsc[g]), xv[j], s[g]);
                    if (split_kind(KIND) && ((lm[g] >> j) & 1u)) sl[g] = fma(decode<VT>(r, rsc[g]), xv[j], sl[g]);
                }
            }
            // slots beyond the register cache, streamed at every power.  The wide-row
            // kernels, which rely on this path, take eight slots per batch (columns and
            // values, then the gathers: two round trips per batch); the others take one
            // slot at a time (plans use them only when the caller caps the slots), in a
            // loop whose form leaves the rest of these kernels' schedule as it was
            // (the batched form measured 12-16 % slower on the GS2 chain there).
            if constexpr (REG >= 16) {
                constexpr int kTB = 8;
#pragma unroll
                for (int g = 0; g < G; ++g)
                    for (int j0 = REG; j0 < (local ? 0 : width[g]); j0 += kTB) {
                        int cj[kTB];
                        double vj[kTB], xj[kTB];
#pragma unroll
                        for (int t = 0; t < kTB; ++t) {
                            cj[t] = -1;
                            vj[t] = 0.0;
                            if (j0 + t < width[g]) {
                                const int64_t slot = off[g] + (int64_t)(j0 + t) * kChunkRows + lane;
                                cj[t] = a.P.col[slot];
                                vj[t] = decode<VT>(val[slot], rsc[g]);
                            }
                        }
#pragma unroll
                        for (int t = 0; t < kTB; ++t)
                            xj[t] = cj[t] < 0 ? 0.0
                                              : (kl == 0 || a.plain_gather ? src[cj[t]] : load_coherent(src + cj[t]));
#pragma unroll
                        for (int t = 0; t < kTB; ++t)
                            if (cj[t] >= 0) {
                                s[g] = fma(vj[t], xj[t], s[g]);
                                if (split_kind(KIND) && j0 + t < 32 && ((lm[g] >> (j0 + t)) & 1u))
                                    sl[g] = fma(vj[t], xj[t], sl[g]);
                            }
                    }
            } else {
#pragma unroll
                for (int g = 0; g < G; ++g)
                    for (int j = REG; j < (local ? 0 : width[g]); ++j) {
                        const int64_t slot = off[g] + (int64_t)j * kChunkRows + lane;
                        const int cj = a.P.col[slot];
                        if (cj >= 0) {
                            const double vj = decode<VT>(val[slot], rsc[g]);
                            const double xj = kl == 0 || a.plain_gather ? src[cj] : load_coherent(src + cj);
                            s[g] = fma(vj, xj, s[g]);
                            if (split_kind(KIND) && j < 32 && ((lm[g] >> j) & 1u)) sl[g] = fma(vj, xj, sl[g]);
                        }
                    }
            }
            double* dst = dest(a, kl);
            const bool last = kl + 1 == a.q;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                double y;
                if constexpr (KIND == KIND_SMOOTH) {
                    const int r = (a.base + kl) % a.C.jk;
                    const bool act = c[g] >= 0 && row[g] < a.P.n;
                    const bool fin = a.base + kl + 1 == a.C.chain_len;
                    y = smooth_value(s[g], sl[g], zr[g], link0[g], dg[g], w0[g], r, a.C.jk, fin);
                    if (fin) {
                        if (act) a.res_out[row[g]] = y;
                    } else if (r == a.C.jk - 1) {
                        zr[g] = y;  // the next sweep starts here
                        if (act) a.z_io[row[g]] = y;
                    }
                } else if constexpr (KIND == KIND_GS2) {
                    const int r = (a.base + kl) % a.C.jk;
                    if (r == 0) w0[g] = prev[g];  // the power's input
                    y = gs2_value(s[g], sl[g], prev[g], link0[g], dg[g], w0[g], r, a.C.jk, a.C.pinv, a.C.lam[kl],
                                  a.C.sig[kl]);
                    if (r == 0) link0[g] = y;  // g_0 of this power
                    if (r == a.C.jk - 1 && c[g] >= 0 && row[g] < a.P.n)
                        a.link_out[(int64_t)((a.base + kl) / a.C.jk) * a.link_ld + row[g]] = y;
                } else {
                    y = finish<KIND>(s[g], prev[g], prev2[g], link0[g], a.base + kl + 1, kl, a.C);
                }
                if (c[g] >= 0 && row[g] < a.P.n) {
                    if (!last) store_coherent(dst + row[g], y);
                    else dst[row[g]] = y;  // nobody reads the last power in this launch
                }
                if (KIND == KIND_JCHAIN && (a.base + kl + 1) % a.C.jk == 0) {
                    link0[g] = y;  // the link closes: w_j starts the next one
                    if (c[g] >= 0 && row[g] < a.P.n)
                        a.link_out[(int64_t)((a.base + kl + 1) / a.C.jk - 1) * a.link_ld + row[g]] = y;
                }
                if (POLY) acc[g] = fma(a.C.c[kl], y, acc[g]);
                prev2[g] = prev[g];
                prev[g] = y;
            }
            if (!last) {
                // publish power kl+1 of the unit's chunks once all their stores
                // completed, in the completion word of its first chunk
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                if (lane == 0)
                    __hip_atomic_store(a.P.done + kFlagStride * c[0], a.epoch * 16u + (uint32_t)(kl + 1),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (POLY) {
#pragma unroll
            for (int g = 0; g < G; ++g)
                if (c[g] >= 0 && row[g] < a.P.n) a.acc_out[row[g]] = acc[g];
        }
    }
}

// ---- staged kernel: one stage of the level-group wavefront ------------------
// A stage holds at most q tasks (one per power of the block), each a range of
// permuted rows.  Waves stride over the chunks that cover all the tasks' rows;
// every lane computes its row sum, and only rows inside the task are stored.
struct StageTaskDev {
    const double* in;     // y_{gk-1}
    const double* prev2;  // y_{gk-2} (Chebyshev), null for gk < 2
    const double* link_in;  // KIND_JCHAIN: the chain's value at the start of the link
    const double* pow_in;   // KIND_GS2: the input w0 of the power
    double* out;          // y_gk
    int c0, nchunks;      // chunks covering rows [r0, r1)
    int r0, r1;
    int gk, kl;           // global power; its index in the coefficient arrays
};

struct StageArgs {
    DevPlan P;
    StageTaskDev t[kMaxQ];
    int ntasks;
    double* acc;  // polynomial accumulator, updated in place (null: none)
    double c0;
    double* link_out;  // KIND_JCHAIN: output column j - 1 receives w_j
    int64_t link_ld;
    double* z_io;      // KIND_SMOOTH: the current sweep's start z, rewritten as a sweep closes
    double* res_out;   // KIND_SMOOTH: receives the residual of the final sub-power
    Coefs C;
};

template <int KIND, bool POLY, typename VT>
__global__ __launch_bounds__(kBlockThreads) void stage_kernel(StageArgs a) {
    const int lane = threadIdx.x & 63;
    const int W = gridDim.x * kWaves;
    int total = 0;
    for (int t = 0; t < a.ntasks; ++t) total += a.t[t].nchunks;
    for (int i = blockIdx.x * kWaves + (threadIdx.x >> 6); i < total; i += W) {
        int t = 0, first = 0;
        while (i >= first + a.t[t].nchunks) first += a.t[t++].nchunks;
        const StageTaskDev& T = a.t[t];
        const int c = T.c0 + (i - first);
        const int row = c * kChunkRows + lane;
        const int64_t off = a.P.off[c];
        const int width = (int)((a.P.off[c + 1] - off) / kChunkRows);
        if constexpr (split_kind(KIND)) {
            const int r = (T.gk - 1) % a.C.jk;
            double sA = 0.0, sL = 0.0, d = 1.0;
            if (r == 0 && KIND == KIND_GS2) {  // g_0 = D^{-1} w: row-local, only the diagonal entry is read
                if (row < a.P.n)
                    d = decode<VT>(((const VT*)a.P.val)[off + (int64_t)a.P.dslot[row] * kChunkRows + lane],
                                   row_scale<VT>(a.P, row));
            } else {
                row_sums_gs2<VT>(a.P, T.in, off, width, lane, row, sA, sL, d);
            }
            if (row >= T.r0 && row < T.r1) {
                if constexpr (KIND == KIND_SMOOTH) {
                    const bool fin = T.gk == a.C.chain_len;
                    double g0 = T.link_in[row];
                    const double y = smooth_value(sA, sL, a.z_io[row], g0, d, T.pow_in[row], r, a.C.jk, fin);
                    T.out[row] = y;
                    if (fin) a.res_out[row] = y;
                    else if (r == a.C.jk - 1) a.z_io[row] = y;
                } else {
                    const double y = gs2_value(sA, sL, T.in[row], T.link_in[row], d, T.pow_in[row], r, a.C.jk,
                                               a.C.pinv, a.C.lam[T.kl], a.C.sig[T.kl]);
                    T.out[row] = y;
                    if (r == a.C.jk - 1) a.link_out[(int64_t)((T.gk - 1) / a.C.jk) * a.link_ld + row] = y;
                }
            }
            continue;
        }
        const double s = row_sum_mem<VT>(a.P, T.in, off, width, lane, row);
        if (row >= T.r0 && row < T.r1) {
            const double prev = (KIND != KIND_MONO || POLY) ? T.in[row] : 0.0;
            const double prev2 = (KIND == KIND_CHEB && T.prev2) ? T.prev2[row] : 0.0;
            const double link0 = KIND == KIND_JCHAIN ? T.link_in[row] : 0.0;
            const double y = finish<KIND>(s, prev, prev2, link0, T.gk, T.kl, a.C);
            T.out[row] = y;
            if (KIND == KIND_JCHAIN && T.gk % a.C.jk == 0)
                a.link_out[(int64_t)(T.gk / a.C.jk - 1) * a.link_ld + row] = y;
            if (POLY) {
                const double acc = T.gk == 1 ? a.c0 * prev : a.acc[row];
                a.acc[row] = fma(a.C.c[T.kl], y, acc);
            }
        }
    }
}

__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// dir 0: out[i] = in[perm[i]]; dir 1: out[perm[i]] = in[i]; `nvec` vectors
__global__ void permute_kernel(const double* in, int64_t ld_in, double* out, int64_t ld_out,
                               const int32_t* perm, int32_t n, int dir) {
    const double* src = in + blockIdx.y * ld_in;
    double* dst = out + blockIdx.y * ld_out;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (dir == 0) dst[i] = src[perm[i]];
        else dst[perm[i]] = src[i];
    }
}

// out[row] = the row's diagonal entry of P A P^T as stored (0 if none), level order
template <typename VT>
__global__ void diagonal_kernel(DevPlan P, double* out) {
    const int lane = threadIdx.x & 63;
    const int nchunks = (P.n + kChunkRows - 1) / kChunkRows;
    for (int c = blockIdx.x * kWaves + (threadIdx.x >> 6); c < nchunks; c += gridDim.x * kWaves) {
        const int row = c * kChunkRows + lane;
        if (row >= P.n) continue;
        const int64_t off = P.off[c];
        const int width = (int)((P.off[c + 1] - off) / kChunkRows);
        double d = 0.0;
        for (int j = 0; j < width; ++j) {
            const int64_t slot = off + (int64_t)j * kChunkRows + lane;
            if (P.col[slot] == row) d = decode<VT>(((const VT*)P.val)[slot], row_scale<VT>(P, row));
        }
        out[row] = d;
    }
}

__global__ void scale_kernel(const double* x, double* out, double a, int32_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = a * x[i];
}

// ---- iterative refinement helpers ------------------------------------------
constexpr int kRedParts = 2048;  // workgroups of the reduction kernels (fixed: deterministic sums)

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Sum of the four waves' values, left by thread 0 in part[blockIdx.x].
__device__ __forceinline__ void block_partial(double v, double* part) {
    __shared__ double red[kWaves];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// r = b - A x with the SpMV kernel's row arithmetic (FP64 sums); each
// workgroup leaves the sum of r_i^2 over its rows in part[blockIdx.x].
template <typename VT>
__global__ __launch_bounds__(kBlockThreads) void residual_kernel(DevPlan P, const double* b, const double* x,
                                                                 double* r, double* part) {
    const int lane = threadIdx.x & 63;
    const int W = gridDim.x * kWaves;
    const int nchunks = (P.n + kChunkRows - 1) / kChunkRows;
    double acc = 0.0;
    for (int c = blockIdx.x * kWaves + (threadIdx.x >> 6); c < nchunks; c += W) {
        const int row = c * kChunkRows + lane;
        const int64_t off = P.off[c];
        const int width = (int)((P.off[c + 1] - off) / kChunkRows);
        const double s = row_sum_mem<VT>(P, x, off, width, lane, row);
        if (row < P.n) {
            const double ri = b[row] - s;
            r[row] = ri;
            acc = fma(ri, ri, acc);
        }
    }
    block_partial(acc, part);
}

__global__ __launch_bounds__(kBlockThreads) void sumsq_kernel(const double* v, int64_t n, double* part) {
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc = fma(v[i], v[i], acc);
    block_partial(acc, part);
}

// One workgroup adds the m partial sums in a fixed order into out[0].
__global__ __launch_bounds__(kBlockThreads) void reduce_kernel(const double* part, int m, double* out) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < m; i += blockDim.x) acc += part[i];
    __shared__ double red[kWaves];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void axpy_kernel(double* x, const double* z, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] += z[i];
}

// ------------------------------------------------------------------ host
thread_local std::string g_err;

mpk_status fail(mpk_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

void set_error_text(const char* msg) { g_err = msg; }

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) return fail(MPK_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
    size_t val, rowscale, col, off, perm, iperm, seq, seq_ptr, unit_ptr, unit_rec, wide_ptr[mpk::kWide], wide_rec[mpk::kWide],
        wide_dep[mpk::kWide], dep_idx, done, tickets, status, lmask, dslot, total;
};

Layout make_layout(const mpk::HostPlan& H) {
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    const size_t slots = H.sell_val.size();
    L.val = take(slots * (H.value_type == MPK_VALUES_BF16_ROWSCALE ? 2 : H.value_type == MPK_VALUES_F32 ? 4 : 8));
    L.rowscale = take(H.value_type == MPK_VALUES_BF16_ROWSCALE ? (size_t)H.nchunks * kChunkRows * 4 : 0);
    L.col = take(slots * 4);
    L.off = take((H.nchunks + 1) * 8);
    L.perm = take((size_t)H.n * 4);
    L.iperm = take((size_t)H.n * 4);
    L.seq = take((size_t)H.nchunks * 4);
    L.seq_ptr = take((kParts + 1) * 4);
    L.unit_ptr = take((kParts + 1) * 4);
    L.unit_rec = take(std::max<size_t>(1, H.units.rec.size()) * 4);
    for (int i = 0; i < mpk::kWide; ++i) {
        L.wide_ptr[i] = take(H.wide[i].ptr.size() * 4);
        L.wide_rec[i] = take(H.wide[i].rec.size() * 4);
        L.wide_dep[i] = take(H.wide[i].dep_idx.size() * 4);
    }
    L.dep_idx = take(std::max<size_t>(1, H.units.dep_idx.size()) * 4);
    L.done = take(std::max<size_t>(1, H.nchunks) * 4 * kFlagStride);
    L.tickets = take(4 * kParts * 4 * kFlagStride);
    L.status = take(kStatusSlots * 4 * kFlagStride);
    L.lmask = take(H.lmask.size() * 4);
    L.dslot = take(H.dslot.size() * 4);
    L.total = o;
    return L;
}

}  // namespace

struct mpk_plan_s {
    mpk::HostPlan H;
    Layout L{};
    char* dev = nullptr;  // caller-owned device buffer once uploaded
    DevPlan D{};
    uint32_t epoch = 0;
    // blocked launch shape per operator variant [kind][poly]: every workgroup
    // must be resident at once, so the grid is the variant's occupancy limit
    int workers[kKinds][2] = {};  // waves per partition
    int grid_block[kKinds][2] = {};
    int q_eff[kKinds][2] = {};    // powers per launch meeting the deadlock bound
    int reg[kKinds][2] = {};      // register slots per row of the kernel in use
    int group[kKinds][2] = {};    // chunks per worker of the kernel in use (H.units or H.wide)
    const int32_t* wide_ptr[mpk::kWide] = {};  // device copies of H.wide
    const int32_t* wide_rec[mpk::kWide] = {};
    const int32_t* wide_dep[mpk::kWide] = {};
    int grid_spmv = 0;       // workgroups of a plain launch
    int cus = 0;             // compute units of the device the plan was uploaded on
    int column_scaling = MPK_SCALE_NONE;             // the plan holds A, or B = A D^{-1}
    int q_cap = 0;                                   // powers per blocked launch at most (0: none)
    std::vector<std::vector<mpk::StageTask>> sched;  // wavefront schedule per q (lazy, under mu)
    // status slot of each calling stream (device failures are reported to the
    // stream whose launch failed), with a use stamp for reuse
    std::vector<std::pair<void*, uint64_t>> status_owner = std::vector<std::pair<void*, uint64_t>>(kStatusSlots);
    uint64_t status_clock = 0;
    std::mutex mu;
};

namespace {

using BlockFn = void (*)(BlockArgs);
using SpmvFn = void (*)(SpmvArgs);

template <int G, int KIND, bool POLY, typename VT>
BlockFn block_fn(int reg) {
    switch (reg) {
        case 4: return mpk_block_kernel<4, G, KIND, POLY, VT>;
        case 7: return mpk_block_kernel<7, G, KIND, POLY, VT>;
        case 8: return mpk_block_kernel<8, G, KIND, POLY, VT>;
        case 16: return mpk_block_kernel<16, G, KIND, POLY, VT>;
        default: break;
    }
    // 32 register slots exist with one chunk per worker only (the planner
    // sets G = 1 for such rows), so only G = 1 instantiates them
    if constexpr (G == 1) return reg == 32 ? mpk_block_kernel<32, 1, KIND, POLY, VT> : nullptr;
    return nullptr;
}

template <int G, typename VT>
BlockFn pick_block_g(int reg, int kind, bool poly) {
    if (kind == KIND_JCHAIN) return block_fn<G, KIND_JCHAIN, false, VT>(reg);  // never polynomial
    if (kind == KIND_GS2) return block_fn<G, KIND_GS2, false, VT>(reg);
    if (kind == KIND_SMOOTH) return block_fn<G, KIND_SMOOTH, false, VT>(reg);
    if (kind == KIND_MONO)
        return poly ? block_fn<G, KIND_MONO, true, VT>(reg) : block_fn<G, KIND_MONO, false, VT>(reg);
    if (kind == KIND_NEWTON)
        return poly ? block_fn<G, KIND_NEWTON, true, VT>(reg) : block_fn<G, KIND_NEWTON, false, VT>(reg);
    return poly ? block_fn<G, KIND_CHEB, true, VT>(reg) : block_fn<G, KIND_CHEB, false, VT>(reg);
}

template <typename VT>
BlockFn pick_block_vt(int reg, int group, int kind, bool poly) {
    if (reg >= 32 || group == 1) return pick_block_g<1, VT>(reg, kind, poly);
    if (group == 2) return pick_block_g<2, VT>(reg, kind, poly);
    if (group == 4) return pick_block_g<4, VT>(reg, kind, poly);
    return nullptr;
}

// Three, five and six chunks per worker (H.wide): rows of up to 8 slots.  At 7
// slots and FP64 values the three-chunk kernels take 138 to 156 VGPRs (three
// waves per SIMD) and the five-chunk ones 216 to 255 (two); the smoother's
// would drop a wave more than the others, so it has none of them.
template <int G, int KIND, bool POLY, typename VT>
BlockFn block_fn_wide(int reg) {
    switch (reg) {
        case 4: return mpk_block_kernel<4, G, KIND, POLY, VT>;
        case 7: return mpk_block_kernel<7, G, KIND, POLY, VT>;
        case 8: return mpk_block_kernel<8, G, KIND, POLY, VT>;
        default: return nullptr;
    }
}

template <int G, typename VT>
BlockFn pick_block_wide(int reg, int kind, bool poly) {
    switch (kind) {
        case KIND_MONO:
            return poly ? block_fn_wide<G, KIND_MONO, true, VT>(reg) : block_fn_wide<G, KIND_MONO, false, VT>(reg);
        case KIND_NEWTON:
            return poly ? block_fn_wide<G, KIND_NEWTON, true, VT>(reg) : block_fn_wide<G, KIND_NEWTON, false, VT>(reg);
        case KIND_CHEB:
            return poly ? block_fn_wide<G, KIND_CHEB, true, VT>(reg) : block_fn_wide<G, KIND_CHEB, false, VT>(reg);
        case KIND_JCHAIN: return block_fn_wide<G, KIND_JCHAIN, false, VT>(reg);
        // the GS2 chain measured 7-9 % slower at five chunks (two waves) than at three
        case KIND_GS2: return G == 3 ? block_fn_wide<G, KIND_GS2, false, VT>(reg) : nullptr;
        default: return nullptr;
    }
}

template <typename VT>
BlockFn pick_block_wide_vt(int group, int reg, int kind, bool poly) {
    if (group == 3) return pick_block_wide<3, VT>(reg, kind, poly);
    if (group == 5) return pick_block_wide<5, VT>(reg, kind, poly);
    // six chunks: the plain powers at 7 slots with FP64 or FP32 values only,
    // held to two waves per SIMD (FP64: 3 registers spill); 2-3 % faster than
    // five at 160^3 (166 against 169 us for a block of 4 powers, 284 against
    // 294 us for 8).  BF16 values and 8 slots spill far more.
    if constexpr (sizeof(VT) >= 4)
        if (group == 6 && kind == KIND_MONO && !poly && reg == 7) return mpk_block_kernel<7, 6, KIND_MONO, false, VT>;
    return nullptr;
}

// The planner keeps one chunk per worker when rows need more than 16 slots.
BlockFn pick_block(const mpk::HostPlan& H, int group, int reg, int kind, bool poly) {
    // every group of an extra unit table goes to the kernels built for that group (a
    // kernel of another G would leave part of each unit's chunks undone)
    if (group != 1 && group != 2 && group != 4) {
        if (H.value_type == MPK_VALUES_BF16_ROWSCALE) return pick_block_wide_vt<uint16_t>(group, reg, kind, poly);
        return H.value_type == MPK_VALUES_F32 ? pick_block_wide_vt<float>(group, reg, kind, poly)
                                              : pick_block_wide_vt<double>(group, reg, kind, poly);
    }
    if (H.value_type == MPK_VALUES_BF16_ROWSCALE) return pick_block_vt<uint16_t>(reg, group, kind, poly);
    return H.value_type == MPK_VALUES_F32 ? pick_block_vt<float>(reg, group, kind, poly)
                                          : pick_block_vt<double>(reg, group, kind, poly);
}

template <typename VT>
SpmvFn pick_spmv_vt(int kind, bool poly) {
    if (kind == KIND_JCHAIN) return spmv_kernel<KIND_JCHAIN, false, VT>;
    if (kind == KIND_GS2) return spmv_kernel<KIND_GS2, false, VT>;
    if (kind == KIND_SMOOTH) return spmv_kernel<KIND_SMOOTH, false, VT>;
    if (kind == KIND_MONO) return poly ? spmv_kernel<KIND_MONO, true, VT> : spmv_kernel<KIND_MONO, false, VT>;
    if (kind == KIND_NEWTON) return poly ? spmv_kernel<KIND_NEWTON, true, VT> : spmv_kernel<KIND_NEWTON, false, VT>;
    return poly ? spmv_kernel<KIND_CHEB, true, VT> : spmv_kernel<KIND_CHEB, false, VT>;
}

using StageFn = void (*)(StageArgs);
template <typename VT>
StageFn pick_stage_vt(int kind, bool poly) {
    if (kind == KIND_JCHAIN) return stage_kernel<KIND_JCHAIN, false, VT>;
    if (kind == KIND_GS2) return stage_kernel<KIND_GS2, false, VT>;
    if (kind == KIND_SMOOTH) return stage_kernel<KIND_SMOOTH, false, VT>;
    if (kind == KIND_MONO) return poly ? stage_kernel<KIND_MONO, true, VT> : stage_kernel<KIND_MONO, false, VT>;
    if (kind == KIND_NEWTON)
        return poly ? stage_kernel<KIND_NEWTON, true, VT> : stage_kernel<KIND_NEWTON, false, VT>;
    return poly ? stage_kernel<KIND_CHEB, true, VT> : stage_kernel<KIND_CHEB, false, VT>;
}

StageFn pick_stage(const mpk::HostPlan& H, int kind, bool poly) {
    if (H.value_type == MPK_VALUES_BF16_ROWSCALE) return pick_stage_vt<uint16_t>(kind, poly);
    return H.value_type == MPK_VALUES_F32 ? pick_stage_vt<float>(kind, poly) : pick_stage_vt<double>(kind, poly);
}

SpmvFn pick_spmv(const mpk::HostPlan& H, int kind, bool poly) {
    if (H.value_type == MPK_VALUES_BF16_ROWSCALE) return pick_spmv_vt<uint16_t>(kind, poly);
    return H.value_type == MPK_VALUES_F32 ? pick_spmv_vt<float>(kind, poly) : pick_spmv_vt<double>(kind, poly);
}

int grid_1d(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(4096, (n + 255) / 256)); }

// Vectors in the ring of a polynomial: q + 2 (one launch's q outputs, its
// input and, for Chebyshev, the power before it stay distinct, so the
// launch may gather with plain loads).
int poly_ring(mpk_plan_t p) { return p->H.p_block + 2; }

mpk_status check_uploaded(mpk_plan_t p) {
    if (!p) return fail(MPK_ERR_ARG, "null plan");
    if (!p->dev) return fail(MPK_ERR_STATE, "plan has no device buffer: call mpk_upload first");
    return MPK_OK;
}

// Blocked launches run one at a time per device, whatever stream or plan they
// come from: a persistent kernel needs enough of its waves resident together,
// and two at once could each hold part of the GPU while waiting for the rest.
// Each launch waits for an event recorded after the previous one; all other
// work keeps overlapping.
struct BlockedChain {
    std::mutex mu;
    hipEvent_t last = nullptr;
    bool recorded = false;
};
BlockedChain g_chain[16];

// Status slot of `stream` on plan p: assigned on the stream's first blocked
// launch, the least recently used slot reused once all are taken.  Returns
// null for a stream that has none when `assign` is false.
int32_t* status_slot(mpk_plan_t p, void* stream, bool assign) {
    std::lock_guard<std::mutex> lk(p->mu);
    int pick = -1;
    for (int i = 0; i < kStatusSlots; ++i)
        if (p->status_owner[i].second != 0 && p->status_owner[i].first == stream) pick = i;
    if (pick < 0) {
        if (!assign) return nullptr;
        pick = 0;
        for (int i = 1; i < kStatusSlots; ++i)
            if (p->status_owner[i].second < p->status_owner[pick].second) pick = i;
        p->status_owner[pick].first = stream;
    }
    p->status_owner[pick].second = ++p->status_clock;
    return (int32_t*)(p->dev + p->L.status) + (size_t)pick * kFlagStride;
}

// Launches the blocked kernel for powers base+1 .. base+q.
mpk_status launch_block(mpk_plan_t p, hipStream_t st, int kind, bool poly, BlockArgs a) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    BlockedChain& ch = g_chain[dev & 15];
    std::lock_guard<std::mutex> lk(ch.mu);
    if (!ch.last) HIP_TRY(hipEventCreateWithFlags(&ch.last, hipEventDisableTiming));
    if (ch.recorded) HIP_TRY(hipStreamWaitEvent(st, ch.last, 0));
    if (p->epoch + 1 >= kEpochLimit) {  // restart the done words from zero
        const int64_t nc = (int64_t)std::max<int32_t>(1, p->H.nchunks) * kFlagStride;
        fill_u32_kernel<<<grid_1d(nc), 256, 0, st>>>(p->D.done, nc, 0u);
        HIP_TRY(hipGetLastError());
        fill_u32_kernel<<<8, 256, 0, st>>>(p->D.tickets, 4 * kParts * kFlagStride, 0u);
        HIP_TRY(hipGetLastError());
        p->epoch = 0;
    }
    a.P = p->D;
    const int group = p->group[kind][poly];
    for (int i = 0; i < mpk::kWide; ++i)
        if (group == mpk::kWideGroups[i]) {
            a.P.unit_ptr = p->wide_ptr[i];
            a.P.unit_rec = p->wide_rec[i];
            a.P.dep_idx = p->wide_dep[i];
            a.P.ndeps = (int32_t)p->H.wide[i].dep_idx.size();
        }
    a.epoch = ++p->epoch;
    a.workers = p->workers[kind][poly];
    a.status = status_slot(p, st, true);
    a.spin_limit = p->H.watchdog == 0 ? kSpinLimit : p->H.watchdog;
    const BlockFn fn = pick_block(p->H, group, p->reg[kind][poly], kind, poly);
    if (!fn) return fail(MPK_ERR_UNSUPPORTED, "no blocked kernel for this row width and group");
    hipLaunchKernelGGL(fn, dim3(p->grid_block[kind][poly]),
                       dim3(kBlockThreads), 0, st, a);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(ch.last, st));
    ch.recorded = true;
    return MPK_OK;
}

mpk_status launch_spmv(mpk_plan_t p, hipStream_t st, int kind, bool poly, SpmvArgs a) {
    a.P = p->D;
    hipLaunchKernelGGL(pick_spmv(p->H, kind, poly), dim3(p->grid_spmv), dim3(kBlockThreads), 0, st, a);
    HIP_TRY(hipGetLastError());
    return MPK_OK;
}

mpk_status permute_vecs(mpk_plan_t p, hipStream_t st, const double* in, int64_t ld_in, double* out,
                        int64_t ld_out, int nvec, int dir) {
    if (p->H.n == 0 || nvec == 0) return MPK_OK;
    const int32_t* perm = (const int32_t*)(p->dev + p->L.perm);
    permute_kernel<<<dim3(grid_1d(p->H.n), nvec), 256, 0, st>>>(in, ld_in, out, ld_out, perm, p->H.n, dir);
    HIP_TRY(hipGetLastError());
    return MPK_OK;
}

// Runs the p powers of one operator kind.  dest_k(k) gives the destination of
// y_k (k >= 1).  For POLY the accumulator `acc` (n) receives sum c_k y_k.
struct PowerJob {
    int kind = KIND_MONO;
    bool poly = false;
    int p = 0;
    const double* x = nullptr;  // y_0
    double* out0 = nullptr;     // destinations: out0 + ((k-1) % mod) * ld
    int64_t ld = 0;
    int mod = 1 << 30;
    double* copy0 = nullptr;
    double* acc = nullptr;
    std::vector<double> lam, sig, c;  // per global power k (index k-1); c[0] = c_0
    double theta = 0, delta = 1;
    int jk = 1;                 // KIND_JCHAIN: sub-powers per link; KIND_GS2: per power
    int pinv = 0;               // KIND_GS2: apply P^{-1} only
    double jc = 0;              // KIND_JCHAIN: coefficient of (B - I)^k closing a link
    double* link_out = nullptr; // KIND_JCHAIN: w_j (j = 1..p / jk) at link_out + (j-1) * link_ld
    int64_t link_ld = 0;
    const double* rhs = nullptr; // KIND_SMOOTH: b
    double* z_io = nullptr;     // KIND_SMOOTH: z at the start of the current sweep (in/out)
    double* res_out = nullptr;  // KIND_SMOOTH: the residual of the final sub-power
};

double* job_dest(const PowerJob& j, int k) { return j.out0 + (int64_t)((k - 1) % j.mod) * j.ld; }
const double* job_vec(const PowerJob& j, int k) { return k == 0 ? j.x : job_dest(j, k); }
// KIND_JCHAIN: the chain's value at the start of the link that holds sub-power k.
// KIND_GS2: g_0 of the power that holds sub-power k (the ring slot of the power's
// first sub-power; any valid vector when k is itself that first sub-power).
const double* link_start(const PowerJob& j, int k) {
    const int t = (k - 1) / j.jk * j.jk;
    if (split_kind(j.kind)) return t + 1 < k ? job_dest(j, t + 1) : job_vec(j, t);
    return t == 0 ? j.x : j.link_out + (int64_t)(t / j.jk - 1) * j.link_ld;
}
// KIND_GS2: the input of the power that holds sub-power k (x, or the ring slot of the
// previous power's closing sub-power); the smoother: b
const double* power_start(const PowerJob& j, int k) {
    return j.kind == KIND_SMOOTH ? j.rhs : job_vec(j, (k - 1) / j.jk * j.jk);
}
void set_chain(const PowerJob& j, Coefs& C) {
    C.jk = j.jk;
    C.jc = j.jc;
    C.pinv = j.pinv;
    C.chain_len = j.p;
}

const std::vector<mpk::StageTask>& schedule(mpk_plan_t p, int q) {
    std::lock_guard<std::mutex> lk(p->mu);  // sched is sized at plan creation: no reallocation
    if (p->sched[q].empty()) p->sched[q] = mpk::wavefront_schedule(p->H, q);
    return p->sched[q];
}

// The level-group wavefront (readings R14, R15): blocks of q powers, each as
// G + q - 1 stage launches.
mpk_status run_staged(mpk_plan_t p, hipStream_t st, const PowerJob& j) {
    if (j.copy0) HIP_TRY(hipMemcpyAsync(j.copy0, j.x, sizeof(double) * p->H.n, hipMemcpyDeviceToDevice, st));
    const StageFn fn = pick_stage(p->H, j.kind, j.poly);
    for (int base = 0; base < j.p; base += p->H.p_block) {
        const int qb = std::min(p->H.p_block, j.p - base);
        const auto& tasks = schedule(p, qb);
        for (size_t t0 = 0; t0 < tasks.size();) {
            StageArgs a{};
            a.P = p->D;
            a.acc = j.poly ? j.acc : nullptr;
            a.c0 = j.poly ? j.c[0] : 0.0;
            a.C.theta = j.theta;
            a.C.delta = j.delta;
            set_chain(j, a.C);
            a.link_out = j.link_out;
            a.link_ld = j.link_ld;
            a.z_io = j.z_io;
            a.res_out = j.res_out;
            int total = 0;
            size_t t1 = t0;
            for (; t1 < tasks.size() && tasks[t1].stage == tasks[t0].stage; ++t1) {
                const auto& T = tasks[t1];
                const int gk = base + T.k, kl = T.k - 1;
                StageTaskDev& d = a.t[a.ntasks++];
                d.in = job_vec(j, gk - 1);
                d.prev2 = (j.kind == KIND_CHEB && gk >= 2) ? job_vec(j, gk - 2) : nullptr;
                d.link_in = (j.kind == KIND_JCHAIN || split_kind(j.kind)) ? link_start(j, gk) : nullptr;
                d.pow_in = split_kind(j.kind) ? power_start(j, gk) : nullptr;
                d.out = job_dest(j, gk);
                d.r0 = T.row_begin;
                d.r1 = T.row_end;
                d.c0 = T.row_begin / kChunkRows;
                d.nchunks = (T.row_end - 1) / kChunkRows - d.c0 + 1;
                d.gk = gk;
                d.kl = kl;
                a.C.lam[kl] = j.lam.empty() ? 0.0 : j.lam[gk - 1];
                a.C.sig[kl] = j.sig.empty() ? 1.0 : j.sig[gk - 1];
                a.C.c[kl] = j.poly ? j.c[gk] : 0.0;
                total += d.nchunks;
            }
            const int grid = std::max(1, std::min(p->cus * 32, (total + kWaves - 1) / kWaves));
            hipLaunchKernelGGL(fn, dim3(grid), dim3(kBlockThreads), 0, st, a);
            HIP_TRY(hipGetLastError());
            t0 = t1;
        }
    }
    return MPK_OK;
}

// Power k of the job as one full SpMV launch (Alg. 1).
mpk_status plain_power(mpk_plan_t p, hipStream_t st, const PowerJob& j, int k) {
    SpmvArgs a{};
    a.in = job_vec(j, k - 1);
    a.prev2 = (j.kind == KIND_CHEB && k >= 2) ? job_vec(j, k - 2) : nullptr;
    a.out = job_dest(j, k);
    a.acc_in = (j.poly && k >= 2) ? j.acc : nullptr;
    a.acc_out = j.poly ? j.acc : nullptr;
    a.c0 = j.poly ? j.c[0] : 0.0;
    a.gk = k;
    a.C.lam[0] = j.lam.empty() ? 0.0 : j.lam[k - 1];
    a.C.sig[0] = j.sig.empty() ? 1.0 : j.sig[k - 1];
    a.C.c[0] = j.poly ? j.c[k] : 0.0;
    a.C.theta = j.theta;
    a.C.delta = j.delta;
    set_chain(j, a.C);
    a.link_in = (j.kind == KIND_JCHAIN || split_kind(j.kind)) ? link_start(j, k) : nullptr;
    a.pow_in = split_kind(j.kind) ? power_start(j, k) : nullptr;
    a.link_out = j.link_out;
    a.link_ld = j.link_ld;
    a.z_io = j.z_io;
    a.res_out = j.res_out;
    if (k == 1 && j.copy0) {
        HIP_TRY(hipMemcpyAsync(j.copy0, j.x, sizeof(double) * p->H.n, hipMemcpyDeviceToDevice, st));
    }
    return launch_spmv(p, st, j.kind, j.poly, a);
}

mpk_status run_powers(mpk_plan_t p, hipStream_t st, const PowerJob& j, bool plain, bool staged = false) {
    if (j.p == 0) return MPK_OK;
    if (p->H.n == 0) return MPK_OK;
    if (staged && !plain) return run_staged(p, st, j);
    // A block of one power cannot reuse the matrix, and when the deadlock bound
    // admits only one power per launch (levels too wide for the resident waves)
    // every block is such a block: the plain kernel is faster there, and both
    // give bitwise-equal results.
    const int qe = p->q_cap > 0 ? std::min(p->q_eff[j.kind][j.poly], p->q_cap) : p->q_eff[j.kind][j.poly];
    if (plain || qe <= 1) {
        for (int k = 1; k <= j.p; ++k) {
            mpk_status s = plain_power(p, st, j, k);
            if (s != MPK_OK) return s;
        }
        return MPK_OK;
    }
    for (int base = 0; base < j.p; base += qe) {
        const int q = std::min(qe, j.p - base);
        if (q == 1) {  // a one-power block (p = 1, or the remainder)
            mpk_status s = plain_power(p, st, j, base + 1);
            if (s != MPK_OK) return s;
            continue;
        }
        BlockArgs a{};
        a.in = job_vec(j, base);
        a.prev2 = (j.kind == KIND_CHEB && base >= 1) ? job_vec(j, base - 1) : nullptr;
        a.out0 = j.out0;
        a.out_ld = j.ld;
        a.out_mod = j.mod;
        // Plain loads may read the powers written in this launch when no
        // 128-byte line is read before its producer publishes it: the launch
        // writes q slots distinct from each other and from the slots it reads
        // (y_base, and y_{base-1} for Chebyshev), which holds when every power
        // of the job has its own slot or the ring has at least q + 2 slots, and
        // chunks start on line boundaries.  A launch begins with clean caches
        // and producers store through to memory before publishing.  Otherwise
        // device-coherent loads.
        a.plain_gather = (j.mod >= j.p || j.mod >= q + 2) && ((uintptr_t)j.out0 & 127) == 0 &&
                         ((j.ld * 8) & 127) == 0;
        a.base_slot = base % j.mod;
        a.copy0 = base == 0 ? j.copy0 : nullptr;
        a.acc_in = (j.poly && base > 0) ? j.acc : nullptr;
        a.acc_out = j.poly ? j.acc : nullptr;
        a.c0 = j.poly ? j.c[0] : 0.0;
        a.base = base;
        a.q = q;
        for (int kl = 0; kl < q; ++kl) {
            a.C.lam[kl] = j.lam.empty() ? 0.0 : j.lam[base + kl];
            a.C.sig[kl] = j.sig.empty() ? 1.0 : j.sig[base + kl];
            a.C.c[kl] = j.poly ? j.c[base + kl + 1] : 0.0;
        }
        a.C.theta = j.theta;
        a.C.delta = j.delta;
        set_chain(j, a.C);
        a.link_in = (j.kind == KIND_JCHAIN || split_kind(j.kind)) ? link_start(j, base + 1) : nullptr;
        a.pow_in = split_kind(j.kind) ? power_start(j, base + 1) : nullptr;
        a.link_out = j.link_out;
        a.link_ld = j.link_ld;
        a.z_io = j.z_io;
        a.res_out = j.res_out;
        mpk_status s = launch_block(p, st, j.kind, j.poly, a);
        if (s != MPK_OK) return s;
    }
    return MPK_OK;
}

}  // namespace

// =================================================================== C ABI
mpk_status mpk::set_error(mpk_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    set_error_text(buf);
    return s;
}

mpk_status mpk::plan_uploaded(mpk_plan_t p) { return check_uploaded(p); }

int mpk::plan_column_scaling(mpk_plan_t p) { return p ? p->column_scaling : MPK_SCALE_NONE; }

bool mpk::plan_split_lower(mpk_plan_t p) { return p && p->H.split_lower; }

int mpk::plan_p_block(mpk_plan_t p) { return p ? p->H.p_block : 0; }

mpk_status mpk::plan_diagonal(mpk_plan_t p, double* out, void* stream) {
    mpk_status s = check_uploaded(p);
    if (s != MPK_OK || p->H.n == 0) return s;
    hipStream_t st = (hipStream_t)stream;
    const int grid = std::max(1, std::min(p->cus * 8, (p->H.nchunks + kWaves - 1) / kWaves));
    if (p->H.value_type == MPK_VALUES_BF16_ROWSCALE)
        diagonal_kernel<uint16_t><<<grid, kBlockThreads, 0, st>>>(p->D, out);
    else if (p->H.value_type == MPK_VALUES_F32)
        diagonal_kernel<float><<<grid, kBlockThreads, 0, st>>>(p->D, out);
    else
        diagonal_kernel<double><<<grid, kBlockThreads, 0, st>>>(p->D, out);
    HIP_TRY(hipGetLastError());
    return MPK_OK;
}

bool mpk::plan_is_f64(mpk_plan_t p) { return p && p->H.value_type == MPK_VALUES_F64; }

bool mpk::plans_match(mpk_plan_t a, mpk_plan_t b) {
    return a && b && a->H.n == b->H.n && a->H.nnz == b->H.nnz && a->H.perm == b->H.perm;
}

namespace {
// B = A D^{-1} for column_scaling = MPK_SCALE_JACOBI: every value divided by its
// column's diagonal entry, in FP64, into `scaled`, and *val pointed there.
mpk_status column_scaled(int scaling, int32_t n, const int32_t* rowptr, const int32_t* col, const double** val,
                         std::vector<double>& scaled) {
    if (scaling != MPK_SCALE_JACOBI) return MPK_OK;
    try {
        std::vector<double> diag(n, 0.0);
        for (int32_t i = 0; i < n; ++i) {
            for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
                if (col[e] == i) diag[i] = (*val)[e];
            if (diag[i] == 0.0)
                return fail(MPK_ERR_CSR, "row %d has no nonzero diagonal entry (needed by column_scaling)", i);
        }
        const int32_t nnz = n > 0 ? rowptr[n] : 0;
        scaled.resize(nnz);
        for (int32_t e = 0; e < nnz; ++e) scaled[e] = (*val)[e] / diag[col[e]];
    } catch (const std::bad_alloc&) {
        return fail(MPK_ERR_NOMEM, "out of host memory");
    }
    *val = scaled.data();
    return MPK_OK;
}
}  // namespace

MPK_API void mpk_options_default(mpk_options* opt) {
    if (opt) memset(opt, 0, sizeof *opt);
}

MPK_API const char* mpk_version(void) { return "mpk-mi355x 0.1 (gfx950)"; }

MPK_API const char* mpk_last_error(void) { return g_err.c_str(); }

MPK_API mpk_status mpk_build_levels(int32_t n, const int32_t* rowptr, const int32_t* col,
                                    const double* val, const mpk_options* opt,
                                    mpk_plan_t* plan_out, size_t* device_bytes_out) {
    if (!plan_out) return fail(MPK_ERR_ARG, "plan_out is null");
    *plan_out = nullptr;
    if (n < 0) return fail(MPK_ERR_ARG, "n must be >= 0 (got %d)", n);
    if (!rowptr) return fail(MPK_ERR_ARG, "rowptr is null");
    if (n > 0 && rowptr[n] > 0 && (!col || !val)) return fail(MPK_ERR_ARG, "col or val is null");
    mpk_options o{};
    if (opt) o = *opt;
    for (int i = 0; i < 4; ++i)
        if (o.reserved[i] != 0) return fail(MPK_ERR_ARG, "mpk_options.reserved must be zero");
    if (o.split_lower != 0 && o.split_lower != 1) return fail(MPK_ERR_ARG, "split_lower must be 0 or 1");
    if (o.column_scaling != MPK_SCALE_NONE && o.column_scaling != MPK_SCALE_JACOBI)
        return fail(MPK_ERR_ARG, "column_scaling must be MPK_SCALE_NONE (0) or MPK_SCALE_JACOBI (1)");
    if (o.cache_mib < 0) return fail(MPK_ERR_ARG, "cache_mib must be >= 0");
    if (o.min_group_rows < 0) return fail(MPK_ERR_ARG, "min_group_rows must be >= 0");
    if (o.max_reg_slots != 0 && o.max_reg_slots != 4 && o.max_reg_slots != 7 && o.max_reg_slots != 8 &&
        o.max_reg_slots != 16 && o.max_reg_slots != 32)
        return fail(MPK_ERR_ARG, "max_reg_slots must be 0, 4, 7, 8, 16 or 32");
    if (o.value_type < MPK_VALUES_F64 || o.value_type > MPK_VALUES_BF16_ROWSCALE)
        return fail(MPK_ERR_ARG, "value_type must be MPK_VALUES_F64 (0), MPK_VALUES_F32 (1) or "
                                 "MPK_VALUES_BF16_ROWSCALE (2)");
    if (o.root_mode != 0 && o.root_mode != 1) return fail(MPK_ERR_ARG, "root_mode must be 0 or 1");
    if (o.root_mode == 1 && (o.root < 0 || o.root >= n)) return fail(MPK_ERR_ARG, "root out of range");
    if (o.p_block < 0 || o.p_block > mpk::kMaxBlock)
        return fail(MPK_ERR_ARG, "p_block must be in 0..%d", mpk::kMaxBlock);
    if (o.workers_per_xcd < 0) return fail(MPK_ERR_ARG, "workers_per_xcd must be >= 0");
    if (o.chunks_per_worker != 0 && o.chunks_per_worker != 1 && o.chunks_per_worker != 2 &&
        o.chunks_per_worker != 4)
        return fail(MPK_ERR_ARG, "chunks_per_worker must be 0, 1, 2 or 4");
    std::string why = mpk::validate_csr(n, rowptr, col);
    if (!why.empty()) return fail(MPK_ERR_CSR, "%s", why.c_str());
    if (o.split_lower) {  // GS2 needs every diagonal entry and at most 32 entries per row
        for (int32_t i = 0; i < n; ++i) {
            if (rowptr[i + 1] - rowptr[i] > 32)
                return fail(MPK_ERR_UNSUPPORTED, "split_lower supports rows of at most 32 entries (row %d has %d)", i,
                            rowptr[i + 1] - rowptr[i]);
            bool diag = false;
            for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) diag = diag || (col[e] == i && val[e] != 0.0);
            if (!diag) return fail(MPK_ERR_CSR, "row %d has no nonzero diagonal entry (needed by split_lower)", i);
        }
    }
    std::vector<double> scaled;
    mpk_status sc = column_scaled(o.column_scaling, n, rowptr, col, &val, scaled);
    if (sc != MPK_OK) return sc;
    mpk_plan_s* p = new (std::nothrow) mpk_plan_s;
    if (!p) return fail(MPK_ERR_NOMEM, "out of host memory");
    try {
        p->sched.resize(mpk::kMaxBlock + 1);
        p->H.root_mode = o.root_mode;
        p->H.root = o.root;
        p->H.p_block = o.p_block ? o.p_block : 4;
        p->H.workers_req = o.workers_per_xcd;
        p->H.watchdog = o.watchdog_polls;
        p->H.group = o.chunks_per_worker;  // 0: the planner chooses
        p->H.value_type = o.value_type;
        p->H.max_reg = o.max_reg_slots;
        p->H.cache_bytes = (int64_t)(o.cache_mib ? o.cache_mib : 256) << 20;
        p->H.min_group_rows = o.min_group_rows;
        p->column_scaling = o.column_scaling;
        p->H.split_lower = o.split_lower;
        mpk::build_plan(p->H, n, rowptr, col, val);
        p->L = make_layout(p->H);
    } catch (const std::bad_alloc&) {
        delete p;
        return fail(MPK_ERR_NOMEM, "out of host memory while planning");
    }
    if (device_bytes_out) *device_bytes_out = p->L.total;
    *plan_out = p;
    return MPK_OK;
}

namespace {
mpk_status upload_values(mpk_plan_t p, char* d, hipStream_t st);
}

MPK_API mpk_status mpk_update_values(mpk_plan_t p, int32_t n, const int32_t* rowptr, const int32_t* col,
                                     const double* val, void* stream) {
    if (!p) return fail(MPK_ERR_ARG, "null plan");
    if (n != p->H.n) return fail(MPK_ERR_ARG, "n (%d) differs from the plan's (%d)", n, p->H.n);
    if (!rowptr || (n > 0 && rowptr[n] > 0 && (!col || !val))) return fail(MPK_ERR_ARG, "null CSR array");
    std::string why = mpk::validate_csr(n, rowptr, col);
    if (!why.empty()) return fail(MPK_ERR_CSR, "%s", why.c_str());
    uint64_t key[2];
    mpk::pattern_hash(n, rowptr, col, key);
    if (key[0] != p->H.pattern_key[0] || key[1] != p->H.pattern_key[1])
        return fail(MPK_ERR_ARG, "the sparsity pattern differs from the plan's");
    if (p->H.split_lower)
        for (int32_t i = 0; i < n; ++i) {
            bool diag = false;
            for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) diag = diag || (col[e] == i && val[e] != 0.0);
            if (!diag) return fail(MPK_ERR_CSR, "row %d has no nonzero diagonal entry (needed by split_lower)", i);
        }
    std::vector<double> scaled;
    mpk_status s = column_scaled(p->column_scaling, n, rowptr, col, &val, scaled);
    if (s != MPK_OK) return s;
    try {
        mpk::refill_values(p->H, rowptr, col, val);
    } catch (const std::bad_alloc&) {
        return fail(MPK_ERR_NOMEM, "out of host memory");
    }
    if (p->dev) return upload_values(p, p->dev, (hipStream_t)stream);
    return MPK_OK;
}

MPK_API mpk_status mpk_get_levels(mpk_plan_t p, int32_t* nlevels, int32_t* level_ptr,
                                  int32_t* level_of_row, int32_t* perm, int32_t* iperm) {
    if (!p) return fail(MPK_ERR_ARG, "null plan");
    const auto& H = p->H;
    if (nlevels) *nlevels = H.nlevels;
    if (level_ptr) std::copy(H.level_ptr.begin(), H.level_ptr.end(), level_ptr);
    if (level_of_row) std::copy(H.level_of_row.begin(), H.level_of_row.end(), level_of_row);
    if (perm) std::copy(H.perm.begin(), H.perm.end(), perm);
    if (iperm) std::copy(H.iperm.begin(), H.iperm.end(), iperm);
    return MPK_OK;
}

MPK_API mpk_status mpk_get_partition(mpk_plan_t p, int32_t* nchunks, int32_t* chunk_rows,
                                     int32_t* nparts, int32_t* owner) {
    if (!p) return fail(MPK_ERR_ARG, "null plan");
    if (nchunks) *nchunks = p->H.nchunks;
    if (chunk_rows) *chunk_rows = kChunkRows;
    if (nparts) *nparts = kParts;
    if (owner) std::copy(p->H.owner.begin(), p->H.owner.end(), owner);
    return MPK_OK;
}

MPK_API mpk_status mpk_get_deps(mpk_plan_t p, int64_t* ndeps, int32_t* dep_ptr, int32_t* dep_idx) {
    if (!p) return fail(MPK_ERR_ARG, "null plan");
    if (ndeps) *ndeps = (int64_t)p->H.dep_idx.size();
    if (dep_ptr) std::copy(p->H.dep_ptr.begin(), p->H.dep_ptr.end(), dep_ptr);
    if (dep_idx) std::copy(p->H.dep_idx.begin(), p->H.dep_idx.end(), dep_idx);
    return MPK_OK;
}

MPK_API mpk_status mpk_min_workers(mpk_plan_t p, int32_t q, int32_t* w) {
    if (!p || !w) return fail(MPK_ERR_ARG, "null argument");
    if (q < 1 || q > p->H.p_block) return fail(MPK_ERR_ARG, "q must be in 1..p_block (%d)", p->H.p_block);
    *w = p->H.units.min_workers[q];
    return MPK_OK;
}

MPK_API mpk_status mpk_min_workers_units(mpk_plan_t p, int32_t group, int32_t q, int32_t* w) {
    if (!p || !w) return fail(MPK_ERR_ARG, "null argument");
    if (q < 1 || q > p->H.p_block) return fail(MPK_ERR_ARG, "q must be in 1..p_block (%d)", p->H.p_block);
    const mpk::Units* U = group == p->H.units.group ? &p->H.units : nullptr;
    for (const mpk::Units& W : p->H.wide)
        if (group == W.group) U = &W;
    if (!U || group < 1) return fail(MPK_ERR_ARG, "the plan holds no units of %d chunks", group);
    *w = U->min_workers[q];
    return MPK_OK;
}

namespace {
// operator kinds of the ABI (MPK_OP_*) -> kernel kind and polynomial flag
constexpr int kOpKind[8] = {KIND_MONO, KIND_MONO, KIND_NEWTON, KIND_CHEB, KIND_NEWTON, KIND_JCHAIN, KIND_GS2, KIND_SMOOTH};
constexpr int kOpPoly[8] = {0, 1, 1, 1, 0, 0, 0, 0};
}  // namespace

MPK_API mpk_status mpk_block_powers(mpk_plan_t p, int32_t op, int32_t* q) {
    if (!p || !q) return fail(MPK_ERR_ARG, "null argument");
    if (op < 0 || op > 7) return fail(MPK_ERR_ARG, "unknown operator kind %d", op);
    mpk_status s = check_uploaded(p);
    if (s != MPK_OK) return s;
    const int qe = p->q_eff[kOpKind[op]][kOpPoly[op]];
    *q = p->q_cap > 0 ? std::min(qe, p->q_cap) : qe;
    return MPK_OK;
}

MPK_API mpk_status mpk_block_shape(mpk_plan_t p, int32_t op, int32_t* workers, int32_t* group, int32_t* reg) {
    if (!p) return fail(MPK_ERR_ARG, "null plan");
    if (op < 0 || op > 7) return fail(MPK_ERR_ARG, "unknown operator kind %d", op);
    mpk_status s = check_uploaded(p);
    if (s != MPK_OK) return s;
    if (workers) *workers = p->workers[kOpKind[op]][kOpPoly[op]];
    if (group) *group = p->group[kOpKind[op]][kOpPoly[op]];
    if (reg) *reg = p->reg[kOpKind[op]][kOpPoly[op]];
    return MPK_OK;
}

MPK_API mpk_status mpk_plan_info(mpk_plan_t p, int64_t* n, int64_t* nnz, int32_t* nlevels,
                                 int32_t* nchunks, int64_t* sell_slots, int32_t* reg_slots,
                                 int32_t* workers_per_xcd, int32_t* p_block) {
    if (!p) return fail(MPK_ERR_ARG, "null plan");
    if (n) *n = p->H.n;
    if (nnz) *nnz = p->H.nnz;
    if (nlevels) *nlevels = p->H.nlevels;
    if (nchunks) *nchunks = p->H.nchunks;
    if (sell_slots) *sell_slots = (int64_t)p->H.sell_val.size();
    // after upload: the register slots of the plain powers' kernel in use
    if (reg_slots) *reg_slots = p->dev ? p->reg[KIND_MONO][0] : p->H.reg_slots;
    // reported for the plain matrix powers (mpk_apply's blocked kernel)
    if (workers_per_xcd) *workers_per_xcd = p->workers[KIND_MONO][0];
    if (p_block) *p_block = p->dev ? p->q_eff[KIND_MONO][0] : p->H.p_block;
    return MPK_OK;
}

namespace {
// Converts the plan's SELL values to their storage type and copies them (with
// the BF16 row scales) into the bound device buffer on `st`; synchronises `st`.
mpk_status upload_values(mpk_plan_t p, char* d, hipStream_t st) {
    const auto& H = p->H;
    const auto& L = p->L;
    auto put = [&](size_t at, const void* src, size_t nb) -> hipError_t {
        if (nb == 0) return hipSuccess;
        return hipMemcpyAsync(d + at, src, nb, hipMemcpyHostToDevice, st);
    };
    std::vector<float> val32;  // FP32 storage: each value rounded once to nearest
    std::vector<uint16_t> val16;
    std::vector<float> scale;
    if (H.value_type == MPK_VALUES_BF16_ROWSCALE) {
        // per permuted row: s = fl32(max |a|) (1 for an empty or zero row), and
        // each value as the BF16 nearest (ties to even) to fl32(a / s)
        const size_t rows = (size_t)H.nchunks * kChunkRows;
        std::vector<double> amax(rows, 0.0);
        for (int32_t c = 0; c < H.nchunks; ++c)
            for (int64_t sl = H.chunk_off[c]; sl < H.chunk_off[c + 1]; ++sl) {
                const size_t r = (size_t)c * kChunkRows + (size_t)((sl - H.chunk_off[c]) % kChunkRows);
                amax[r] = std::max(amax[r], std::fabs(H.sell_val[sl]));
            }
        scale.resize(rows);
        for (size_t r = 0; r < rows; ++r) scale[r] = amax[r] > 0.0 ? (float)amax[r] : 1.0f;
        val16.resize(H.sell_val.size());
        for (int32_t c = 0; c < H.nchunks; ++c)
            for (int64_t sl = H.chunk_off[c]; sl < H.chunk_off[c + 1]; ++sl) {
                const size_t r = (size_t)c * kChunkRows + (size_t)((sl - H.chunk_off[c]) % kChunkRows);
                const float q = (float)(H.sell_val[sl] / (double)scale[r]);
                uint32_t b;
                std::memcpy(&b, &q, 4);
                val16[sl] = (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
            }
        HIP_TRY(put(L.val, val16.data(), val16.size() * 2));
        HIP_TRY(put(L.rowscale, scale.data(), scale.size() * 4));
    } else if (H.value_type == MPK_VALUES_F32) {
        val32.resize(H.sell_val.size());
        for (size_t i = 0; i < val32.size(); ++i) val32[i] = (float)H.sell_val[i];
        HIP_TRY(put(L.val, val32.data(), val32.size() * 4));
    } else {
        HIP_TRY(put(L.val, H.sell_val.data(), H.sell_val.size() * 8));
    }
    // the host vectors must outlive the asynchronous copies
    HIP_TRY(hipStreamSynchronize(st));
    return MPK_OK;
}
}  // namespace

MPK_API mpk_status mpk_upload(mpk_plan_t p, void* dev_buf, size_t bytes, void* stream) {
    if (!p) return fail(MPK_ERR_ARG, "null plan");
    if (!dev_buf) return fail(MPK_ERR_ARG, "dev_buf is null");
    if (((uintptr_t)dev_buf & 255) != 0) return fail(MPK_ERR_ARG, "dev_buf must be 256-byte aligned");
    if (bytes < p->L.total)
        return fail(MPK_ERR_NOMEM, "device buffer too small: %zu < %zu bytes", bytes, p->L.total);
    hipStream_t st = (hipStream_t)stream;
    const auto& H = p->H;
    const auto& L = p->L;
    char* d = (char*)dev_buf;
    auto put = [&](size_t at, const void* src, size_t nb) -> hipError_t {
        if (nb == 0) return hipSuccess;
        return hipMemcpyAsync(d + at, src, nb, hipMemcpyHostToDevice, st);
    };
    mpk_status vs = upload_values(p, d, st);
    if (vs != MPK_OK) return vs;
    HIP_TRY(put(L.col, H.sell_col.data(), H.sell_col.size() * 4));
    HIP_TRY(put(L.off, H.chunk_off.data(), H.chunk_off.size() * 8));
    HIP_TRY(put(L.perm, H.perm.data(), H.perm.size() * 4));
    HIP_TRY(put(L.iperm, H.iperm.data(), H.iperm.size() * 4));
    HIP_TRY(put(L.seq, H.seq.data(), H.seq.size() * 4));
    HIP_TRY(put(L.seq_ptr, H.seq_ptr.data(), H.seq_ptr.size() * 4));
    HIP_TRY(put(L.unit_ptr, H.units.ptr.data(), H.units.ptr.size() * 4));
    HIP_TRY(put(L.unit_rec, H.units.rec.data(), H.units.rec.size() * 4));
    for (int i = 0; i < mpk::kWide; ++i) {
        HIP_TRY(put(L.wide_ptr[i], H.wide[i].ptr.data(), H.wide[i].ptr.size() * 4));
        HIP_TRY(put(L.wide_rec[i], H.wide[i].rec.data(), H.wide[i].rec.size() * 4));
        HIP_TRY(put(L.wide_dep[i], H.wide[i].dep_idx.data(), H.wide[i].dep_idx.size() * 4));
    }
    HIP_TRY(put(L.dep_idx, H.units.dep_idx.data(), H.units.dep_idx.size() * 4));
    HIP_TRY(put(L.lmask, H.lmask.data(), H.lmask.size() * 4));
    HIP_TRY(put(L.dslot, H.dslot.data(), H.dslot.size() * 4));
    const int64_t nd = (int64_t)std::max<int32_t>(1, H.nchunks) * kFlagStride;
    fill_u32_kernel<<<grid_1d(nd), 256, 0, st>>>((uint32_t*)(d + L.done), nd, 0u);
    HIP_TRY(hipGetLastError());
    fill_u32_kernel<<<8, 256, 0, st>>>((uint32_t*)(d + L.status), kStatusSlots * kFlagStride, 0u);
    HIP_TRY(hipGetLastError());
    fill_u32_kernel<<<8, 256, 0, st>>>((uint32_t*)(d + L.tickets), 4 * kParts * kFlagStride, 0u);
    HIP_TRY(hipGetLastError());
    // the host vectors must outlive the asynchronous copies
    HIP_TRY(hipStreamSynchronize(st));

    DevPlan D{};
    D.val = (const void*)(d + L.val);
    D.rowscale = (const float*)(d + L.rowscale);
    D.col = (const int32_t*)(d + L.col);
    D.off = (const int64_t*)(d + L.off);
    D.seq = (const int32_t*)(d + L.seq);
    D.seq_ptr = (const int32_t*)(d + L.seq_ptr);
    D.unit_ptr = (const int32_t*)(d + L.unit_ptr);
    D.unit_rec = (const int32_t*)(d + L.unit_rec);
    for (int i = 0; i < mpk::kWide; ++i) {
        p->wide_ptr[i] = (const int32_t*)(d + L.wide_ptr[i]);
        p->wide_rec[i] = (const int32_t*)(d + L.wide_rec[i]);
        p->wide_dep[i] = (const int32_t*)(d + L.wide_dep[i]);
    }
    D.ndeps = (int32_t)H.units.dep_idx.size();
    D.dep_idx = (const int32_t*)(d + L.dep_idx);
    D.done = (uint32_t*)(d + L.done);
    D.lmask = (const uint32_t*)(d + L.lmask);
    D.dslot = (const int32_t*)(d + L.dslot);
    D.tickets = (uint32_t*)(d + L.tickets);
    D.n = H.n;
    p->D = D;
    p->dev = d;
    p->epoch = 0;
    {
        std::lock_guard<std::mutex> lk(p->mu);
        for (auto& o : p->status_owner) o = {nullptr, 0};
        p->status_clock = 0;
    }

    // launch shapes: every workgroup of the blocked kernel must be resident at
    // once (waves wait on each other), so its grid is the occupancy limit
    int dev_id = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev_id));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id));
    int maxlen = 0;
    for (int x = 0; x < kParts; ++x) maxlen = std::max(maxlen, H.seq_ptr[x + 1] - H.seq_ptr[x]);
    // one candidate kernel: its powers per launch (qe) and workgroups per partition
    struct Shape {
        int qe = 0, wg_per_part = 0, occ = 0;  // occ: workgroups (= waves per SIMD) per CU
    };
    auto shape_of = [&](BlockFn fn, const mpk::Units& U, Shape& sh) -> mpk_status {
        int occ = 0;
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)fn, kBlockThreads, 0));
        int wg_per_part = std::max(1, (cus / kParts) * std::max(occ, 1));
        if (H.workers_req > 0) wg_per_part = std::min(wg_per_part, std::max(1, H.workers_req / kWaves));
        // no more waves than units
        const int maxunits = (maxlen + U.group - 1) / U.group;
        wg_per_part = std::min(wg_per_part, std::max(1, (maxunits + kWaves - 1) / kWaves));
        // units come from in-order tickets, so only running waves hold work, and
        // every launched workgroup is resident at once on an idle GPU (the grid is
        // the occupancy limit) or starts once the kernels ahead of it finish: a
        // block of q powers needs the deadlock bound within the launched waves
        sh.qe = 1;
        for (int q = H.p_block; q >= 1; --q)
            if (U.min_workers[q] <= wg_per_part * kWaves) {
                sh.qe = q;
                break;
            }
        sh.wg_per_part = wg_per_part;
        sh.occ = occ;
        return MPK_OK;
    };
    for (int kind = 0; kind < kKinds; ++kind)
        for (int poly = 0; poly < 2; ++poly) {
            auto take = [&](const Shape& sh, int reg, int group) {
                p->q_eff[kind][poly] = sh.qe;
                p->reg[kind][poly] = reg;
                p->group[kind][poly] = group;
                p->grid_block[kind][poly] = sh.wg_per_part * kParts;
                p->workers[kind][poly] = sh.wg_per_part * kWaves;
            };
            // wide rows: the kernel holding 32 slots per row in registers and the one
            // holding 16 (streaming the rest at each power) use the same units of
            // one chunk; the leaner one keeps more waves resident, which deep level
            // structures need for a block of q powers.  Take the one that admits
            // more powers per launch, the 32-slot one on a tie.
            const int cand[2] = {H.reg_slots, H.reg_slots >= 32 ? 16 : 0};
            p->q_eff[kind][poly] = 0;
            Shape best;
            for (int ci = 0; ci < 2 && cand[ci] > 0; ++ci) {
                const BlockFn fn = pick_block(H, H.units.group, cand[ci], kind, poly);
                if (!fn) return fail(MPK_ERR_UNSUPPORTED, "no blocked kernel for this plan");
                Shape sh;
                mpk_status ss = shape_of(fn, H.units, sh);
                if (ss != MPK_OK) return ss;
                if (sh.qe > best.qe) {
                    best = sh;
                    take(sh, cand[ci], H.units.group);
                }
            }
            // three, then five chunks per worker where a kernel exists for them: the
            // largest that keeps two waves per SIMD and admits as many powers per
            // launch.  Fewer, larger units cost fewer tickets, polls and store waits
            // per row: at 160^3 with 7 slots a block of 4 powers took 278, 220, 202,
            // 201 and 190 us at 1 to 5 chunks per wave (7, 5, 3, 2 and 2 waves)
            for (int i = 0; i < mpk::kWide; ++i) {
                const mpk::Units& W = H.wide[i];
                const BlockFn fw = W.group > 0 ? pick_block(H, W.group, H.reg_slots, kind, poly) : nullptr;
                if (!fw) continue;
                Shape sh;
                mpk_status ss = shape_of(fw, W, sh);
                if (ss != MPK_OK) return ss;
                if (sh.occ >= 2 && sh.qe >= best.qe) {
                    best = sh;
                    take(sh, H.reg_slots, W.group);
                }
            }
        }
    // plain launches: up to 32 workgroups per CU (128 waves), a few chunks per
    // wave; this measured faster than 8 per CU at the 160^3 Laplacian
    p->grid_spmv = std::max(1, std::min(cus * 32, (H.nchunks + kWaves - 1) / kWaves));
    p->cus = cus;
    return MPK_OK;
}

MPK_API mpk_status mpk_work_bytes(mpk_plan_t p, int32_t call, int32_t pw, uint32_t flags, size_t* bytes) {
    if (!p || !bytes) return fail(MPK_ERR_ARG, "null argument");
    if (pw < 0) return fail(MPK_ERR_ARG, "p must be >= 0");
    const size_t v = (size_t)p->H.n * 8;
    const bool perm = flags & MPK_IO_PERMUTED;
    switch (call) {
        case MPK_CALL_APPLY: *bytes = perm ? 0 : v * (1 + (size_t)pw); break;
        case MPK_CALL_POLY: *bytes = v * (poly_ring(p) + (perm ? 0 : 2)); break;
        case MPK_CALL_SSTEP: *bytes = perm ? 0 : v * (1 + (size_t)pw); break;
        case MPK_CALL_SOLVE: *bytes = v * (2 + poly_ring(p) + (perm ? 0 : 2)) + 8 * (size_t)(kRedParts + 8); break;
        default: return fail(MPK_ERR_ARG, "unknown call kind %d", call);
    }
    return MPK_OK;
}

MPK_API mpk_status mpk_apply(mpk_plan_t p, const double* x, double* Y, int64_t ldy, int32_t pw,
                             uint32_t flags, void* work, size_t work_bytes, void* stream) {
    if (!p) return fail(MPK_ERR_ARG, "null plan");
    if (pw < 1) return fail(MPK_ERR_ARG, "p must be >= 1 (got %d)", pw);
    if (ldy < p->H.n) return fail(MPK_ERR_ARG, "ldy (%lld) < n (%d)", (long long)ldy, p->H.n);
    if (p->H.n > 0 && (!x || !Y)) return fail(MPK_ERR_ARG, "x or Y is null");
    if (flags & ~(MPK_IO_PERMUTED | MPK_PLAIN | MPK_STAGED)) return fail(MPK_ERR_ARG, "unknown flag bits");
    size_t need = 0;
    mpk_work_bytes(p, MPK_CALL_APPLY, pw, flags, &need);
    if (need > 0 && (!work || work_bytes < need))
        return fail(MPK_ERR_ARG, "work buffer too small: %zu < %zu bytes", work_bytes, need);
    mpk_status s = check_uploaded(p);
    if (s != MPK_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    const bool permuted = flags & MPK_IO_PERMUTED;
    PowerJob j;
    j.p = pw;
    if (permuted) {
        j.x = x;
        j.out0 = Y;
        j.ld = ldy;
    } else {
        double* xw = (double*)work;
        s = permute_vecs(p, st, x, 0, xw, 0, 1, 0);
        if (s != MPK_OK) return s;
        j.x = xw;
        j.out0 = xw + p->H.n;
        j.ld = p->H.n;
    }
    s = run_powers(p, st, j, flags & MPK_PLAIN, flags & MPK_STAGED);
    if (s != MPK_OK) return s;
    if (!permuted) s = permute_vecs(p, st, j.out0, p->H.n, Y, ldy, pw, 1);
    return s;
}

MPK_API mpk_status poly_apply(mpk_plan_t p, int32_t kind, int32_t d, const double* c,
                              const double* params, const double* x, double* out, uint32_t flags,
                              void* work, size_t work_bytes, void* stream) {
    if (!p) return fail(MPK_ERR_ARG, "null plan");
    if (d < 0) return fail(MPK_ERR_ARG, "degree must be >= 0 (got %d)", d);
    if (kind < MPK_POLY_MONOMIAL || kind > MPK_POLY_CHEBYSHEV) return fail(MPK_ERR_ARG, "unknown kind %d", kind);
    if (!c) return fail(MPK_ERR_ARG, "coefficients are null");
    if (kind != MPK_POLY_MONOMIAL && d > 0 && !params) return fail(MPK_ERR_ARG, "params are null");
    if (kind == MPK_POLY_CHEBYSHEV && d > 0 && params[1] == 0.0) return fail(MPK_ERR_ARG, "delta must be nonzero");
    if (p->H.n > 0 && (!x || !out)) return fail(MPK_ERR_ARG, "x or out is null");
    if (x == out && p->H.n > 0) return fail(MPK_ERR_ARG, "out must not alias x");
    if (flags & ~(MPK_IO_PERMUTED | MPK_PLAIN | MPK_STAGED)) return fail(MPK_ERR_ARG, "unknown flag bits");
    size_t need = 0;
    mpk_work_bytes(p, MPK_CALL_POLY, d, flags, &need);
    if (need > 0 && (!work || work_bytes < need))
        return fail(MPK_ERR_ARG, "work buffer too small: %zu < %zu bytes", work_bytes, need);
    mpk_status s = check_uploaded(p);
    if (s != MPK_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    const int32_t n = p->H.n;
    if (n == 0) return MPK_OK;
    const bool permuted = flags & MPK_IO_PERMUTED;
    double* w = (double*)work;
    const double* xin = x;
    double* acc = out;
    if (!permuted) {  // level-order copies after the ring
        const size_t ring = (size_t)poly_ring(p) * n;
        s = permute_vecs(p, st, x, 0, w + ring, 0, 1, 0);
        if (s != MPK_OK) return s;
        xin = w + ring;
        acc = w + ring + n;
    }
    if (d == 0) {
        scale_kernel<<<grid_1d(n), 256, 0, st>>>(xin, acc, c[0], n);
        HIP_TRY(hipGetLastError());
    } else {
        PowerJob j;
        j.kind = kind == MPK_POLY_MONOMIAL ? KIND_MONO : kind == MPK_POLY_NEWTON ? KIND_NEWTON : KIND_CHEB;
        j.poly = true;
        j.p = d;
        j.x = xin;
        j.out0 = w;  // ring of poly_ring(p) vectors: t_k in slot (k-1) % mod
        j.ld = n;
        j.mod = poly_ring(p);
        j.acc = acc;
        j.c.assign(c, c + d + 1);
        if (j.kind == KIND_NEWTON) j.lam.assign(params, params + d);
        if (j.kind == KIND_CHEB) {
            j.theta = params[0];
            j.delta = params[1];
        }
        s = run_powers(p, st, j, flags & MPK_PLAIN, flags & MPK_STAGED);
        if (s != MPK_OK) return s;
    }
    if (!permuted) s = permute_vecs(p, st, acc, 0, out, 0, 1, 1);
    return s;
}

// Scratch of poly_apply_static, one copy per GPU (the array's name is a host
// stand-in: host code uses only the device address looked up per device).
static __device__ __align__(256) unsigned char scratch[MPK_STATIC_SCRATCH_BYTES];

namespace {
struct StaticScratch {
    std::mutex mu;
    void* ptr[64] = {};  // device address of `scratch` per device id
};
StaticScratch g_static;

// Device address of the current device's scratch, looked up on the first call
// on that device.
mpk_status static_scratch(void** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(MPK_ERR_UNSUPPORTED, "device id %d beyond the 64 supported", dev);
    std::lock_guard<std::mutex> lk(g_static.mu);
    if (!g_static.ptr[dev]) {
        void* a = nullptr;
        HIP_TRY(hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)));
        g_static.ptr[dev] = a;
    }
    *out = g_static.ptr[dev];
    return MPK_OK;
}
}  // namespace

MPK_API mpk_status poly_apply_static(mpk_plan_t p, int32_t kind, int32_t d, const double* c,
                                     const double* params, const double* x, double* out, uint32_t flags,
                                     void* stream) {
    if (!p) return fail(MPK_ERR_ARG, "null plan");
    size_t need = 0;
    mpk_status s = mpk_work_bytes(p, MPK_CALL_POLY, std::max(d, 0), flags, &need);
    if (s != MPK_OK) return s;
    if (need > MPK_STATIC_SCRATCH_BYTES)
        return fail(MPK_ERR_ARG, "poly_apply_static needs %zu scratch bytes; the static scratch holds %zu",
                    need, (size_t)MPK_STATIC_SCRATCH_BYTES);
    void* w = nullptr;
    s = static_scratch(&w);
    if (s != MPK_OK) return s;
    return poly_apply(p, kind, d, c, params, x, out, flags, w, MPK_STATIC_SCRATCH_BYTES, stream);
}

MPK_API mpk_status mpk_get_schedule(mpk_plan_t p, int32_t q, int32_t* ntasks, int32_t* ngroups, int32_t* tasks) {
    if (!p || !ntasks || !ngroups) return fail(MPK_ERR_ARG, "null argument");
    if (q < 1 || q > mpk::kMaxBlock) return fail(MPK_ERR_ARG, "q must be in 1..%d", mpk::kMaxBlock);
    const auto& T = schedule(p, q);
    *ntasks = (int32_t)T.size();
    *ngroups = (int32_t)mpk::group_levels(p->H, q).size() - 1;
    if (tasks)
        for (size_t i = 0; i < T.size(); ++i) {
            tasks[4 * i + 0] = T[i].stage;
            tasks[4 * i + 1] = T[i].k;
            tasks[4 * i + 2] = T[i].row_begin;
            tasks[4 * i + 3] = T[i].row_end;
        }
    return MPK_OK;
}

MPK_API mpk_status mpk_refine_solve(mpk_plan_t hi, mpk_plan_t lo, int32_t degree, double lmin, double lmax,
                                    const double* b, double* x, double tol, int32_t max_iter, uint32_t flags,
                                    void* work, size_t work_bytes, int32_t* iters_out, double* relres_out,
                                    void* stream) {
    if (iters_out) *iters_out = 0;
    if (relres_out) *relres_out = 0.0;
    if (!hi || !lo) return fail(MPK_ERR_ARG, "null plan");
    if (hi->H.value_type != MPK_VALUES_F64) return fail(MPK_ERR_ARG, "hi must store FP64 values");
    if (hi->H.n != lo->H.n || hi->H.nnz != lo->H.nnz || hi->H.perm != lo->H.perm)
        return fail(MPK_ERR_ARG, "hi and lo must be plans of the same matrix with the same level order");
    if (degree < 1 || degree > 4096) return fail(MPK_ERR_ARG, "degree must be in 1..4096 (got %d)", degree);
    if (!(lmin > 0.0) || !(lmax > lmin)) return fail(MPK_ERR_ARG, "need 0 < lmin < lmax");
    if (!(tol >= 0.0)) return fail(MPK_ERR_ARG, "tol must be >= 0");
    if (max_iter < 0) return fail(MPK_ERR_ARG, "max_iter must be >= 0");
    if (flags & ~(MPK_IO_PERMUTED | MPK_PLAIN | MPK_STAGED)) return fail(MPK_ERR_ARG, "unknown flag bits");
    const int32_t n = hi->H.n;
    if (n > 0 && (!b || !x)) return fail(MPK_ERR_ARG, "b or x is null");
    size_t need = 0;
    mpk_work_bytes(lo, MPK_CALL_SOLVE, degree, flags, &need);
    if (!work || work_bytes < need) return fail(MPK_ERR_ARG, "work buffer too small: %zu < %zu bytes", work_bytes, need);
    mpk_status s = check_uploaded(hi);
    if (s == MPK_OK) s = check_uploaded(lo);
    if (s != MPK_OK) return s;
    if (n == 0) return MPK_OK;
    hipStream_t st = (hipStream_t)stream;
    const bool permuted = flags & MPK_IO_PERMUTED;
    const size_t nn = (size_t)n;
    double* w = (double*)work;
    double* r = w;                // residual
    double* z = w + nn;           // correction
    double* ring = w + 2 * nn;    // Chebyshev vectors
    double* part = w + (2 + poly_ring(lo)) * nn;  // partial sums, then two scalars
    double* sc = part + kRedParts;
    double* bp = (double*)b;
    double* xp = x;
    if (!permuted) {  // level-order copies after the scalars
        bp = sc + 8;
        xp = bp + nn;
        s = permute_vecs(hi, st, b, 0, bp, 0, 1, 0);
        if (s == MPK_OK) s = permute_vecs(hi, st, x, 0, xp, 0, 1, 0);
        if (s != MPK_OK) return s;
    }
    auto norm2 = [&](bool residual, double* out) -> mpk_status {
        if (residual) {
            hipLaunchKernelGGL(hi->H.value_type == MPK_VALUES_F32 ? residual_kernel<float> : residual_kernel<double>,
                               dim3(kRedParts), dim3(kBlockThreads), 0, st, hi->D, (const double*)bp,
                               (const double*)xp, r, part);
        } else {
            sumsq_kernel<<<kRedParts, kBlockThreads, 0, st>>>(bp, n, part);
        }
        HIP_TRY(hipGetLastError());
        reduce_kernel<<<1, kBlockThreads, 0, st>>>(part, kRedParts, sc);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(out, sc, sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        return MPK_OK;
    };
    // Chebyshev interpolant of 1/lam at the d zeros of T_d on [lmin, lmax]: its
    // residual polynomial is T_d((theta - lam)/delta) / T_d(theta/delta)
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
    std::vector<double> coef(degree, 0.0);
    for (int j = 0; j < degree; ++j) {
        const double ang = 3.14159265358979323846 * (j + 0.5) / degree;
        const double inv = 1.0 / (theta + delta * std::cos(ang));
        for (int k = 0; k < degree; ++k) coef[k] += std::cos(k * ang) * inv;
    }
    for (int k = 0; k < degree; ++k) coef[k] *= (k == 0 ? 1.0 : 2.0) / degree;
    double nb2 = 0.0;
    s = norm2(false, &nb2);
    if (s != MPK_OK) return s;
    const double nb = std::sqrt(nb2);
    int it = 0;
    double rel = 0.0;
    for (;; ++it) {
        double rr = 0.0;
        s = norm2(true, &rr);
        if (s != MPK_OK) return s;
        rel = nb > 0.0 ? std::sqrt(rr) / nb : std::sqrt(rr);
        if (rel <= tol || it == max_iter) break;
        if (degree == 1) {
            scale_kernel<<<grid_1d(n), 256, 0, st>>>(r, z, coef[0], n);
            HIP_TRY(hipGetLastError());
        } else {
            PowerJob j;
            j.kind = KIND_CHEB;
            j.poly = true;
            j.p = degree - 1;
            j.x = r;
            j.out0 = ring;
            j.ld = n;
            j.mod = poly_ring(lo);
            j.acc = z;
            j.c = coef;
            j.theta = theta;
            j.delta = delta;
            s = run_powers(lo, st, j, flags & MPK_PLAIN, flags & MPK_STAGED);
            if (s != MPK_OK) return s;
        }
        axpy_kernel<<<grid_1d(n), 256, 0, st>>>(xp, z, n);
        HIP_TRY(hipGetLastError());
    }
    if (!permuted) {
        s = permute_vecs(hi, st, xp, 0, x, 0, 1, 1);
        if (s != MPK_OK) return s;
    }
    if (iters_out) *iters_out = it;
    if (relres_out) *relres_out = rel;
    return MPK_OK;
}

MPK_API mpk_status sstep_basis(mpk_plan_t p, int32_t sdeg, const double* lambda, const double* sigma,
                               const double* v, double* V, int64_t ldv, uint32_t flags, void* work,
                               size_t work_bytes, void* stream) {
    if (!p) return fail(MPK_ERR_ARG, "null plan");
    if (sdeg < 1) return fail(MPK_ERR_ARG, "s must be >= 1 (got %d)", sdeg);
    if (ldv < p->H.n) return fail(MPK_ERR_ARG, "ldv (%lld) < n (%d)", (long long)ldv, p->H.n);
    if (!lambda) return fail(MPK_ERR_ARG, "lambda is null");
    if (sigma)
        for (int k = 0; k < sdeg; ++k)
            if (sigma[k] == 0.0) return fail(MPK_ERR_ARG, "sigma[%d] is zero", k);
    if (p->H.n > 0 && (!v || !V)) return fail(MPK_ERR_ARG, "v or V is null");
    if (flags & ~(MPK_IO_PERMUTED | MPK_PLAIN | MPK_STAGED)) return fail(MPK_ERR_ARG, "unknown flag bits");
    size_t need = 0;
    mpk_work_bytes(p, MPK_CALL_SSTEP, sdeg, flags, &need);
    if (need > 0 && (!work || work_bytes < need))
        return fail(MPK_ERR_ARG, "work buffer too small: %zu < %zu bytes", work_bytes, need);
    mpk_status s = check_uploaded(p);
    if (s != MPK_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    const int32_t n = p->H.n;
    if (n == 0) return MPK_OK;
    const bool permuted = flags & MPK_IO_PERMUTED;
    PowerJob j;
    j.kind = KIND_NEWTON;
    j.p = sdeg;
    j.lam.assign(lambda, lambda + sdeg);
    j.sig = sigma ? std::vector<double>(sigma, sigma + sdeg) : std::vector<double>(sdeg, 1.0);
    double* Vp = V;
    int64_t ld = ldv;
    if (!permuted) {
        Vp = (double*)work;
        ld = n;
        s = permute_vecs(p, st, v, 0, Vp, 0, 1, 0);
        if (s != MPK_OK) return s;
        j.x = Vp;
    } else {
        j.x = v;
        if (v != V) j.copy0 = V;
    }
    j.out0 = Vp + ld;
    j.ld = ld;
    s = run_powers(p, st, j, flags & MPK_PLAIN, flags & MPK_STAGED);
    if (s != MPK_OK) return s;
    if (!permuted) s = permute_vecs(p, st, Vp, ld, V, ldv, sdeg + 1, 1);
    return s;
}

MPK_API mpk_status mpk_jacobi_work_bytes(mpk_plan_t p, int32_t k, int32_t pw, uint32_t flags, size_t* bytes) {
    if (!p || !bytes) return fail(MPK_ERR_ARG, "null argument");
    if (k < 1 || k > 64) return fail(MPK_ERR_ARG, "k must be in 1..64 (got %d)", k);
    if (pw < 1) return fail(MPK_ERR_ARG, "p must be >= 1 (got %d)", pw);
    return k == 1 ? mpk_work_bytes(p, MPK_CALL_APPLY, pw, flags, bytes)
                  : mpk_work_bytes(p, MPK_CALL_POLY, k, flags, bytes);
}

MPK_API mpk_status mpk_jacobi_apply(mpk_plan_t p, int32_t k, const double* x, double* Y, int64_t ldy, int32_t pw,
                                    uint32_t flags, void* work, size_t work_bytes, void* stream) {
    if (!p) return fail(MPK_ERR_ARG, "null plan");
    if (p->column_scaling != MPK_SCALE_JACOBI)
        return fail(MPK_ERR_ARG, "the plan must hold A D^{-1} (column_scaling = MPK_SCALE_JACOBI)");
    if (k < 1 || k > 64) return fail(MPK_ERR_ARG, "k must be in 1..64 (got %d)", k);
    if (pw < 1) return fail(MPK_ERR_ARG, "p must be >= 1 (got %d)", pw);
    if (ldy < p->H.n) return fail(MPK_ERR_ARG, "ldy must be >= n");
    if (p->H.n > 0 && (!x || !Y)) return fail(MPK_ERR_ARG, "x or Y is null");
    if (k == 1) return mpk_apply(p, x, Y, ldy, pw, flags, work, work_bytes, stream);
    if (flags & ~(MPK_IO_PERMUTED | MPK_PLAIN | MPK_STAGED)) return fail(MPK_ERR_ARG, "unknown flag bits");
    size_t need = 0;
    mpk_jacobi_work_bytes(p, k, pw, flags, &need);
    if (need > 0 && (!work || work_bytes < need))
        return fail(MPK_ERR_ARG, "work buffer too small: %zu < %zu bytes", work_bytes, need);
    // A P^{-1} = I - (I - B)^k = I - (-1)^k (B - I)^k.  In level order the p k
    // sub-powers run as one chain (KIND_JCHAIN), blocked across the links.
    const double cjk = (k % 2) ? 1.0 : -1.0;  // -(-1)^k
    if (flags & MPK_IO_PERMUTED) {
        mpk_status s = check_uploaded(p);
        if (s != MPK_OK) return s;
        return mpk::jacobi_chain(p, k, x, Y, ldy, pw, nullptr, nullptr, flags, work, work_bytes, stream);
    }
    // original row order: one Newton polynomial per power (all shifts 1, c_0 = 1,
    // c_k = -(-1)^k) through poly_apply, which permutes; the same arithmetic
    std::vector<double> c(k + 1, 0.0), lam(k, 1.0);
    c[0] = 1.0;
    c[k] = cjk;
    for (int32_t j = 0; j < pw; ++j) {
        const double* in = j == 0 ? x : Y + (int64_t)(j - 1) * ldy;
        mpk_status s = poly_apply(p, MPK_POLY_NEWTON, k, c.data(), lam.data(), in, Y + (int64_t)j * ldy, flags,
                                  work, work_bytes, stream);
        if (s != MPK_OK) return s;
    }
    return MPK_OK;
}

MPK_API mpk_status mpk_gs2_work_bytes(mpk_plan_t p, int32_t gamma, int32_t pw, uint32_t flags, size_t* bytes) {
    if (!p || !bytes) return fail(MPK_ERR_ARG, "null argument");
    if (gamma < 0 || gamma > 16) return fail(MPK_ERR_ARG, "gamma must be in 0..16 (got %d)", gamma);
    if (pw < 1) return fail(MPK_ERR_ARG, "p must be >= 1 (got %d)", pw);
    const size_t v = (size_t)(p->H.n + 31) / 32 * 32 * 8;  // one vector, 256-byte multiple
    // ring: every sub-power a launch writes, plus the g_0 and input it reads
    const size_t ring = (size_t)(p->H.p_block + gamma + 2);
    *bytes = v * (ring + ((flags & MPK_IO_PERMUTED) ? 0 : 1 + (size_t)pw));
    return MPK_OK;
}

MPK_API mpk_status mpk_gs2_apply(mpk_plan_t p, int32_t gamma, const double* x, double* Y, int64_t ldy, int32_t pw,
                                 uint32_t flags, void* work, size_t work_bytes, void* stream) {
    if (!p) return fail(MPK_ERR_ARG, "null plan");
    if (!p->H.split_lower) return fail(MPK_ERR_ARG, "the plan must be built with split_lower = 1");
    if (gamma < 0 || gamma > 16) return fail(MPK_ERR_ARG, "gamma must be in 0..16 (got %d)", gamma);
    if (pw < 1) return fail(MPK_ERR_ARG, "p must be >= 1 (got %d)", pw);
    if (ldy < p->H.n) return fail(MPK_ERR_ARG, "ldy must be >= n");
    if (p->H.n > 0 && (!x || !Y)) return fail(MPK_ERR_ARG, "x or Y is null");
    if (flags & ~(MPK_IO_PERMUTED | MPK_PLAIN | MPK_STAGED)) return fail(MPK_ERR_ARG, "unknown flag bits");
    size_t need = 0;
    mpk_gs2_work_bytes(p, gamma, pw, flags, &need);
    if (!work || work_bytes < need) return fail(MPK_ERR_ARG, "work buffer too small: %zu < %zu bytes", work_bytes, need);
    if (((uintptr_t)work) & 255) return fail(MPK_ERR_ARG, "work must be 256-byte aligned");
    mpk_status s = check_uploaded(p);
    if (s != MPK_OK) return s;
    const int32_t n = p->H.n;
    if (n == 0) return MPK_OK;
    hipStream_t st = (hipStream_t)stream;
    const bool permuted = flags & MPK_IO_PERMUTED;
    const int64_t ld = (n + 31) / 32 * 32;
    double* w = (double*)work;
    const int ring = p->H.p_block + gamma + 2;
    const double* xin = x;
    double* yout = Y;
    int64_t yld = ldy;
    if (!permuted) {  // level-order copies after the ring
        double* xp = w + (int64_t)ring * ld;
        s = permute_vecs(p, st, x, 0, xp, 0, 1, 0);
        if (s != MPK_OK) return s;
        xin = xp;
        yout = xp + ld;
        yld = ld;
    }
    s = mpk::gs2_chain(p, gamma, xin, yout, yld, pw, nullptr, nullptr, 0, flags, w, work_bytes, stream);
    if (s != MPK_OK) return s;
    if (!permuted) s = permute_vecs(p, st, yout, ld, Y, ldy, pw, 1);
    return s;
}

MPK_API mpk_status mpk_gs2_smooth_work_bytes(mpk_plan_t p, int32_t gamma, uint32_t flags, size_t* bytes) {
    if (!p || !bytes) return fail(MPK_ERR_ARG, "null argument");
    if (gamma < 0 || gamma > 16) return fail(MPK_ERR_ARG, "gamma must be in 0..16 (got %d)", gamma);
    const size_t v = (size_t)(p->H.n + 31) / 32 * 32 * 8;  // one vector, 256-byte multiple
    // the ring of the GS2 chain, the chain's own copy of x^0, and in original row
    // order the level-order z, b and r
    const size_t ring = (size_t)(p->H.p_block + gamma + 2);
    *bytes = v * (ring + 1 + ((flags & MPK_IO_PERMUTED) ? 0 : 3));
    return MPK_OK;
}

MPK_API mpk_status mpk_gs2_smooth(mpk_plan_t p, int32_t gamma, int32_t sweeps, const double* b, double* x, double* r,
                                  uint32_t flags, void* work, size_t work_bytes, void* stream) {
    if (!p) return fail(MPK_ERR_ARG, "null plan");
    if (!p->H.split_lower) return fail(MPK_ERR_ARG, "the plan must be built with split_lower = 1");
    if (gamma < 0 || gamma > 16) return fail(MPK_ERR_ARG, "gamma must be in 0..16 (got %d)", gamma);
    if (sweeps < 0 || sweeps > (1 << 16)) return fail(MPK_ERR_ARG, "sweeps must be in 0..65536 (got %d)", sweeps);
    if (p->H.n > 0 && (!b || !x || !r)) return fail(MPK_ERR_ARG, "b, x or r is null");
    if (flags & ~(MPK_IO_PERMUTED | MPK_PLAIN | MPK_STAGED)) return fail(MPK_ERR_ARG, "unknown flag bits");
    size_t need = 0;
    mpk_gs2_smooth_work_bytes(p, gamma, flags, &need);
    if (!work || work_bytes < need) return fail(MPK_ERR_ARG, "work buffer too small: %zu < %zu bytes", work_bytes, need);
    if (((uintptr_t)work) & 255) return fail(MPK_ERR_ARG, "work must be 256-byte aligned");
    mpk_status s = check_uploaded(p);
    if (s != MPK_OK) return s;
    const int32_t n = p->H.n;
    if (n == 0) return MPK_OK;
    hipStream_t st = (hipStream_t)stream;
    const bool permuted = flags & MPK_IO_PERMUTED;
    const int64_t ld = (n + 31) / 32 * 32;
    double* w = (double*)work;
    const int ring = p->H.p_block + gamma + 2;
    // The chain reads x^0 from its own copy: with gamma = 0 a row closes its first
    // sweep (writing z) while a neighbour may still be gathering x^0.
    double* x0 = w + (int64_t)ring * ld;
    const double* bb = b;
    double* z = x;
    double* rr = r;
    if (!permuted) {
        double* zp = x0 + ld;
        double* bp = zp + ld;
        double* rp = bp + ld;
        s = permute_vecs(p, st, x, 0, x0, 0, 1, 0);
        if (s == MPK_OK) s = permute_vecs(p, st, b, 0, bp, 0, 1, 0);
        if (s != MPK_OK) return s;
        HIP_TRY(hipMemcpyAsync(zp, x0, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
        bb = bp;
        z = zp;
        rr = rp;
    } else {
        HIP_TRY(hipMemcpyAsync(x0, x, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    }
    PowerJob j;
    j.kind = KIND_SMOOTH;
    j.p = sweeps * (gamma + 1) + 1;
    j.x = x0;
    j.out0 = w;
    j.ld = ld;
    j.mod = ring;
    j.jk = gamma + 1;
    j.rhs = bb;
    j.z_io = z;
    j.res_out = rr;
    s = run_powers(p, st, j, flags & MPK_PLAIN, flags & MPK_STAGED);
    if (s != MPK_OK) return s;
    if (!permuted) {
        s = permute_vecs(p, st, z, ld, x, n, 1, 1);
        if (s == MPK_OK) s = permute_vecs(p, st, rr, ld, r, n, 1, 1);
    }
    return s;
}

mpk_status mpk::jacobi_chain(mpk_plan_t p, int k, const double* x, double* Y, int64_t ldy, int pw, const double* lam,
                             const double* sig, uint32_t flags, void* work, size_t work_bytes, void* stream) {
    const int32_t n = p->H.n;
    if (work_bytes < (size_t)poly_ring(p) * n * 8) return fail(MPK_ERR_ARG, "work buffer too small for the ring");
    if (n == 0) return MPK_OK;
    PowerJob j;
    j.kind = KIND_JCHAIN;
    j.p = pw * k;
    j.x = x;
    j.out0 = (double*)work;  // ring of sub-powers
    j.ld = n;
    j.mod = poly_ring(p);
    j.jk = k;
    j.jc = (k % 2) ? 1.0 : -1.0;  // -(-1)^k
    j.link_out = Y;
    j.link_ld = ldy;
    if (lam || sig) {  // Newton shifts where each link closes
        j.lam.assign((size_t)j.p, 0.0);
        j.sig.assign((size_t)j.p, 1.0);
        for (int q = 0; q < pw; ++q) {
            j.lam[(size_t)(q + 1) * k - 1] = lam ? lam[q] : 0.0;
            j.sig[(size_t)(q + 1) * k - 1] = sig ? sig[q] : 1.0;
        }
    }
    return run_powers(p, (hipStream_t)stream, j, flags & MPK_PLAIN, flags & MPK_STAGED);
}

mpk_status mpk::gs2_chain(mpk_plan_t p, int gamma, const double* x, double* Y, int64_t ldy, int pw,
                          const double* lam, const double* sig, int pinv, uint32_t flags, void* work,
                          size_t work_bytes, void* stream) {
    // x and Y in level order; work holds the ring of p_block + gamma + 2 vectors
    const int32_t n = p->H.n;
    const int64_t ld = (n + 31) / 32 * 32;
    const int ring = p->H.p_block + gamma + 2;
    if (work_bytes < (size_t)ring * ld * 8) return fail(MPK_ERR_ARG, "work buffer too small for the GS2 ring");
    if (n == 0) return MPK_OK;
    const int gl = gamma + (pinv ? 1 : 2);
    PowerJob j;
    j.kind = KIND_GS2;
    j.p = pw * gl;
    j.x = x;
    j.out0 = (double*)work;
    j.ld = ld;
    j.mod = ring;
    j.jk = gl;
    j.pinv = pinv;
    j.link_out = Y;
    j.link_ld = ldy;
    if (lam || sig) {  // Newton shifts on the closing sub-power of each power
        j.lam.assign((size_t)j.p, 0.0);
        j.sig.assign((size_t)j.p, 1.0);
        for (int q = 0; q < pw; ++q) {
            j.lam[(size_t)(q + 1) * gl - 1] = lam ? lam[q] : 0.0;
            j.sig[(size_t)(q + 1) * gl - 1] = sig ? sig[q] : 1.0;
        }
    }
    return run_powers(p, (hipStream_t)stream, j, flags & MPK_PLAIN, flags & MPK_STAGED);
}

MPK_API mpk_status mpk_set_watchdog(mpk_plan_t p, int32_t polls) {
    if (!p) return fail(MPK_ERR_ARG, "null plan");
    p->H.watchdog = polls;
    return MPK_OK;
}

MPK_API mpk_status mpk_set_block(mpk_plan_t p, int32_t q) {
    if (!p) return fail(MPK_ERR_ARG, "null plan");
    if (q < 0 || q > mpk::kMaxBlock) return fail(MPK_ERR_ARG, "q must be in 0..%d", mpk::kMaxBlock);
    p->q_cap = q;
    return MPK_OK;
}

MPK_API mpk_status mpk_tune_block(mpk_plan_t p, int32_t pw, const double* x, double* Y, int64_t ldy, void* stream,
                                  int32_t* q_out, double* seconds_out) {
    if (!p || !q_out) return fail(MPK_ERR_ARG, "null argument");
    if (pw < 1) return fail(MPK_ERR_ARG, "p must be >= 1 (got %d)", pw);
    if (ldy < p->H.n) return fail(MPK_ERR_ARG, "ldy must be >= n");
    if (p->H.n > 0 && (!x || !Y)) return fail(MPK_ERR_ARG, "x or Y is null");
    mpk_status s = check_uploaded(p);
    if (s != MPK_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    const int qmax = std::min<int>(pw, p->q_eff[KIND_MONO][0]);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        hipEventDestroy(e0);
        return fail(MPK_ERR_HIP, "event: %s", hipGetErrorString(he));
    }
    int best = 1;
    double best_t = 0.0;
    const int saved = p->q_cap;
    for (int q = 1; q <= std::max(qmax, 1) && s == MPK_OK; ++q) {
        p->q_cap = q;
        s = mpk_apply(p, x, Y, ldy, pw, MPK_IO_PERMUTED, nullptr, 0, st);  // warm-up
        if (s == MPK_OK && (he = hipEventRecord(e0, st)) != hipSuccess) s = MPK_ERR_HIP;
        for (int r = 0; r < 3 && s == MPK_OK; ++r) s = mpk_apply(p, x, Y, ldy, pw, MPK_IO_PERMUTED, nullptr, 0, st);
        if (s == MPK_OK && (he = hipEventRecord(e1, st)) != hipSuccess) s = MPK_ERR_HIP;
        if (s == MPK_OK && (he = hipEventSynchronize(e1)) != hipSuccess) s = MPK_ERR_HIP;
        float ms = 0.0f;
        if (s == MPK_OK && (he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) s = MPK_ERR_HIP;
        if (s == MPK_OK && (q == 1 || ms / 3.0 * 1e-3 < best_t)) {
            best = q;
            best_t = ms / 3.0 * 1e-3;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (s == MPK_ERR_HIP && he != hipSuccess) fail(MPK_ERR_HIP, "timing: %s", hipGetErrorString(he));
    if (s == MPK_OK) s = mpk_check_device(p, stream);
    p->q_cap = s == MPK_OK ? best : saved;
    if (s != MPK_OK) return s;
    *q_out = best;
    if (seconds_out) *seconds_out = best_t;
    return MPK_OK;
}

MPK_API mpk_status mpk_permute(mpk_plan_t p, const double* in, double* out, int32_t direction, void* stream) {
    mpk_status s = check_uploaded(p);
    if (s != MPK_OK) return s;
    if (direction != 0 && direction != 1) return fail(MPK_ERR_ARG, "direction must be 0 or 1");
    if (p->H.n > 0 && (!in || !out)) return fail(MPK_ERR_ARG, "null vector");
    if (in == out && p->H.n > 0) return fail(MPK_ERR_ARG, "in and out must not alias");
    return permute_vecs(p, (hipStream_t)stream, in, 0, out, 0, 1, direction);
}

MPK_API mpk_status mpk_check_device(mpk_plan_t p, void* stream) {
    mpk_status s = check_uploaded(p);
    if (s != MPK_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipStreamSynchronize(st));
    int32_t* slot = status_slot(p, stream, false);
    if (!slot) return MPK_OK;  // no blocked launch on this stream
    int32_t h[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(h, slot, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (h[0] == 0) return MPK_OK;
    fill_u32_kernel<<<1, 64, 0, st>>>((uint32_t*)slot, 4, 0u);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    return fail(MPK_ERR_DEVICE,
                "blocked kernel watchdog: chunk %d waited too long before power %d "
                "(not every worker was resident, or a dependency never completed)",
                h[1], h[2]);
}

MPK_API void mpk_destroy(mpk_plan_t p) { delete p; }
