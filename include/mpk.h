/*
 * mpk.h -- C ABI of the MI355X matrix power kernel library (libmpk.so).
 *
 * The library computes the matrix power kernel (MPK) of Sec. 3 of
 * "Algebraic temporal blocking for sparse iterative solvers on multi-core
 * CPUs" (Alappat, Thies, Hager, Fehske, Wellein): for a square sparse A and a
 * vector x, y_k = A y_{k-1} for k = 1..p with y_0 = x (Alg. 1), every power
 * stored.  Powers are temporally blocked by the BFS level structure of the
 * matrix graph (Sec. 3): a persistent kernel keeps each 64-row chunk of the
 * matrix in registers while it advances that chunk through a block of q
 * powers, waiting only for the neighbouring chunks of the previous power.
 * The polynomial forms built on the MPK are also provided: a fixed-coefficient
 * polynomial p(A) x (Sec. 5.2, Eq. (3); Chebyshev as in Sec. 5.3) and the
 * Newton basis of the s-step Krylov method (Sec. 4).
 *
 * Conventions (every entry point):
 *   - Return an mpk_status; nothing aborts the process and no C++ exception
 *     crosses the ABI.  mpk_last_error() returns a thread-local message for
 *     the last failing call of the calling thread.
 *   - Argument and CSR validation is synchronous.  Device work is enqueued
 *     asynchronously on `stream` (a hipStream_t passed as void*; NULL is the
 *     legacy default stream).  Device-side failures (the watchdog of the
 *     blocked kernel) are reported by mpk_check_device().
 *   - Vector pointers marked "device" must point to device memory of the
 *     current device and hold FP64 values; they must not alias each other
 *     unless stated.  The caller owns every buffer it passes; the library
 *     owns only the plan object (host memory), released by mpk_destroy().
 *   - Calls on one plan may overlap on several streams and host threads:
 *     blocked (persistent) launches on one device are chained one after the
 *     other by the library, whatever stream or plan issues them, and all
 *     other launches use only caller buffers.  A device error raised by a
 *     call is reported by mpk_check_device for the stream that call ran on
 *     (each stream has its own status on each plan, see mpk_check_device).
 *   - Indices are 0-based int32; n and nnz must be below 2^31.
 */
#ifndef MPK_H
#define MPK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mpk_plan_s* mpk_plan_t;     /* opaque; owned by the library */
typedef struct mpk_server_s* mpk_server_t; /* opaque; owned by the library */
typedef struct mpk_plan_cache_s* mpk_plan_cache_t; /* opaque; owned by the library */

typedef enum {
    MPK_OK = 0,
    MPK_ERR_ARG = -1,         /* bad scalar argument or null pointer          */
    MPK_ERR_CSR = -2,         /* malformed CSR input                          */
    MPK_ERR_NOMEM = -3,       /* host allocation failed, or buffer too small  */
    MPK_ERR_HIP = -4,         /* a HIP runtime call failed                    */
    MPK_ERR_UNSUPPORTED = -5, /* valid request the library does not provide   */
    MPK_ERR_STATE = -6,       /* call order violated (e.g. apply before upload) */
    MPK_ERR_DEVICE = -7       /* device-side failure reported by the kernel   */
} mpk_status;

/* flags for mpk_apply / poly_apply / sstep_basis / mpk_refine_solve */
#define MPK_IO_PERMUTED 1u /* x and outputs are in the plan's level order (perm space) */
#define MPK_PLAIN 2u       /* comparator: one full SpMV launch per power (Alg. 1),
                              same layout and same per-row arithmetic            */
#define MPK_STAGED 4u      /* the level-group wavefront of Sec. 3 (see
                              mpk_get_schedule): one launch per stage, same
                              per-row arithmetic; ignored with MPK_PLAIN       */
#define MPK_RITZ_SHIFTS 16u /* mpk_sstep_gmres_ex only: Newton shifts from Ritz values
                               (see there) instead of a spectrum interval */
#define MPK_LAST_POWER 8u  /* mpk_server_submit_apply only: Y receives y_p alone
                              (n doubles) instead of all p powers                */

/* polynomial kinds for poly_apply */
#define MPK_POLY_MONOMIAL 0  /* phi_k = A^k                                     */
#define MPK_POLY_NEWTON 1    /* phi_k = prod_{i<=k} (A - lambda_i I)            */
#define MPK_POLY_CHEBYSHEV 2 /* phi_k = T_k((A - theta I) / delta)             */

/* value storage for mpk_options.value_type */
#define MPK_VALUES_F64 0
#define MPK_VALUES_F32 1
#define MPK_VALUES_BF16_ROWSCALE 2 /* a_ij ~ s_i q_ij: s_i = fl32(max_j |a_ij|) per row,
                                     q_ij = BF16 nearest (ties to even) to
                                     fl32(a_ij / s_i); s_i q_ij is formed exactly
                                     in FP64 at every use                      */

/* mpk_options.column_scaling */
#define MPK_SCALE_NONE 0
#define MPK_SCALE_JACOBI 1

/* call kinds for mpk_work_bytes */
#define MPK_CALL_APPLY 0
#define MPK_CALL_POLY 1
#define MPK_CALL_SSTEP 2
#define MPK_CALL_SOLVE 3

typedef struct {
    int32_t root_mode;       /* 0: per connected component, the George-Liu
                                pseudo-peripheral node reached from the
                                component's lowest-index row; 1: `root` is the
                                BFS root of its component (others as in 0)    */
    int32_t root;            /* used when root_mode == 1; 0 <= root < n       */
    int32_t p_block;         /* powers per blocked launch, q (p_opt of Sec. 3);
                                1..15; 0 selects 4                           */
    int32_t workers_per_xcd; /* waves per XCD of the blocked kernel; 0 = as
                                many as stay resident together               */
    int32_t watchdog_polls;  /* polls before a dependency wait of the blocked
                                kernel gives up and reports MPK_ERR_DEVICE;
                                0 = default (2^20, about a second); a
                                negative value makes every wait give up at
                                once (forces the failure path in tests)      */
    int32_t chunks_per_worker; /* chunks a wave of the blocked kernel carries
                                together through a block (1, 2 or 4; 0 = 2;
                                always 1 when rows need more than 16 register
                                slots).  With FP32 values, 4 suits mpk_apply
                                on rows of at most 8 slots.  With 0 on rows
                                of at most 8 slots the kernels may carry 3,
                                5 or 6 (mpk_block_shape)                      */
    int32_t value_type;      /* storage of the matrix values on the device:
                                MPK_VALUES_F64 (0), MPK_VALUES_F32 (1) or
                                MPK_VALUES_BF16_ROWSCALE (2).  The reduced
                                forms round each value once at upload; vectors,
                                products and sums stay FP64, so every call
                                returns the FP64 MPK of the rounded matrix (the
                                paper works in FP64 only; FP32 halves the value
                                bytes, BF16 quarters them and adds 4 bytes of
                                scale per row)                                */
    int32_t max_reg_slots;   /* largest number of SELL slots per row the
                                blocked kernel keeps in registers (4, 7, 8,
                                16 or 32; 0 = automatic: the smallest of these
                                covering the widest chunk, 32 at most).  Slots
                                beyond it are re-read from memory at every
                                power.                                        */
    int32_t cache_mib;       /* C of the level groups used by mpk_get_schedule
                                and MPK_STAGED, in MiB (0 = 256, the MI355X
                                Infinity Cache, the closest analogue of the
                                last-level cache the paper blocks for)        */
    int32_t min_group_rows;  /* row floor below which a level group is never
                                closed (>= 0)                                 */
    int32_t column_scaling;  /* MPK_SCALE_NONE (0): the plan holds A;
                                MPK_SCALE_JACOBI (1): it holds B = A D^{-1},
                                each value divided by its column's diagonal
                                entry in FP64 before any rounding of
                                value_type (the fused diagonally preconditioned
                                operator of Sec. 5.1; every call then applies
                                to B).  Needs a stored nonzero diagonal entry
                                in every row (else MPK_ERR_CSR)               */
    int32_t split_lower;     /* 1: also record, per row, which stored entries
                                lie in the strictly lower triangle L (original
                                numbering) and which is the diagonal, for the
                                GS2-preconditioned MPK (mpk_gs2_apply).  Needs
                                a stored nonzero diagonal entry in every row
                                (else MPK_ERR_CSR) and at most 32 entries per
                                row (else MPK_ERR_UNSUPPORTED)                */
    int32_t reserved[4];     /* must be zero                                  */
} mpk_options;

/* Fills *opt with the defaults (all zero). */
void mpk_options_default(mpk_options* opt);

/* Library version string (static storage). */
const char* mpk_version(void);

/* Message for the last failing call on this thread (static thread-local
 * storage, valid until the next failing call on the thread). */
const char* mpk_last_error(void);

/*
 * Host-side planning (Sec. 3: BFS levels of the matrix graph and an execution
 * order derived from them).  Input is a host CSR matrix: rowptr[n+1] monotone
 * with rowptr[0] == 0, col[rowptr[n]] with columns strictly ascending in each
 * row and in [0, n), val[rowptr[n]] FP64.  Empty rows and explicit zeros are
 * allowed; n == 0 is allowed.  The library copies what it needs: the caller
 * keeps ownership of the arrays, which may be freed on return.
 *
 * Steps: (1) the undirected graph of pattern(A) union pattern(A^T) without
 * self-loops; (2) BFS levels per component from the root chosen by
 * opt->root_mode, components in order of their lowest row index, levels of a
 * later component numbered after those of earlier ones; (3) perm sorts rows
 * by (level, original index); (4) the permuted matrix P A P^T in SELL-64
 * layout (chunks of 64 consecutive permuted rows, column-major inside a
 * chunk); (5) chunk ownership by XCD from each chunk's position inside its
 * level, per-XCD chunk sequences, and per-chunk dependency lists.
 *
 * On success *plan_out owns a new plan and *device_bytes_out (if not NULL)
 * receives the size of the device buffer mpk_upload needs.
 * Errors: MPK_ERR_ARG (null pointers, n < 0, bad options), MPK_ERR_CSR
 * (non-monotone rowptr, column out of range, unsorted or duplicate columns),
 * MPK_ERR_NOMEM.
 */
mpk_status mpk_build_levels(int32_t n, const int32_t* rowptr, const int32_t* col,
                            const double* val, const mpk_options* opt,
                            mpk_plan_t* plan_out, size_t* device_bytes_out);

/*
 * Level structure of a plan (host arrays supplied by the caller; any pointer
 * may be NULL to skip it).  nlevels receives L; level_ptr[L+1] the first
 * permuted row of each level; level_of_row[n] the level of each original row;
 * perm[n] with perm[new] = old; iperm[n] with iperm[old] = new.
 */
mpk_status mpk_get_levels(mpk_plan_t plan, int32_t* nlevels, int32_t* level_ptr,
                          int32_t* level_of_row, int32_t* perm, int32_t* iperm);

/*
 * Chunk partition of a plan: *nchunks chunks of *chunk_rows (= 64) permuted
 * rows (the last may be shorter); owner[nchunks] (may be NULL) receives the
 * XCD partition (0..*nparts-1) that computes each chunk.
 */
mpk_status mpk_get_partition(mpk_plan_t plan, int32_t* nchunks, int32_t* chunk_rows,
                             int32_t* nparts, int32_t* owner);

/*
 * Chunk dependency lists: chunk c waits, before computing power k >= 2 of a
 * block, until every chunk in dep_idx[dep_ptr[c] .. dep_ptr[c+1]-1] has
 * finished power k-1.  The lists are the chunks holding a row adjacent to a
 * row of c in the symmetrised pattern, c itself excluded, ascending.  Call
 * once with dep_ptr = dep_idx = NULL to get *ndeps, then with arrays of
 * nchunks+1 and *ndeps entries.
 */
mpk_status mpk_get_deps(mpk_plan_t plan, int64_t* ndeps, int32_t* dep_ptr, int32_t* dep_idx);

/*
 * Smallest number of resident workers (waves) per XCD partition for which the
 * blocked kernel cannot deadlock with blocks of q powers.  Units of
 * chunks_per_worker consecutive chunks of a partition's sequence are handed
 * out in sequence order; the bound W is the smallest value such that, for
 * every partition and unit position j >= W, the first chunk of unit j - W has
 * a smaller index than the first chunk of every unit within q-1 dependency
 * hops of unit j.  mpk_upload picks, per operator kind, the largest q <= p_block
 * whose bound fits the waves it launches (mpk_block_powers).  1 <= q <= p_block.
 */
mpk_status mpk_min_workers(mpk_plan_t plan, int32_t q, int32_t* workers_per_xcd);

/*
 * mpk_min_workers for units of chunks_per_worker chunks.  A plan holds the
 * units of its own chunks_per_worker and, when its chunks_per_worker was left
 * at 0 and its rows fit 8 register slots, units of 3, 5 and 6 as well.  For
 * each operator kind mpk_upload takes the largest of these whose kernel keeps
 * two waves per SIMD resident and admits as many powers per launch (at 7
 * slots: 6 for MPK_OP_POWERS with FP64 or FP32 values, 5 for the other kinds,
 * 3 for MPK_OP_GS2_CHAIN, 2 for MPK_OP_GS2_SMOOTH; see mpk_block_shape).
 * Errors: MPK_ERR_ARG (null pointers, q outside 1..p_block, no units of that
 * size in the plan).
 */
mpk_status mpk_min_workers_units(mpk_plan_t plan, int32_t chunks_per_worker, int32_t q, int32_t* workers_per_xcd);

/* Operator kinds of mpk_block_powers. */
#define MPK_OP_POWERS 0           /* mpk_apply (and mpk_jacobi_apply with k = 1)  */
#define MPK_OP_POLY_MONOMIAL 1    /* poly_apply, MPK_POLY_MONOMIAL                */
#define MPK_OP_POLY_NEWTON 2      /* poly_apply, MPK_POLY_NEWTON                  */
#define MPK_OP_POLY_CHEBYSHEV 3   /* poly_apply, MPK_POLY_CHEBYSHEV (and the      */
                                  /* Chebyshev preconditioner of the solvers)     */
#define MPK_OP_NEWTON_BASIS 4     /* sstep_basis                                  */
#define MPK_OP_JACOBI_CHAIN 5     /* mpk_jacobi_apply with k > 1                  */
#define MPK_OP_GS2_CHAIN 6        /* mpk_gs2_apply                                */
#define MPK_OP_GS2_SMOOTH 7       /* mpk_gs2_smooth                               */

/*
 * Powers (or sub-powers of a chain) per blocked launch that calls of operator
 * kind `op` use on this uploaded plan: p_block lowered to the deadlock bound of
 * the resident waves (Sec. 3 temporal blocking needs the matrix rows of a
 * block of levels to stay on chip while q powers advance) and to the cap of
 * mpk_set_block.  1 means those calls run one plain SpMV launch per power (no
 * blocking engages).  A call also never uses more than the powers it asks for.
 * Errors: MPK_ERR_ARG (null pointers, unknown op), MPK_ERR_STATE (not
 * uploaded).
 */
mpk_status mpk_block_powers(mpk_plan_t plan, int32_t op, int32_t* q);

/*
 * Launch shape of the blocked kernel that calls of operator kind op use on
 * this uploaded plan: its waves per XCD partition, the chunks each wave
 * carries (the units of mpk_min_workers_units) and the SELL slots per row it
 * keeps in registers.  Any output pointer may be null.
 * Errors: MPK_ERR_ARG (unknown op), MPK_ERR_STATE (not uploaded).
 */
mpk_status mpk_block_shape(mpk_plan_t plan, int32_t op, int32_t* workers_per_xcd, int32_t* chunks_per_worker,
                           int32_t* reg_slots);

/*
 * Binds caller-owned device memory (at least device_bytes from
 * mpk_build_levels; 256-byte aligned) and uploads the permuted matrix, the
 * permutation, the schedule tables and zeroed synchronisation counters on
 * `stream`.  The buffer must stay allocated, and must not be written by the
 * caller, for as long as the plan is used.  Re-uploading into another buffer
 * is allowed once earlier work on the plan has finished.
 */
mpk_status mpk_upload(mpk_plan_t plan, void* dev_buf, size_t bytes, void* stream);

/*
 * New values for the matrix of a plan, with the sparsity pattern the plan was
 * built from (n, rowptr, col identical; checked through a 128-bit hash of the
 * pattern): the BFS levels, permutation, layout and schedule are kept (the
 * preprocessing of Sec. 3 is amortised over calls on one pattern, Sec. 6) and
 * only the values are refilled (column scaling and value storage type as at
 * build) and, if the plan is uploaded, copied to its device buffer on
 * `stream`, which is then synchronised.  Must not overlap other calls on the
 * plan; earlier device work on the plan must have finished.
 * Errors: MPK_ERR_ARG (null pointers, n or pattern differs), MPK_ERR_CSR,
 * MPK_ERR_NOMEM, MPK_ERR_HIP.
 */
mpk_status mpk_update_values(mpk_plan_t plan, int32_t n, const int32_t* rowptr, const int32_t* col,
                             const double* val, void* stream);

/*
 * ---- Plan cache ---------------------------------------------------------
 * Plans keyed by the sparsity pattern of their matrix (a 128-bit hash of n,
 * rowptr and col) and by the options that shape them, on the device current
 * at mpk_plan_cache_create, within `device_bytes` of plan buffers (the cache
 * allocates one buffer per plan when a pattern is first planned).
 * mpk_plan_cache_get returns the cached, uploaded plan of the pattern
 * (*outcome 0: same values; 1: new values, refilled as by mpk_update_values,
 * allowed only while no other user holds the plan), or plans and uploads a new
 * pattern (*outcome 2), evicting least recently used plans that no user holds
 * when the budget requires.  Each get must be paired with
 * mpk_plan_cache_release once the caller's work on the plan has finished; the
 * plan belongs to the cache (never mpk_destroy it).  Thread-safe.
 * Errors: MPK_ERR_ARG, MPK_ERR_CSR, MPK_ERR_STATE (new values for a plan in
 * use), MPK_ERR_NOMEM (plan larger than the budget, or every plan in use),
 * MPK_ERR_HIP, and those of mpk_build_levels / mpk_upload.
 */
mpk_status mpk_plan_cache_create(size_t device_bytes, mpk_plan_cache_t* out);
mpk_status mpk_plan_cache_get(mpk_plan_cache_t cache, int32_t n, const int32_t* rowptr, const int32_t* col,
                              const double* val, const mpk_options* opt, void* stream, mpk_plan_t* plan,
                              int32_t* outcome);
mpk_status mpk_plan_cache_release(mpk_plan_cache_t cache, mpk_plan_t plan);
/* Plans held, device bytes used, and gets served by each outcome so far. */
mpk_status mpk_plan_cache_stats(mpk_plan_cache_t cache, int32_t* plans, size_t* bytes_used, int64_t* hits,
                                int64_t* value_updates, int64_t* misses);
void mpk_plan_cache_destroy(mpk_plan_cache_t cache);

/*
 * Device work-buffer size (bytes) that mpk_apply (call = MPK_CALL_APPLY),
 * poly_apply (MPK_CALL_POLY, p = degree d), sstep_basis (MPK_CALL_SSTEP,
 * p = s) or mpk_refine_solve (MPK_CALL_SOLVE, p = degree, asked of the `lo`
 * plan) needs with the given flags.  Zero when none is needed.
 */
mpk_status mpk_work_bytes(mpk_plan_t plan, int32_t call, int32_t p, uint32_t flags,
                          size_t* bytes);

/*
 * Matrix power kernel (Sec. 3, Alg. 1): Y[(k-1)*ldy + i] = (A^k x)[i] for
 * k = 1..p.  x (device, n) is only read; Y (device, p*ldy, ldy >= n) receives
 * p vectors; y_0 = x is not stored.  With MPK_IO_PERMUTED, x and Y are in perm
 * space (x_perm[i] = x[perm[i]]), which is the fast path; otherwise the library
 * permutes through `work` (mpk_work_bytes).  Powers run in blocks of
 * q = p_block (the last block holds the remaining p mod q, Sec. 3 remainder
 * loop); q is lowered until the deadlock bound of the plan (mpk_min_workers)
 * fits the resident waves, and when only q = 1 fits (BFS levels too wide for
 * the waves) the call runs one SpMV launch per power, as blocking could not
 * reuse the matrix; so does any block of a single power (p = 1, or a
 * one-power remainder).  MPK_PLAIN always runs p full SpMV launches (the
 * comparator).  Results of the blocked and plain paths are bitwise identical.
 * Errors: MPK_ERR_ARG (p < 1, ldy < n, null pointers, work too small),
 * MPK_ERR_STATE (not uploaded), MPK_ERR_HIP.
 */
mpk_status mpk_apply(mpk_plan_t plan, const double* x, double* Y, int64_t ldy, int32_t p,
                     uint32_t flags, void* work, size_t work_bytes, void* stream);

/*
 * Polynomial applied to a vector (Sec. 5.2, Eq. (3)):
 *   out = sum_{k=0..d} c[k] * phi_k(A) x
 * kind MPK_POLY_MONOMIAL: phi_k = A^k; MPK_POLY_NEWTON: phi_0 = I,
 * phi_k = (A - params[k-1] I) phi_{k-1} (params = lambda[d]);
 * MPK_POLY_CHEBYSHEV: the Chebyshev polynomials on [theta - delta,
 * theta + delta] with params = {theta, delta}: t_0 = x,
 * t_1 = (A - theta I) x / delta, t_{k+1} = 2 (A - theta I) t_k / delta - t_{k-1}.
 * c (host, d+1 entries) and params (host) are copied before return.
 * x and out are device vectors of n entries (perm space with
 * MPK_IO_PERMUTED); out must not alias x.  Intermediate vectors live in
 * `work`: a ring of p_block + 2 vectors (so that a launch never rewrites a
 * vector it reads and may gather with plain loads), plus two more without
 * MPK_IO_PERMUTED.
 * Errors: MPK_ERR_ARG (d < 0, unknown kind, delta == 0, null pointers, work
 * too small), MPK_ERR_STATE, MPK_ERR_HIP.
 */
mpk_status poly_apply(mpk_plan_t plan, int32_t kind, int32_t d, const double* c,
                      const double* params, const double* x, double* out, uint32_t flags,
                      void* work, size_t work_bytes, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): poly_apply
 * without a work argument.  The intermediate vectors live in a scratch array
 * the library holds on each GPU it runs on, MPK_STATIC_SCRATCH_BYTES (64 MiB)
 * per device, kept until the process ends; its address is looked up once per
 * device on the first call there.  The call itself allocates nothing.
 * The result equals poly_apply's with the same arguments.  It needs
 * mpk_work_bytes(plan, MPK_CALL_POLY, d, flags) bytes of that scratch, i.e.
 * 8 n (p_block + 2) bytes (plus 16 n without MPK_IO_PERMUTED); larger
 * requests fail with MPK_ERR_ARG.  Every call on one GPU shares that GPU's
 * scratch, and it keeps the last call's contents: calls that overlap on one
 * GPU (from several streams or host threads) race and must be serialised by
 * the caller.  Errors: as poly_apply, plus MPK_ERR_ARG when the scratch is too
 * small, MPK_ERR_HIP if the scratch address cannot be obtained.
 */
#define MPK_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
mpk_status poly_apply_static(mpk_plan_t plan, int32_t kind, int32_t d, const double* c,
                             const double* params, const double* x, double* out, uint32_t flags,
                             void* stream);

/*
 * Level groups and wavefront schedule of one block of q powers (Sec. 3: an
 * execution order from the level structure and the cache size):
 *   levels are grouped greedily and contiguously: a group is closed before
 *   level l when it is non-empty, has at least min_group_rows rows and
 *   w(group) + w(l) > floor(C / q), with w(level) = sum over its rows of
 *   nnz_row * (value bytes + 4) + 20;
 *   task (k, g), k = 1..q, computes power k on the levels of group g shifted
 *   down by k - 1 (from level 0 for g = 0, to the last level for the last
 *   group) and runs at stage g + k - 1; a stage's tasks are independent.
 * On return *ntasks holds the number of non-empty tasks and *ngroups the
 * number of groups; if `tasks` is not NULL it receives 4 ints per task,
 * {stage, k, row_begin, row_end} (permuted rows, end exclusive), in stage
 * order, then k.  q must be in 1..15.  Host only; no upload needed.
 * Errors: MPK_ERR_ARG (null plan or counts, q out of range).
 */
mpk_status mpk_get_schedule(mpk_plan_t plan, int32_t q, int32_t* ntasks, int32_t* ngroups, int32_t* tasks);

/*
 * Solve A x = b by FP64 iterative refinement around the degree-d Chebyshev
 * polynomial preconditioner (the polynomial preconditioner of Sec. 5; the
 * refinement goes beyond the paper, which works in FP64 throughout):
 *   r_i = b - A x_i, computed in FP64 with `hi` (FP64 values);
 *   stop when ||r_i||_2 <= tol ||b||_2 or i == max_iter;
 *   x_{i+1} = x_i + s(A) r_i, with s of degree d - 1 such that
 *   1 - lam s(lam) = T_d((theta - lam)/delta) / T_d(theta/delta),
 *   theta = (lmax + lmin)/2, delta = (lmax - lmin)/2 (the interpolant of
 *   1/lam at the d zeros of T_d on [lmin, lmax]), applied through the
 *   Chebyshev recurrence of poly_apply on `lo` (FP32 values for the mixed-
 *   precision solve, or FP64), blocked unless MPK_PLAIN.
 * The iteration contracts when [lmin, lmax] holds the spectrum of an SPD A
 * (for example lmin a known shift and lmax a Gershgorin bound).
 * hi and lo must be uploaded plans of the same matrix with the same level
 * order (checked).  b and x are device vectors of n entries (perm space
 * with MPK_IO_PERMUTED); x holds the initial guess on entry and the result
 * on return; b must not alias x.  work: mpk_work_bytes(lo, MPK_CALL_SOLVE,
 * d, flags) bytes.  iters_out (corrections applied) and relres_out (the
 * last ||r||/||b||, or ||r|| when b = 0) are host pointers and may be NULL.
 * The call synchronises `stream` once per step to read the residual norm;
 * norms are reduced in a fixed order, so repeated calls give identical
 * results.  Errors: MPK_ERR_ARG (hi not FP64, plans of different matrices,
 * d outside 1..4096, lmin/lmax not 0 < lmin < lmax, tol < 0, max_iter < 0,
 * null pointers, work too small), MPK_ERR_STATE, MPK_ERR_HIP, MPK_ERR_DEVICE.
 */
mpk_status mpk_refine_solve(mpk_plan_t hi, mpk_plan_t lo, int32_t degree, double lmin, double lmax,
                            const double* b, double* x, double tol, int32_t max_iter, uint32_t flags,
                            void* work, size_t work_bytes, int32_t* iters_out, double* relres_out,
                            void* stream);

/*
 * Solve A x = b by restarted s-step GMRES (Sec. 4: Alg. 3a around the subspace
 * routine of Alg. 3c) with the degree-d Chebyshev polynomial preconditioner
 * applied from the right (Sec. 5: A P^{-1} u = b, x = P^{-1} u):
 *   P^{-1} = s(A), s of degree d - 1 as in mpk_refine_solve, so the operator
 *   M = A s(A) = I - T_d((theta I - A)/delta) / T_d(theta/delta) costs d
 *   matrix powers per vector (one poly_apply launch on `lo`);
 *   each restart cycle starts from r = b - A x computed with `hi` (FP64
 *   values) and stops the solve when ||r||_2 <= tol ||b||_2 or after
 *   max_cycles cycles;
 *   a cycle builds at most m basis vectors in blocks of s: the Newton basis
 *   W_k = (M - lambda_k I) W_{k-1} / sigma_k from the block's first vector,
 *   with lambda_k the s Chebyshev points of [1 - eps, 1 + eps] (M's spectrum
 *   when A's lies in [lmin, lmax]; eps = 1 / T_d(theta/delta)) in Leja order
 *   and sigma_k = eps / 2; BOrtho, one block classical Gram-Schmidt sweep
 *   against the previous vectors; TSQR, a Cholesky QR of the block in FP64,
 *   which ends the cycle at a column whose Cholesky pivot is at most 2^-24
 *   of its length before BOrtho (the Krylov space is then invariant); the
 *   Hessenberg matrix follows from the change of basis and the small least-
 *   squares problem is solved on the host after every block, ending the
 *   cycle when its residual is at most tol ||b||;
 *   x += s(A) Q y at the end of a cycle.
 * The shifts need no Arnoldi run (the paper takes them from Ritz values);
 * they assume a symmetric positive definite A with spectrum in [lmin, lmax].
 * hi and lo: uploaded plans of the same matrix and level order (lo may be hi,
 * or a plan with FP32 values for a mixed-precision solve: then the basis and
 * the preconditioner use the rounded matrix and the residuals stay FP64).
 * s in 1..16, m in s..256, d in 1..4096.  b and x are device vectors of n
 * entries (perm space with MPK_IO_PERMUTED); x holds the initial guess on
 * entry and the result on return.  work: device, 256-byte aligned,
 * mpk_sstep_gmres_work_bytes(lo, s, m, d, flags) bytes.  iters_out (basis
 * vectors built over all cycles), cycles_out and relres_out (the last
 * ||r||/||b||, or ||r|| when b = 0) are host pointers and may be NULL.
 * MPK_PLAIN / MPK_STAGED select the executor of the polynomial launches.
 * The call synchronises `stream` twice per block and once per cycle; sums are
 * reduced in a fixed order, so repeated calls give identical results.
 * Errors: MPK_ERR_ARG (hi not FP64, plans of different matrices, s, m or d
 * out of range, not 0 < lmin < lmax, tol < 0, max_cycles < 0, null pointers,
 * work too small or misaligned), MPK_ERR_STATE, MPK_ERR_HIP, MPK_ERR_NOMEM.
 */
mpk_status mpk_sstep_gmres(mpk_plan_t hi, mpk_plan_t lo, int32_t s, int32_t m, int32_t degree, double lmin,
                           double lmax, const double* b, double* x, double tol, int32_t max_cycles,
                           uint32_t flags, void* work, size_t work_bytes, int32_t* iters_out,
                           int32_t* cycles_out, double* relres_out, void* stream);

/* preconditioners of mpk_sstep_gmres_ex */
#define MPK_PRECOND_CHEBYSHEV 0 /* P^{-1} = s(A) of degree d - 1 (as mpk_sstep_gmres)     */
#define MPK_PRECOND_NONE 1      /* M = A, x = x0 + Q y                                     */
#define MPK_PRECOND_JACOBI 2    /* k = degree Jacobi sweeps: M = A P^{-1} (k = 1: A D^{-1},
                                   fused), x = x0 + P^{-1} Q y (Sec. 5.1)                 */
#define MPK_PRECOND_GS2 3       /* M = A P^{-1}, P^{-1} one GS2 iteration from zero with
                                   gamma = degree inner sweeps, x = x0 + P^{-1} Q y        */

/*
 * mpk_sstep_gmres with a choice of right preconditioner (Sec. 4 and Sec. 5.1).
 * MPK_PRECOND_CHEBYSHEV is mpk_sstep_gmres.  With MPK_PRECOND_NONE and
 * MPK_PRECOND_JACOBI each block of s basis vectors is one blocked Newton MPK of
 * s powers (sstep_basis on `lo`: Alg. 3c's back-to-back SpMVs replaced by an
 * MPK); [lmin, lmax] must then hold the spectrum of M (A, or A D^{-1}, which
 * is similar to D^{-1/2} A D^{-1/2}) and gives the shifts: its s Chebyshev
 * points in Leja order, each column scaled by (lmax - lmin) / 4.  `lo` holds
 * A (MPK_PRECOND_NONE) or A D^{-1} (column_scaling = MPK_SCALE_JACOBI for
 * MPK_PRECOND_JACOBI), with FP64 or FP32 values; `hi` holds A in FP64 and gives
 * the residuals and, for Jacobi, the diagonal.  With MPK_PRECOND_GS2, `lo` is
 * built with split_lower, `degree` is gamma (0..16), each block's basis is one
 * GS2 chain of s powers (s (gamma + 2) sub-powers blocked together, the Newton
 * shift applied as each power closes; see mpk_gs2_apply), [lmin, lmax] holds
 * the spectrum of A P^{-1}, and x = x0 + P^{-1} Q y with P^{-1} as a chain of
 * gamma + 1 sub-powers.  With MPK_PRECOND_JACOBI, `degree` is the number k
 * of Jacobi sweeps (1..64): k = 1 builds each block with sstep_basis on
 * A D^{-1}; k > 1 with one Jacobi chain of s k sub-powers (mpk_jacobi_apply)
 * with the shifts applied as each link closes, and x = x0 + D^{-1}
 * sum_{i<k} (I - A D^{-1})^i Q y.  `degree` is unused by MPK_PRECOND_NONE
 * (pass 1); lmin may be <= 0 for all but Chebyshev.  With MPK_RITZ_SHIFTS in
 * flags (not for MPK_PRECOND_CHEBYSHEV) lmin and lmax are ignored and the shifts
 * come from Ritz values, as Sec. 4 takes them from a few steps of standard GMRES:
 * the first cycle runs s Arnoldi steps on M from r0 / ||r0|| (classical
 * Gram-Schmidt with one reorthogonalisation, stopping early on an invariant
 * space), the eigenvalues of the square Hessenberg matrix are the Ritz values,
 * and their real parts in Leja order (repeated cyclically when fewer than s were
 * found) are the shifts of the whole solve, each column scaled by a quarter of
 * their spread.  Errors as mpk_sstep_gmres, plus MPK_ERR_ARG for an unknown
 * preconditioner, a `lo` plan of the wrong form or MPK_RITZ_SHIFTS with the
 * Chebyshev preconditioner, and MPK_ERR_UNSUPPORTED if the Ritz values' QR
 * iteration does not converge.
 */
mpk_status mpk_sstep_gmres_ex(mpk_plan_t hi, mpk_plan_t lo, int32_t precond, int32_t s, int32_t m, int32_t degree,
                              double lmin, double lmax, const double* b, double* x, double tol,
                              int32_t max_cycles, uint32_t flags, void* work, size_t work_bytes,
                              int32_t* iters_out, int32_t* cycles_out, double* relres_out, void* stream);

/*
 * Eigenvalues of the k x k upper Hessenberg matrix H (host, column-major, leading
 * dimension ldh >= k; entries below the subdiagonal are ignored), e.g. the Ritz
 * values of an Arnoldi run (Sec. 4: Newton shifts from Ritz values): re[i] + i im[i],
 * i < k, in no particular order.  Shifted QR iteration in complex arithmetic, host
 * only.  Errors: MPK_ERR_ARG (k outside 0..512, ldh < k, null pointers),
 * MPK_ERR_UNSUPPORTED (no convergence), MPK_ERR_NOMEM.
 */
mpk_status mpk_ritz_values(const double* H, int64_t ldh, int32_t k, double* re, double* im);

/* Device work bytes that mpk_sstep_gmres or mpk_sstep_gmres_ex needs for these
 * arguments (n, s, m, d and MPK_IO_PERMUTED in flags; the same for every
 * preconditioner).  Errors: MPK_ERR_ARG. */
mpk_status mpk_sstep_gmres_work_bytes(mpk_plan_t lo, int32_t s, int32_t m, int32_t degree, uint32_t flags,
                                      size_t* bytes);

/*
 * s-step Krylov basis with constant real shifts (Sec. 4):
 *   V[:,0] = v, V[:,k] = (A - lambda[k-1] I) V[:,k-1] / sigma[k-1], k = 1..s,
 * with column k at V + k*ldv (device, ldv >= n).  lambda (host, s entries) are
 * the Newton shifts (all zero gives the monomial basis); sigma (host, s
 * entries) are column scalings, NULL meaning all ones.  v (device, n) may
 * alias V's column 0.  Perm space with MPK_IO_PERMUTED; otherwise through
 * `work`.  Errors: MPK_ERR_ARG (s < 1, ldv < n, zero sigma, null pointers,
 * work too small), MPK_ERR_STATE, MPK_ERR_HIP.
 */
mpk_status sstep_basis(mpk_plan_t plan, int32_t s, const double* lambda, const double* sigma,
                       const double* v, double* V, int64_t ldv, uint32_t flags, void* work,
                       size_t work_bytes, void* stream);

/*
 * Jacobi-preconditioned matrix power kernel (Sec. 5.1 with the right
 * preconditioning of Sec. 5): Y[(j-1)*ldy + i] = ((A P^{-1})^j x)[i] for
 * j = 1..p, where P^{-1} v is the k-th Jacobi iterate
 * z^{i+1} = D^{-1} v - D^{-1} (L + U) z^i from z^0 = 0.  The plan must hold
 * B = A D^{-1} (column_scaling = MPK_SCALE_JACOBI).  Since
 * A P^{-1} = I - (I - B)^k, k = 1 is the MPK of B (the fused A D^{-1} of the
 * paper, blocked over all p powers).  For k > 1 (the Neumann-series polynomial
 * preconditioner) the p k sub-powers u = (B - I) u_prev form one chain in
 * which every k-th sub-power closes a link, w_j = w_{j-1} - (-1)^k u; with
 * MPK_IO_PERMUTED the chain is blocked across links like any matrix power
 * (the P^{-1} -> A -> P^{-1} dependencies of Sec. 5), otherwise each power is
 * one Newton polynomial through poly_apply; both give bitwise equal results.
 * x (device, n) is only read; Y (device, p*ldy, ldy >= n) must not overlap x.
 * Perm space with MPK_IO_PERMUTED.  work: mpk_jacobi_work_bytes(plan, k, p,
 * flags) bytes.  Errors: MPK_ERR_ARG (plan without Jacobi scaling, k outside
 * 1..64, p < 1, ldy < n, null pointers, work too small), MPK_ERR_STATE,
 * MPK_ERR_HIP.
 */
mpk_status mpk_jacobi_apply(mpk_plan_t plan, int32_t k, const double* x, double* Y, int64_t ldy,
                            int32_t p, uint32_t flags, void* work, size_t work_bytes, void* stream);

/* Work bytes mpk_jacobi_apply needs for k sweeps, p powers and `flags`. */
mpk_status mpk_jacobi_work_bytes(mpk_plan_t plan, int32_t k, int32_t p, uint32_t flags, size_t* bytes);

/*
 * GS2-preconditioned matrix power kernel (Sec. 5.1, two-stage Gauss-Seidel
 * with the right preconditioning of Sec. 5): Y[(j-1)*ldy + i] =
 * ((A P^{-1})^j x)[i] for j = 1..p, where P^{-1} v is one outer GS2 iteration
 * from z^0 = 0 with gamma inner Jacobi-Richardson sweeps:
 *   g_0 = D^{-1} v, g_r = g_0 - D^{-1} L g_{r-1} (r = 1..gamma), P^{-1} v = g_gamma,
 * L the strictly lower triangle of A in the original numbering (the form the
 * paper uses, with its short-circuit for z^0 = 0).  Each power is gamma + 2
 * sub-powers (D^{-1}, gamma sweeps with L, then A), and the sub-powers of all
 * p powers run as one chain blocked across powers; each row keeps g_0 and its
 * diagonal entry in registers, and a sweep sums the row's lower entries during
 * the same gather as the full row.  The plan must be built with
 * split_lower = 1.  x (device, n) is only read; Y (device, p*ldy, ldy >= n).
 * Perm space with MPK_IO_PERMUTED (the fast path), otherwise permuted through
 * `work`.  work: device, 256-byte aligned, mpk_gs2_work_bytes(plan, gamma, p,
 * flags) bytes.  MPK_PLAIN / MPK_STAGED select the executor; all executors
 * give bitwise equal results.  Errors: MPK_ERR_ARG (plan without split_lower,
 * gamma outside 0..16, p < 1, ldy < n, null pointers, work too small or
 * misaligned), MPK_ERR_STATE, MPK_ERR_HIP.
 */
mpk_status mpk_gs2_apply(mpk_plan_t plan, int32_t gamma, const double* x, double* Y, int64_t ldy, int32_t p,
                         uint32_t flags, void* work, size_t work_bytes, void* stream);

/* Work bytes mpk_gs2_apply needs for gamma, p powers and `flags`. */
mpk_status mpk_gs2_work_bytes(mpk_plan_t plan, int32_t gamma, int32_t p, uint32_t flags, size_t* bytes);

/*
 * AMG pre-smoothing fused with the residual (Sec. 5.3: the last sub-power of the
 * smoother's chain computes the residual the cycle needs next, so the matrix is
 * reused once more).  Runs `sweeps` outer GS2 iterations on A x = b from the
 * x^0 held in x, in the non-compact (residual-correction) form that the paper
 * names for its GS2 listing (Sec. 5.1):
 *   g_0 = D^{-1}(b - A x^k), g_r = g_0 - D^{-1} L g_{r-1} (r = 1..gamma),
 *   x^{k+1} = x^k + g_gamma,
 * then r = b - A x^sweeps.  gamma = 0 is the Jacobi smoother
 * x^{k+1} = x^k + D^{-1}(b - A x^k); L is the strictly lower triangle of A in
 * the original numbering.  The sweeps (gamma + 1 sub-powers each) and the
 * residual run as one chain of sweeps * (gamma + 1) + 1 sub-powers, blocked
 * across sweeps; each row keeps its sweep's start value, g_0, b_i and its
 * diagonal entry in registers.  The plan must be built with split_lower = 1.
 * b (device, n) is only read; x (device, n) holds x^0 on entry and the smoothed
 * vector on return; r (device, n) receives the residual.  Perm space with
 * MPK_IO_PERMUTED (the fast path), otherwise permuted through `work`.  work:
 * device, 256-byte aligned, mpk_gs2_smooth_work_bytes(plan, gamma, flags) bytes.
 * MPK_PLAIN / MPK_STAGED select the executor; all executors give bitwise equal
 * results.  sweeps = 0 computes only r = b - A x.  Errors: MPK_ERR_ARG (plan
 * without split_lower, gamma outside 0..16, sweeps outside 0..65536, null
 * pointers, work too small or misaligned), MPK_ERR_STATE, MPK_ERR_HIP.
 */
mpk_status mpk_gs2_smooth(mpk_plan_t plan, int32_t gamma, int32_t sweeps, const double* b, double* x, double* r,
                          uint32_t flags, void* work, size_t work_bytes, void* stream);

/* Work bytes mpk_gs2_smooth needs for gamma and `flags`. */
mpk_status mpk_gs2_smooth_work_bytes(mpk_plan_t plan, int32_t gamma, uint32_t flags, size_t* bytes);

/*
 * p_opt of Sec. 3 (the powers per blocked launch, which the paper tunes over
 * 1..8 per matrix and machine).  mpk_set_block caps the powers per blocked
 * launch of every later call on the plan at q (1..15; 0 removes the cap; the
 * deadlock bound of the plan still applies).  mpk_tune_block times
 * mpk_apply(x, Y, ldy, p, MPK_IO_PERMUTED) on `stream` for each admissible
 * q = 1..min(p, bound) (one warm-up and three timed calls each, HIP events),
 * keeps the fastest as the plan's cap and returns it in *q_out and its time
 * per call in *seconds_out (may be NULL).  x and Y (device, perm space, Y of
 * p*ldy) are the caller's buffers; Y is overwritten.  Every q gives bitwise
 * identical powers, so tuning changes time only.  Synchronises `stream`.
 * Both change the plan's state: they must not overlap other calls on the
 * same plan (unlike the compute calls, which may overlap on several streams).
 * Errors: MPK_ERR_ARG (q or p out of range, ldy < n, null pointers),
 * MPK_ERR_STATE, MPK_ERR_HIP, MPK_ERR_DEVICE.
 */
mpk_status mpk_set_block(mpk_plan_t plan, int32_t q);
mpk_status mpk_tune_block(mpk_plan_t plan, int32_t p, const double* x, double* Y, int64_t ldy, void* stream,
                          int32_t* q_out, double* seconds_out);

/*
 * Permutes a device vector into the plan's level order, x_perm[i] = x[perm[i]]
 * (direction 0), or back, x[perm[i]] = x_perm[i] (direction 1).  in and out
 * must not alias.
 */
mpk_status mpk_permute(mpk_plan_t plan, const double* in, double* out, int32_t direction,
                       void* stream);

/*
 * Waits for `stream`, then reads the plan's device status for that stream:
 * every stream that launches the blocked kernel on a plan gets its own status
 * slot (64 per plan; beyond that the least recently used stream's slot is
 * reused).  MPK_OK if every blocked launch of the plan on `stream` since the
 * last check finished normally; MPK_ERR_DEVICE if a wave gave up waiting
 * (watchdog: an entry it reads not written within the poll limit, about a
 * second by default, e.g. because the GPU could not keep every worker
 * resident); the message names the chunk and power.  After such a failure the
 * launch's outputs are undefined, and later blocked launches of the plan on
 * the same stream stop early until the check clears the status.
 */
mpk_status mpk_check_device(mpk_plan_t plan, void* stream);

/*
 * Sets the watchdog of the plan's blocked launches: polls of a pending entry
 * before a wave gives up (0: the default of about 10^6; negative: give up at
 * the first wait, which tests of the failure path use).  Applies to launches
 * enqueued after the call; must not overlap other calls on the plan.
 * Errors: MPK_ERR_ARG (null plan).
 */
mpk_status mpk_set_watchdog(mpk_plan_t plan, int32_t polls);

/*
 * Plan facts: n, nnz, number of levels, chunk count, SELL slots (padded
 * entries), register slots per row used by the blocked kernel, the blocked
 * kernel's workers per XCD for blocks of p_block powers, and the effective
 * p_block.  Any pointer may be NULL.
 */
mpk_status mpk_plan_info(mpk_plan_t plan, int64_t* n, int64_t* nnz, int32_t* nlevels,
                         int32_t* nchunks, int64_t* sell_slots, int32_t* reg_slots,
                         int32_t* workers_per_xcd, int32_t* p_block);

/* Releases the plan (not the caller's device buffers).  NULL is ignored. */
void mpk_destroy(mpk_plan_t plan);

/*
 * ---- Request server ----------------------------------------------------
 * Serves matrix power requests (mpk_apply), refinement solves
 * (mpk_refine_solve) and s-step GMRES solves (mpk_sstep_gmres) submitted from host memory by any number of host
 * threads, on the device that is current at mpk_server_create.  Each worker
 * thread owns a HIP stream and runs one request at a time: copy in, compute,
 * copy out, mpk_check_device for its stream.  mpk_server_create_ex starts
 * `workers` workers that take any request and `apply_workers` that take
 * matrix power requests only (so that they never wait behind long solves).
 * A free worker starts the oldest waiting request of its kind whose device
 * memory fits in the server's pool of `device_bytes` (one allocation made
 * here, sub-allocated first-fit with 256-byte alignment); younger requests
 * that fit may start before an older one that does not, but once the oldest
 * waiting request has waited more than `max_wait_s` and does not fit, no
 * request starts until it does.  mpk_server_create(workers, device_bytes) is
 * mpk_server_create_ex(workers, 0, device_bytes, 0): strict arrival order.
 * Requests on matrices of fewer than 2^19 rows run the plain kernels (unless
 * MPK_STAGED is asked for): their blocked launches would wait for the
 * device-wide turn of persistent kernels; the results are the same bitwise.
 * Plans must stay alive and uploaded until their requests have been waited
 * for.  Host buffers passed to a submit call belong to the caller but must
 * stay valid, and unwritten by the caller, until mpk_server_wait returns for
 * that ticket.  Results equal those of the same call made alone.
 * Errors: MPK_ERR_ARG (null, bad scalar or flag), MPK_ERR_NOMEM (a request
 * larger than the whole pool is refused at submit), MPK_ERR_HIP.
 */
mpk_status mpk_server_create(int32_t workers, size_t device_bytes, mpk_server_t* out);
mpk_status mpk_server_create_ex(int32_t workers, int32_t apply_workers, size_t device_bytes, double max_wait_s,
                                mpk_server_t* out);

/*
 * Queues Y(:, k-1) = y_k, k = 1..p, for x (host, n doubles) into Y (host,
 * n x p column-major), as mpk_apply with `flags`; with MPK_LAST_POWER in
 * flags, Y (n doubles) receives y_p only.  Device memory taken: n + n*p
 * doubles plus mpk_work_bytes(plan, MPK_CALL_APPLY, p, flags).
 * *ticket identifies the request for mpk_server_wait.
 */
mpk_status mpk_server_submit_apply(mpk_server_t server, mpk_plan_t plan, const double* x, int32_t p,
                                   double* Y, uint32_t flags, int64_t* ticket);

/*
 * Queues mpk_refine_solve(hi, lo, degree, lmin, lmax, b, x, tol, max_iter,
 * flags): b (host, n doubles) is the right-hand side, x (host, n doubles)
 * holds the initial guess on entry and the solution when the request is
 * done.  Device memory taken: 2n doubles plus
 * mpk_work_bytes(lo, MPK_CALL_SOLVE, degree, flags).
 */
mpk_status mpk_server_submit_solve(mpk_server_t server, mpk_plan_t hi, mpk_plan_t lo, const double* b,
                                   double* x, int32_t degree, double lmin, double lmax, double tol,
                                   int32_t max_iter, uint32_t flags, int64_t* ticket);

/*
 * Queues mpk_sstep_gmres(hi, lo, s, m, degree, lmin, lmax, b, x, tol,
 * max_cycles, flags): b (host, n doubles) is the right-hand side, x (host, n
 * doubles) holds the initial guess on entry and the solution when the request
 * is done; mpk_server_wait reports the basis vectors built as `iters`.
 * Device memory taken: 2n doubles plus mpk_sstep_gmres_work_bytes(lo, s, m,
 * degree, flags).  Errors at submit: MPK_ERR_ARG (null, unknown flag, s, m or
 * degree out of range), MPK_ERR_NOMEM; the solve's own errors at wait.
 */
mpk_status mpk_server_submit_gmres(mpk_server_t server, mpk_plan_t hi, mpk_plan_t lo, const double* b,
                                   double* x, int32_t s, int32_t m, int32_t degree, double lmin, double lmax,
                                   double tol, int32_t max_cycles, uint32_t flags, int64_t* ticket);

/*
 * Blocks until request `ticket` is done and releases it (a ticket may be
 * waited for once).  *status receives the request's own status (its message
 * is then available from mpk_last_error on this thread); latency_s is the
 * time from submit to completion, queue_s the time spent waiting for
 * admission; iters and relres are the solve's (0 for applies).  Any output
 * pointer may be NULL.  Returns MPK_ERR_ARG for an unknown ticket.
 */
mpk_status mpk_server_wait(mpk_server_t server, int64_t ticket, mpk_status* status, double* latency_s,
                           double* queue_s, int32_t* iters, double* relres);

/* Finishes every queued request, joins the workers and frees the pool. */
void mpk_server_destroy(mpk_server_t server);

#ifdef __cplusplus
}
#endif

#endif /* MPK_H */
