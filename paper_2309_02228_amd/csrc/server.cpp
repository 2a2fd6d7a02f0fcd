// Request server of the MPK library: MPK applications, refinement solves and
// s-step GMRES solves submitted from the host run on worker threads, each with
// its own HIP stream.  A waiting request is admitted as soon as a worker of its
// lane is free and its device memory fits in the server's pool: matrix powers
// have workers of their own, so short applications do not queue behind long
// solves, and any waiting request that fits may start before older ones that
// do not, until the oldest has waited longer than the aging bound (then the
// pool is kept for it).  Work of different requests overlaps on the GPU;
// blocked (persistent) launches take turns, as everywhere in the library, so
// that each has its waves resident together.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <exception>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"

MPK_API void mpk_server_destroy(mpk_server_t S);

namespace {

using Clock = std::chrono::steady_clock;
constexpr size_t kAlign = 256;
// Requests on matrices with fewer rows run the plain kernels: a blocked launch
// waits for the device-wide turn of persistent kernels (behind the launches of
// concurrent solves), which costs small matrices more than blocking saves; the
// results are the same bitwise.
constexpr int32_t kSmallRows = 1 << 19;

// The executor flags of a request: the caller's, with the plain kernels for
// small matrices unless the staged executor was asked for.
uint32_t exec_flags(uint32_t flags, int32_t n) {
    if (n < kSmallRows && !(flags & MPK_STAGED)) flags |= MPK_PLAIN;
    return flags;
}

size_t round_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

// First-fit sub-allocator over the server's single device allocation.
struct Pool {
    char* base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_;  // offset -> length, coalesced

    bool alloc(size_t n, size_t* off) {
        n = round_up(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n, at = it->first + n;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }

    bool fits(size_t n) const {
        n = round_up(n);
        for (const auto& kv : free_)
            if (kv.second >= n) return true;
        return false;
    }

    void release(size_t off, size_t n) {
        n = round_up(n);
        auto it = free_.emplace(off, n).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
};

enum { kApply = 0, kSolve = 1, kGmres = 2 };

struct Request {
    int type = kApply;
    mpk_plan_t plan = nullptr, lo = nullptr;
    int32_t n = 0, p = 0, degree = 0, max_iter = 0, s = 0, m = 0;
    double lmin = 0, lmax = 0, tol = 0;
    uint32_t flags = 0;
    const double* in = nullptr;  // host: x (apply) or b (solve)
    double* out = nullptr;       // host: Y (apply) or x (solve; the initial guess on entry)
    size_t bytes = 0, work = 0, off = 0;
    Clock::time_point t_submit, t_start, t_done;
    bool done = false;
    mpk_status status = MPK_OK;
    std::string error;
    int32_t iters = 0;
    double relres = 0.0;
};

}  // namespace

struct mpk_server_s {
    int device = 0;
    int apply_workers = 0;            // workers that take matrix-power requests only
    double max_wait_s = 0.25;         // aging bound of any-fit admission
    Pool pool;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> queue;
    std::unordered_map<int64_t, Request*> requests;
    int64_t next_ticket = 1;
    bool stop = false;
    std::vector<std::thread> threads;
};

namespace {

// Runs one admitted request on the worker's stream, with its device memory
// at `d` (r->bytes bytes).
void execute(Request* r, char* d, hipStream_t st) {
    const size_t n = (size_t)r->n;
    auto hip = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && r->status == MPK_OK) {
            r->status = MPK_ERR_HIP;
            r->error = std::string(what) + ": " + hipGetErrorString(e);
        }
        return e == hipSuccess;
    };
    auto lib = [&](mpk_status s) {
        if (s != MPK_OK && r->status == MPK_OK) {
            r->status = s;
            r->error = mpk_last_error();
        }
        return s == MPK_OK;
    };
    if (r->type == kApply) {
        double* x = (double*)d;
        double* Y = (double*)(d + round_up(n * 8));
        void* w = r->work ? (void*)(d + round_up(n * 8) + round_up(n * 8 * r->p)) : nullptr;
        if (!hip(hipMemcpyAsync(x, r->in, n * 8, hipMemcpyHostToDevice, st), "copy x")) return;
        const bool last = r->flags & MPK_LAST_POWER;
        const uint32_t fl = exec_flags(r->flags & ~MPK_LAST_POWER, r->n);
        if (!lib(mpk_apply(r->plan, x, Y, (int64_t)n, r->p, fl, w, r->work, st))) return;
        const double* from = last ? Y + n * (size_t)(r->p - 1) : Y;
        if (!hip(hipMemcpyAsync(r->out, from, n * 8 * (last ? 1 : r->p), hipMemcpyDeviceToHost, st), "copy Y"))
            return;
        lib(mpk_check_device(r->plan, st));
    } else {
        double* b = (double*)d;
        double* x = (double*)(d + round_up(n * 8));
        void* w = d + 2 * round_up(n * 8);
        if (!hip(hipMemcpyAsync(b, r->in, n * 8, hipMemcpyHostToDevice, st), "copy b")) return;
        if (!hip(hipMemcpyAsync(x, r->out, n * 8, hipMemcpyHostToDevice, st), "copy x")) return;
        if (r->type == kSolve) {
            if (!lib(mpk_refine_solve(r->plan, r->lo, r->degree, r->lmin, r->lmax, b, x, r->tol, r->max_iter,
                                      exec_flags(r->flags, r->n), w, r->work, &r->iters, &r->relres, st)))
                return;
        } else {
            int32_t cycles = 0;
            if (!lib(mpk_sstep_gmres(r->plan, r->lo, r->s, r->m, r->degree, r->lmin, r->lmax, b, x, r->tol,
                                     r->max_iter, exec_flags(r->flags, r->n), w, r->work, &r->iters, &cycles,
                                     &r->relres, st)))
                return;
        }
        if (!hip(hipMemcpyAsync(r->out, x, n * 8, hipMemcpyDeviceToHost, st), "copy x back")) return;
        if (lib(mpk_check_device(r->plan, st))) lib(mpk_check_device(r->lo, st));
    }
    hip(hipStreamSynchronize(st), "synchronize");
}

// Picks the request a worker of the given lane starts now (holding S->mu), or
// null: the oldest waiting request of the lane whose device memory fits.  While
// the oldest waiting request overall has waited longer than the aging bound and
// its memory does not fit, no request is admitted, so that the pool fills up for
// it; it is taken as soon as it fits by a worker of its lane.
Request* admit(mpk_server_s* S, bool applies_only) {
    if (S->queue.empty()) return nullptr;
    Request* oldest = S->queue.front();
    const bool aged = std::chrono::duration<double>(Clock::now() - oldest->t_submit).count() > S->max_wait_s;
    if (aged && !S->pool.fits(oldest->bytes)) return nullptr;
    for (auto it = S->queue.begin(); it != S->queue.end(); ++it) {
        Request* r = *it;
        if (applies_only && r->type != kApply) continue;
        if (S->pool.alloc(r->bytes, &r->off)) {
            S->queue.erase(it);
            return r;
        }
    }
    return nullptr;
}

void worker(mpk_server_s* S, bool applies_only) {
    hipSetDevice(S->device);
    hipStream_t st = nullptr;
    const hipError_t se = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    for (;;) {
        Request* r = nullptr;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            for (;;) {
                r = admit(S, applies_only);
                if (r || (S->stop && S->queue.empty())) break;
                // wake up at least every millisecond so that the aging bound is
                // applied while nothing completes
                S->cv_work.wait_for(lk, std::chrono::milliseconds(1));
            }
            if (!r) break;
        }
        r->t_start = Clock::now();
        if (se != hipSuccess) {
            r->status = MPK_ERR_HIP;
            r->error = std::string("stream creation: ") + hipGetErrorString(se);
        } else {
            execute(r, S->pool.base + r->off, st);
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->pool.release(r->off, r->bytes);
            r->t_done = Clock::now();
            r->done = true;
        }
        S->cv_work.notify_all();
        S->cv_done.notify_all();
    }
    if (st) hipStreamDestroy(st);
}

mpk_status submit(mpk_server_t S, Request* r, int64_t* ticket) {
    if (r->bytes > S->pool.size) {
        const size_t need = r->bytes, have = S->pool.size;
        delete r;
        return mpk::set_error(MPK_ERR_NOMEM, "request needs %zu device bytes, the server holds %zu", need, have);
    }
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        *ticket = S->next_ticket++;
        S->requests[*ticket] = r;
        S->queue.push_back(r);
    }
    S->cv_work.notify_all();
    return MPK_OK;
}

}  // namespace

MPK_API mpk_status mpk_server_create_ex(int32_t workers, int32_t apply_workers, size_t device_bytes,
                                        double max_wait_s, mpk_server_t* out) {
    if (!out) return mpk::set_error(MPK_ERR_ARG, "out is null");
    *out = nullptr;
    if (workers < 1 || workers > 64) return mpk::set_error(MPK_ERR_ARG, "workers must be in 1..64");
    if (apply_workers < 0 || apply_workers > 64)
        return mpk::set_error(MPK_ERR_ARG, "apply_workers must be in 0..64");
    if (!(max_wait_s >= 0.0)) return mpk::set_error(MPK_ERR_ARG, "max_wait_s must be >= 0");
    if (device_bytes < kAlign) return mpk::set_error(MPK_ERR_ARG, "device_bytes must be at least %zu", kAlign);
    auto* S = new (std::nothrow) mpk_server_s;
    if (!S) return mpk::set_error(MPK_ERR_NOMEM, "out of host memory");
    S->apply_workers = apply_workers;
    S->max_wait_s = max_wait_s;
    hipError_t e = hipGetDevice(&S->device);
    if (e == hipSuccess) e = hipMalloc((void**)&S->pool.base, device_bytes);
    if (e != hipSuccess) {
        delete S;
        return mpk::set_error(MPK_ERR_HIP, "server memory: %s", hipGetErrorString(e));
    }
    S->pool.size = device_bytes / kAlign * kAlign;
    S->pool.free_[0] = S->pool.size;
    try {
        for (int i = 0; i < workers; ++i) S->threads.emplace_back(worker, S, false);
        for (int i = 0; i < apply_workers; ++i) S->threads.emplace_back(worker, S, true);
    } catch (const std::exception& ex) {  // no exception crosses the C ABI
        mpk_server_destroy(S);
        return mpk::set_error(MPK_ERR_NOMEM, "worker threads: %s", ex.what());
    }
    *out = S;
    return MPK_OK;
}

MPK_API mpk_status mpk_server_create(int32_t workers, size_t device_bytes, mpk_server_t* out) {
    // strict arrival order (an aging bound of zero) and no lane of its own for
    // matrix powers
    return mpk_server_create_ex(workers, 0, device_bytes, 0.0, out);
}

MPK_API mpk_status mpk_server_submit_apply(mpk_server_t S, mpk_plan_t plan, const double* x, int32_t p, double* Y,
                                           uint32_t flags, int64_t* ticket) {
    if (!S || !plan || !ticket) return mpk::set_error(MPK_ERR_ARG, "null argument");
    if (p < 1) return mpk::set_error(MPK_ERR_ARG, "p must be >= 1 (got %d)", p);
    if (flags & ~(MPK_IO_PERMUTED | MPK_PLAIN | MPK_STAGED | MPK_LAST_POWER))
        return mpk::set_error(MPK_ERR_ARG, "unknown flag bits");
    int64_t n = 0, nnz = 0, slots = 0;
    int32_t nl, nc, reg, wk, pb;
    mpk_status s = mpk_plan_info(plan, &n, &nnz, &nl, &nc, &slots, &reg, &wk, &pb);
    if (s != MPK_OK) return s;
    if (n > 0 && (!x || !Y)) return mpk::set_error(MPK_ERR_ARG, "x or Y is null");
    auto* r = new Request;
    r->type = kApply;
    r->plan = plan;
    r->n = (int32_t)n;
    r->p = p;
    r->flags = flags;
    r->in = x;
    r->out = Y;
    mpk_work_bytes(plan, MPK_CALL_APPLY, p, flags & ~MPK_LAST_POWER, &r->work);
    r->bytes = round_up(n * 8) + round_up(n * 8 * p) + round_up(r->work) + kAlign;
    return submit(S, r, ticket);
}

MPK_API mpk_status mpk_server_submit_solve(mpk_server_t S, mpk_plan_t hi, mpk_plan_t lo, const double* b, double* x,
                                           int32_t degree, double lmin, double lmax, double tol, int32_t max_iter,
                                           uint32_t flags, int64_t* ticket) {
    if (!S || !hi || !lo || !ticket) return mpk::set_error(MPK_ERR_ARG, "null argument");
    if (flags & ~(MPK_IO_PERMUTED | MPK_PLAIN | MPK_STAGED)) return mpk::set_error(MPK_ERR_ARG, "unknown flag bits");
    int64_t n = 0, nnz = 0, slots = 0;
    int32_t nl, nc, reg, wk, pb;
    mpk_status s = mpk_plan_info(hi, &n, &nnz, &nl, &nc, &slots, &reg, &wk, &pb);
    if (s != MPK_OK) return s;
    if (n > 0 && (!b || !x)) return mpk::set_error(MPK_ERR_ARG, "b or x is null");
    if (degree < 1) return mpk::set_error(MPK_ERR_ARG, "degree must be >= 1");
    auto* r = new Request;
    r->type = kSolve;
    r->plan = hi;
    r->lo = lo;
    r->n = (int32_t)n;
    r->degree = degree;
    r->lmin = lmin;
    r->lmax = lmax;
    r->tol = tol;
    r->max_iter = max_iter;
    r->flags = flags;
    r->in = b;
    r->out = x;
    s = mpk_work_bytes(lo, MPK_CALL_SOLVE, degree, flags, &r->work);
    if (s != MPK_OK) {
        delete r;
        return s;
    }
    r->bytes = 2 * round_up(n * 8) + round_up(r->work) + kAlign;
    return submit(S, r, ticket);
}

MPK_API mpk_status mpk_server_submit_gmres(mpk_server_t S, mpk_plan_t hi, mpk_plan_t lo, const double* b, double* x,
                                           int32_t s, int32_t m, int32_t degree, double lmin, double lmax, double tol,
                                           int32_t max_cycles, uint32_t flags, int64_t* ticket) {
    if (!S || !hi || !lo || !ticket) return mpk::set_error(MPK_ERR_ARG, "null argument");
    if (flags & ~(MPK_IO_PERMUTED | MPK_PLAIN | MPK_STAGED)) return mpk::set_error(MPK_ERR_ARG, "unknown flag bits");
    int64_t n = 0;
    mpk_status st = mpk_plan_info(hi, &n, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    if (st != MPK_OK) return st;
    if (n > 0 && (!b || !x)) return mpk::set_error(MPK_ERR_ARG, "b or x is null");
    auto* r = new Request;
    r->type = kGmres;
    r->plan = hi;
    r->lo = lo;
    r->n = (int32_t)n;
    r->s = s;
    r->m = m;
    r->degree = degree;
    r->lmin = lmin;
    r->lmax = lmax;
    r->tol = tol;
    r->max_iter = max_cycles;
    r->flags = flags;
    r->in = b;
    r->out = x;
    st = mpk_sstep_gmres_work_bytes(lo, s, m, degree, flags, &r->work);
    if (st != MPK_OK) {
        delete r;
        return st;
    }
    r->bytes = 2 * round_up(n * 8) + round_up(r->work) + kAlign;
    return submit(S, r, ticket);
}

MPK_API mpk_status mpk_server_wait(mpk_server_t S, int64_t ticket, mpk_status* status, double* latency_s,
                                   double* queue_s, int32_t* iters, double* relres) {
    if (!S) return mpk::set_error(MPK_ERR_ARG, "null server");
    Request* r = nullptr;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        auto it = S->requests.find(ticket);
        if (it == S->requests.end()) return mpk::set_error(MPK_ERR_ARG, "unknown ticket %lld", (long long)ticket);
        r = it->second;
        S->cv_done.wait(lk, [&] { return r->done; });
        S->requests.erase(it);
    }
    using sec = std::chrono::duration<double>;
    if (status) *status = r->status;
    if (latency_s) *latency_s = sec(r->t_done - r->t_submit).count();
    if (queue_s) *queue_s = sec(r->t_start - r->t_submit).count();
    if (iters) *iters = r->iters;
    if (relres) *relres = r->relres;
    if (r->status != MPK_OK) mpk::set_error(r->status, "%s", r->error.c_str());
    delete r;
    return MPK_OK;
}

MPK_API void mpk_server_destroy(mpk_server_t S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    for (auto& t : S->threads) t.join();  // workers drain the queue first
    for (auto& kv : S->requests) delete kv.second;
    hipSetDevice(S->device);
    hipFree(S->pool.base);
    delete S;
}
