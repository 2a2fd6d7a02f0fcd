/*
 * Plain C reference of the matrix power kernel -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py
 * use it; it shares nothing with the HIP path.  It restates the definition of
 * the MPK (Sec. 3, Alg. 1: y_0 = x, y_k = A y_{k-1} for k = 1..p, every y_k
 * stored): each row's sum runs over its stored entries in order, from zero,
 * each product rounded on its own.  Built with -ffp-contract=off so that no
 * multiply-add is fused; the result then equals the NumPy oracle's bitwise.
 *
 * mpk_ref      -- one thread.
 * mpk_ref_omp  -- the same loops, rows split over OpenMP threads (each row is
 *                 still summed by one thread in the same order, so the result
 *                 is identical); nthreads <= 0 uses the OpenMP default.
 *
 * A is CSR with n rows (rowptr[n+1], col[nnz], val[nnz], 0-based); x has n
 * entries; Y receives p vectors of n entries, Y[(k-1) n + i] = (A^k x)[i].
 */
#include <stdint.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static void power_rows(int64_t r0, int64_t r1, const int32_t* rowptr, const int32_t* col, const double* val,
                       const double* in, double* out) {
    for (int64_t i = r0; i < r1; ++i) {
        double sum = 0.0;
        for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) sum = sum + val[e] * in[col[e]];
        out[i] = sum;
    }
}

void mpk_ref(int32_t n, const int32_t* rowptr, const int32_t* col, const double* val, const double* x, double* Y,
             int32_t p) {
    for (int32_t k = 1; k <= p; ++k) {
        const double* in = k == 1 ? x : Y + (int64_t)(k - 2) * n;
        power_rows(0, n, rowptr, col, val, in, Y + (int64_t)(k - 1) * n);
    }
}

int32_t mpk_ref_omp(int32_t n, const int32_t* rowptr, const int32_t* col, const double* val, const double* x,
                    double* Y, int32_t p, int32_t nthreads) {
    int32_t used = 1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    for (int32_t k = 1; k <= p; ++k) {
        const double* in = k == 1 ? x : Y + (int64_t)(k - 2) * n;
        double* out = Y + (int64_t)(k - 1) * n;
#ifdef _OPENMP
#pragma omp parallel
        {
            const int64_t t = omp_get_thread_num(), nt = omp_get_num_threads();
#pragma omp single
            used = (int32_t)nt;
            power_rows(n * t / nt, n * (t + 1) / nt, rowptr, col, val, in, out);
        }
#else
        power_rows(0, n, rowptr, col, val, in, out);
#endif
    }
    return used;
}
