// s-step GMRES (Sec. 4, Alg. 3a with the subspace routine of Alg. 3c) with a right
// Chebyshev polynomial preconditioner (Sec. 5), on one MI355X.
//
// The operator is M = A s(A), s the degree d - 1 Chebyshev interpolant of 1/lambda
// on [lmin, lmax]; its residual polynomial gives M = I - T_d((theta I - A)/delta) /
// T_d(theta/delta), so one Newton basis step (M - lambda_k I) v / sigma_k is a single
// Chebyshev polynomial of degree d in A with two nonzero coefficients, run as one
// blocked matrix power launch of d powers (poly_apply).  The orthogonalisation is
// one block classical Gram-Schmidt sweep (BOrtho) and a Cholesky QR (TSQR), both in
// FP64; the Hessenberg matrix is rebuilt from the change of basis on the host.
//
// Device work per block of s vectors: s polynomial launches, two tall-skinny Gram
// products (Q^T W, then W'^T W') and two linear combinations (W - Q R_prev, then
// W' R^{-1}).  The Gram products stream their operands once, coalesced (a row per
// lane), and their partial sums are added in a fixed order, so a solve is
// deterministic.  Small matrices travel between host and device with one
// synchronisation per Gram product.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <limits>
#include <new>
#include <vector>

#include "internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kMaxParts = 1024;     // row blocks of a Gram product
constexpr int kMaxS = 16;           // vectors per block
constexpr int kMaxM = 256;          // restart length
constexpr int kMaxC = (kMaxM + 1) * kMaxS;  // coefficients of a linear combination
constexpr double kEta = 1.0 / 16777216.0;   // 2^-24: the dependent-column threshold

// ------------------------------------------------------------------ kernels
// Sum over the 64 lanes of a wave of 64 values per lane by recursive halving: at
// distance w each lane keeps the half of its values selected by its lane bit w and
// receives the partner's copy of that half.  Lane L ends with the total of value L.
template <int W>
__device__ __forceinline__ void halve(double* v, int lane) {
    const bool hi = lane & W;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        const double send = hi ? v[i] : v[i + W];
        const double keep = hi ? v[i + W] : v[i];
        v[i] = keep + __shfl_xor(send, W);
    }
}

// part[j][k][rb] = sum over rows r of block rb of X[j][r] * Y[k][r], j < a, k < b
// (element-major, so that the reduction reads each element's partials contiguously).
// A workgroup covers one row block and one JB x KB tile; workgroups of the same row
// block sit on the same XCD (workgroup i runs on XCD i mod 8), so the tiles re-read
// each other's rows from that XCD's L2.
template <int JB, int KB>
__global__ __launch_bounds__(kThreads) void gram_partial_kernel(const double* __restrict__ X, int64_t ldx, int a,
                                                                const double* __restrict__ Y, int64_t ldy, int b,
                                                                int n, int rows_per_blk, int nrb, int ntj, int ntk,
                                                                double* __restrict__ part) {
    const int tiles = ntj * ntk;
    const int id = blockIdx.x, xcd = id & 7, loc = id >> 3;
    const int rb = (loc / tiles) * 8 + xcd;
    const int tile = loc % tiles;
    if (rb >= nrb) return;
    const int j0 = (tile % ntj) * JB, k0 = (tile / ntj) * KB;
    double acc[JB * KB];
#pragma unroll
    for (int e = 0; e < JB * KB; ++e) acc[e] = 0.0;
    const int r0 = rb * rows_per_blk;
    const int r1 = min(n, r0 + rows_per_blk);
#pragma unroll 2
    for (int r = r0 + (int)threadIdx.x; r < r1; r += kThreads) {
        double xv[JB], yv[KB];
#pragma unroll
        for (int j = 0; j < JB; ++j) xv[j] = (j0 + j < a) ? __builtin_nontemporal_load(X + (j0 + j) * ldx + r) : 0.0;
#pragma unroll
        for (int k = 0; k < KB; ++k) yv[k] = (k0 + k < b) ? Y[(k0 + k) * ldy + r] : 0.0;
#pragma unroll
        for (int j = 0; j < JB; ++j)
#pragma unroll
            for (int k = 0; k < KB; ++k) acc[j * KB + k] = fma(xv[j], yv[k], acc[j * KB + k]);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __shared__ double red[kThreads / 64][64];
    if constexpr (JB * KB == 64) {
        halve<32>(acc, lane);
        halve<16>(acc, lane);
        halve<8>(acc, lane);
        halve<4>(acc, lane);
        halve<2>(acc, lane);
        halve<1>(acc, lane);
        red[wave][lane] = acc[0];
    } else {
#pragma unroll
        for (int e = 0; e < JB * KB; ++e)
            for (int off = 32; off > 0; off >>= 1) acc[e] += __shfl_xor(acc[e], off);
        if (lane < JB * KB) {
#pragma unroll
            for (int e = 0; e < JB * KB; ++e)
                if (e == lane) red[wave][lane] = acc[e];
        }
    }
    __syncthreads();
    if (threadIdx.x < JB * KB) {
        const int e = threadIdx.x, j = e / KB, k = e % KB;
        double sum = 0.0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) sum += red[w][e];
        if (j0 + j < a && k0 + k < b) part[((int64_t)(j0 + j) * b + k0 + k) * nrb + rb] = sum;
    }
}

// out[e] = sum over the row blocks of part[e][rb]: one workgroup per element, each
// thread a fixed strided subset of row blocks, then a fixed tree, so the order of the
// additions never changes.
__global__ __launch_bounds__(kThreads) void reduce_parts_kernel(const double* __restrict__ part, int nrb,
                                                                double* __restrict__ out) {
    const int e = blockIdx.x;
    const double* src = part + (int64_t)e * nrb;
    double s = 0.0;
    for (int rb = threadIdx.x; rb < nrb; rb += kThreads) s += src[rb];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    __shared__ double red[kThreads / 64];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) t += red[w];
        out[e] = t;
    }
}

// Y[k][r] = alpha X0[k][r] + sum_{j < a} Q[j][r] C[j b + k], k < b <= KB.
// Y may be X0 (elementwise update in place) or, with a == 1 and b == 1, Q itself.
template <int KB>
__global__ __launch_bounds__(kThreads) void lincomb_kernel(const double* X0, int64_t ldx0, double alpha,
                                                           const double* Q, int64_t ldq, int a,
                                                           const double* __restrict__ C, int b, double* Y,
                                                           int64_t ldy, int n) {
    __shared__ double cs[kMaxC];
    for (int e = threadIdx.x; e < a * b; e += kThreads) cs[e] = C[e];
    __syncthreads();
    for (int r = blockIdx.x * kThreads + threadIdx.x; r < n; r += gridDim.x * kThreads) {
        double acc[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) acc[k] = (k < b && X0) ? alpha * X0[k * ldx0 + r] : 0.0;
#pragma unroll 4
        for (int j = 0; j < a; ++j) {
            const double q = Q[j * ldq + r];
#pragma unroll
            for (int k = 0; k < KB; ++k)
                if (k < b) acc[k] = fma(q, cs[j * b + k], acc[k]);
        }
#pragma unroll
        for (int k = 0; k < KB; ++k)
            if (k < b) Y[k * ldy + r] = acc[k];
    }
}

// x += z / d (the diagonal preconditioner applied to the correction)
__global__ void add_div_kernel(double* __restrict__ x, const double* __restrict__ z, const double* __restrict__ d,
                               int n) {
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) x[i] = x[i] + z[i] / d[i];
}

// r = b - t
__global__ void sub_kernel(const double* __restrict__ b, const double* __restrict__ t, double* __restrict__ r, int n) {
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) r[i] = b[i] - t[i];
}

int grid_rows(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(8192, (n + kThreads - 1) / kThreads)); }

// ------------------------------------------------------------ host helpers
struct Layout {
    int64_t ld = 0;          // doubles between vectors (256-byte multiple)
    int rows_per_blk = 0, nrb = 0;
    size_t q = 0, w = 0, t = 0, z = 0, diag = 0, part = 0, small = 0, cbuf = 0, io = 0, poly = 0, total = 0;
    size_t poly_bytes = 0;
};

Layout layout(int64_t n, int s, int m, size_t poly_bytes, bool permuted) {
    Layout L;
    L.ld = std::max<int64_t>(32, (n + 31) / 32 * 32);
    const int64_t rpt = std::max<int64_t>(4, (n + (int64_t)kThreads * kMaxParts - 1) / ((int64_t)kThreads * kMaxParts));
    L.rows_per_blk = (int)(rpt * kThreads);
    L.nrb = (int)std::max<int64_t>(1, (n + L.rows_per_blk - 1) / L.rows_per_blk);
    size_t at = 0;
    auto take = [&](size_t doubles) {
        const size_t here = at;
        at += (doubles + 31) / 32 * 32;
        return here;
    };
    L.q = take((size_t)(m + 1) * L.ld);
    L.w = take((size_t)(s + 1) * L.ld);  // the block's first vector, then W_1..W_s
    L.t = take(L.ld);
    L.z = take(L.ld);
    L.diag = take(L.ld);
    L.part = take((size_t)L.nrb * (m + 1) * s);
    L.small = take((size_t)(m + 1) * s);
    L.cbuf = take((size_t)4 * kMaxC);
    L.io = take(permuted ? 0 : 2 * (size_t)L.ld);
    L.poly = take((poly_bytes + 7) / 8);
    L.poly_bytes = poly_bytes;
    L.total = at * 8;
    return L;
}

// Dense least squares min ||e - H y|| for H (rows x cols, column-major, rows >= cols)
// by Householder QR; returns y.
std::vector<double> least_squares(const std::vector<double>& H, int rows, int cols, std::vector<double> e) {
    std::vector<double> R(H);
    for (int k = 0; k < cols; ++k) {
        double nrm = 0.0;
        for (int i = k; i < rows; ++i) nrm += R[k * rows + i] * R[k * rows + i];
        nrm = std::sqrt(nrm);
        if (nrm == 0.0) continue;
        const double alpha = R[k * rows + k] > 0 ? -nrm : nrm;
        std::vector<double> v(rows - k);
        for (int i = k; i < rows; ++i) v[i - k] = R[k * rows + i];
        v[0] -= alpha;
        double vv = 0.0;
        for (double t : v) vv += t * t;
        if (vv == 0.0) continue;
        for (int j = k; j < cols; ++j) {
            double d = 0.0;
            for (int i = k; i < rows; ++i) d += v[i - k] * R[j * rows + i];
            d = 2.0 * d / vv;
            for (int i = k; i < rows; ++i) R[j * rows + i] -= d * v[i - k];
        }
        double d = 0.0;
        for (int i = k; i < rows; ++i) d += v[i - k] * e[i];
        d = 2.0 * d / vv;
        for (int i = k; i < rows; ++i) e[i] -= d * v[i - k];
    }
    std::vector<double> y(cols, 0.0);
    for (int k = cols - 1; k >= 0; --k) {
        double s = e[k];
        for (int j = k + 1; j < cols; ++j) s -= R[j * rows + k] * y[j];
        y[k] = R[k * rows + k] != 0.0 ? s / R[k * rows + k] : 0.0;
    }
    return y;
}

// ------------------------------------------------------------------ host helpers
using cplx = std::complex<double>;

// Eigenvalues of the k x k upper Hessenberg matrix A (column-major, leading dimension
// k; overwritten) by the shifted QR algorithm in complex arithmetic: a Wilkinson
// shift from the trailing 2 x 2 block of the active part, one QR step as Givens
// rotations of neighbouring rows followed by their adjoints from the right, and
// deflation where a subdiagonal entry is negligible against its diagonal neighbours.
// Returns false if one eigenvalue takes more than 64 steps.
bool hessenberg_eigenvalues(std::vector<cplx>& A, int k, std::vector<cplx>& ev) {
    auto at = [&](int i, int j) -> cplx& { return A[(size_t)j * k + i]; };
    const double eps = std::numeric_limits<double>::epsilon();
    ev.assign(k, cplx(0.0, 0.0));
    std::vector<cplx> cs(k), sn(k);
    int hi = k - 1, steps = 0;
    while (hi >= 0) {
        int lo = hi;
        for (; lo > 0; --lo) {
            const double scale = std::abs(at(lo - 1, lo - 1)) + std::abs(at(lo, lo));
            if (std::abs(at(lo, lo - 1)) <= eps * (scale > 0.0 ? scale : 1.0)) {
                at(lo, lo - 1) = 0.0;
                break;
            }
        }
        if (lo == hi) {  // a 1 x 1 block: an eigenvalue
            ev[hi] = at(hi, hi);
            --hi;
            steps = 0;
            continue;
        }
        if (++steps > 64) return false;
        const cplx a = at(hi - 1, hi - 1), b = at(hi - 1, hi), c = at(hi, hi - 1), d = at(hi, hi);
        const cplx half = 0.5 * (a + d), disc = std::sqrt(half * half - (a * d - b * c));
        cplx mu = std::abs(half + disc - d) < std::abs(half - disc - d) ? half + disc : half - disc;
        if (steps % 11 == 10) mu = d + std::abs(c);  // an exceptional shift breaks a cycle
        for (int j = lo; j <= hi; ++j) at(j, j) -= mu;
        for (int j = lo; j < hi; ++j) {  // R = G_{hi-1} ... G_lo (A - mu I)
            const cplx x = at(j, j), y = at(j + 1, j);
            const double r = std::hypot(std::abs(x), std::abs(y));
            const cplx c_ = r > 0.0 ? x / r : cplx(1.0, 0.0), s_ = r > 0.0 ? y / r : cplx(0.0, 0.0);
            for (int col = j; col <= hi; ++col) {
                const cplx u = at(j, col), v = at(j + 1, col);
                at(j, col) = std::conj(c_) * u + std::conj(s_) * v;
                at(j + 1, col) = -s_ * u + c_ * v;
            }
            cs[j] = c_;
            sn[j] = s_;
        }
        for (int j = lo; j < hi; ++j)  // R G_lo^H ... G_{hi-1}^H
            for (int row = lo; row <= j + 1; ++row) {
                const cplx u = at(row, j), v = at(row, j + 1);
                at(row, j) = u * cs[j] + v * sn[j];
                at(row, j + 1) = -u * std::conj(sn[j]) + v * std::conj(cs[j]);
            }
        for (int j = lo; j <= hi; ++j) at(j, j) += mu;
    }
    return true;
}

// Leja order (reading R18): the largest modulus first, then each point maximising the
// product of its distances to those already taken; ties to the lowest index.
std::vector<double> leja(const std::vector<double>& pts) {
    std::vector<double> out;
    std::vector<bool> used(pts.size(), false);
    for (size_t t = 0; t < pts.size(); ++t) {
        int best = -1;
        double best_val = -1.0;
        for (size_t i = 0; i < pts.size(); ++i) {
            if (used[i]) continue;
            double v = 1.0;
            if (t == 0)
                v = std::fabs(pts[i]);
            else
                for (double z : out) v *= std::fabs(pts[i] - z);
            if (v > best_val) {
                best = (int)i;
                best_val = v;
            }
        }
        used[best] = true;
        out.push_back(pts[best]);
    }
    return out;
}

struct Solver {
    mpk_plan_t hi, lo;
    int32_t n;
    int s, m, degree;
    double theta, delta, tcheb;
    uint32_t poly_flags;
    int precond;                         // MPK_PRECOND_*
    Layout L;
    double* base;
    hipStream_t st;
    std::vector<double> coef;            // s(A) in T_k((A - theta I)/delta), k < degree
    std::vector<double> lam, sig;        // Newton shifts, Leja order, and scalings
    std::vector<double> host_c[4];       // coefficient staging (rewritten only after a sync)

    double* vec(size_t off) const { return base + off; }
    double* Q(int j) const { return base + L.q + (size_t)j * L.ld; }
    double* W(int k) const { return base + L.w + (size_t)(k + 1) * L.ld; }  // W_{k+1}
    double* V0() const { return base + L.w; }                               // W_0 (a copy)

    mpk_status hip(hipError_t e, const char* what) {
        if (e == hipSuccess) return MPK_OK;
        return mpk::set_error(MPK_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    }

    // out (a x b, row-major a-major: out[j*b + k]) = X^T Y over the first n rows
    mpk_status gram(const double* X, int a, const double* Y, int b, std::vector<double>& out) {
        const bool one = a == 1 && b == 1;
        const int JB = one ? 1 : 8, KB = one ? 1 : 8;
        const int ntj = (a + JB - 1) / JB, ntk = (b + KB - 1) / KB;
        const int grid = ((L.nrb + 7) / 8) * 8 * ntj * ntk;
        double* part = vec(L.part);
        if (one)
            hipLaunchKernelGGL((gram_partial_kernel<1, 1>), dim3(grid), dim3(kThreads), 0, st, X, L.ld, a, Y, L.ld, b,
                               n, L.rows_per_blk, L.nrb, ntj, ntk, part);
        else
            hipLaunchKernelGGL((gram_partial_kernel<8, 8>), dim3(grid), dim3(kThreads), 0, st, X, L.ld, a, Y, L.ld, b,
                               n, L.rows_per_blk, L.nrb, ntj, ntk, part);
        mpk_status s_ = hip(hipGetLastError(), "gram launch");
        if (s_ != MPK_OK) return s_;
        const int count = a * b;
        hipLaunchKernelGGL(reduce_parts_kernel, dim3(count), dim3(kThreads), 0, st, part, L.nrb, vec(L.small));
        s_ = hip(hipGetLastError(), "reduce launch");
        if (s_ != MPK_OK) return s_;
        out.assign(count, 0.0);
        s_ = hip(hipMemcpyAsync(out.data(), vec(L.small), count * sizeof(double), hipMemcpyDeviceToHost, st),
                 "copy Gram");
        if (s_ == MPK_OK) s_ = hip(hipStreamSynchronize(st), "synchronize");
        return s_;
    }

    // Y[k] = alpha X0[k] + sum_j Q_[j] C[j b + k] with C from host; `slot` picks the
    // staging buffer (each is rewritten only after a later synchronisation)
    mpk_status lincomb(const double* X0, double alpha, const double* Qv, int a, const std::vector<double>& C, int b,
                       double* Y, int slot) {
        host_c[slot] = C;
        double* dc = vec(L.cbuf) + (size_t)slot * kMaxC;
        mpk_status s_ = hip(hipMemcpyAsync(dc, host_c[slot].data(), (size_t)a * b * sizeof(double),
                                           hipMemcpyHostToDevice, st),
                            "copy coefficients");
        if (s_ != MPK_OK) return s_;
        if (b <= 1)
            hipLaunchKernelGGL(lincomb_kernel<1>, dim3(grid_rows(n)), dim3(kThreads), 0, st, X0, L.ld, alpha, Qv, L.ld,
                               a, dc, b, Y, L.ld, n);
        else if (b <= 8)
            hipLaunchKernelGGL(lincomb_kernel<8>, dim3(grid_rows(n)), dim3(kThreads), 0, st, X0, L.ld, alpha, Qv, L.ld,
                               a, dc, b, Y, L.ld, n);
        else
            hipLaunchKernelGGL(lincomb_kernel<16>, dim3(grid_rows(n)), dim3(kThreads), 0, st, X0, L.ld, alpha, Qv,
                               L.ld, a, dc, b, Y, L.ld, n);
        return hip(hipGetLastError(), "lincomb launch");
    }

    // out = (M - lambda I) in / sigma, M = I - T_d((theta I - A)/delta) / T_d(theta/delta)
    mpk_status newton_step(const double* in, double* out, double lambda, double sigma) {
        std::vector<double> c(degree + 1, 0.0);
        c[0] = (1.0 - lambda) / sigma;
        c[degree] += -((degree % 2) ? -1.0 : 1.0) / (tcheb * sigma);
        const double params[2] = {theta, delta};
        return poly_apply(lo, MPK_POLY_CHEBYSHEV, degree, c.data(), params, in, out, poly_flags, vec(L.poly),
                          L.poly_bytes, st);
    }

    // out = M in for the block operator without a shift (A, A D^{-1}, the k-sweep Jacobi
    // or the GS2 operator A P^{-1}), on `lo`
    mpk_status apply_M(const double* in, double* out) {
        if (precond == MPK_PRECOND_GS2)
            return mpk::gs2_chain(lo, degree, in, out, L.ld, 1, nullptr, nullptr, 0, poly_flags, vec(L.poly),
                                  L.poly_bytes, st);
        if (precond == MPK_PRECOND_JACOBI && degree > 1)
            return mpk::jacobi_chain(lo, degree, in, out, L.ld, 1, nullptr, nullptr, poly_flags, vec(L.poly),
                                     L.poly_bytes, st);
        return mpk_apply(lo, in, out, L.ld, 1, poly_flags, nullptr, 0, st);
    }

    // Reading R24: Newton shifts from Ritz values.  s steps of standard Arnoldi on M
    // from Q_0 (classical Gram-Schmidt with one reorthogonalisation), writing Q_1.. and
    // stopping when a new vector's norm is at most 2^-48 of ||M q_j|| (an invariant
    // space); the eigenvalues of the square Hessenberg matrix; their real parts in Leja
    // order, repeated cyclically up to s; columns scaled by a quarter of the spread.
    mpk_status ritz_shifts() {
        const int ldh = s + 1;
        std::vector<double> H((size_t)ldh * s, 0.0), g, h, h2;
        int k = s;
        for (int j = 0; j < s; ++j) {
            double* w = W(0);
            mpk_status e = apply_M(Q(j), w);
            if (e == MPK_OK) e = gram(w, 1, w, 1, g);
            if (e != MPK_OK) return e;
            const double wn = std::sqrt(g[0]);
            for (int pass = 0; pass < 2; ++pass) {  // w -= Q_{0..j} (Q^T w), twice
                e = gram(Q(0), j + 1, w, 1, pass == 0 ? h : h2);
                if (e != MPK_OK) return e;
                const std::vector<double>& hp = pass == 0 ? h : h2;
                std::vector<double> neg(j + 1);
                for (int i = 0; i <= j; ++i) {
                    neg[i] = -hp[i];
                    H[(size_t)j * ldh + i] += hp[i];
                }
                e = lincomb(w, 1.0, Q(0), j + 1, neg, 1, w, pass);
                if (e != MPK_OK) return e;
            }
            e = gram(w, 1, w, 1, g);
            if (e != MPK_OK) return e;
            const double nrm = std::sqrt(g[0]);
            if (!(nrm > std::ldexp(1.0, -48) * wn)) {
                k = j + 1;
                break;
            }
            H[(size_t)j * ldh + j + 1] = nrm;
            e = lincomb(nullptr, 0.0, w, 1, std::vector<double>{1.0 / nrm}, 1, Q(j + 1), 2);
            if (e != MPK_OK) return e;
        }
        std::vector<cplx> Hk((size_t)k * k), ev;
        for (int j = 0; j < k; ++j)
            for (int i = 0; i <= std::min(j + 1, k - 1); ++i) Hk[(size_t)j * k + i] = H[(size_t)j * ldh + i];
        if (!hessenberg_eigenvalues(Hk, k, ev))
            return mpk::set_error(MPK_ERR_UNSUPPORTED, "Ritz values: the QR iteration did not converge");
        std::vector<double> re(k);
        for (int i = 0; i < k; ++i) re[i] = ev[i].real();
        const std::vector<double> order = leja(re);
        lam.assign(s, 0.0);
        for (int i = 0; i < s; ++i) lam[i] = order[i % k];
        const auto mm = std::minmax_element(lam.begin(), lam.end());
        const double spread = *mm.second - *mm.first;
        sig.assign(s, spread > 0.0 ? 0.25 * spread : (lam[0] != 0.0 ? std::fabs(lam[0]) : 1.0));
        return MPK_OK;
    }

    // out = s(A) in
    mpk_status precondition(const double* in, double* out) {
        const double params[2] = {theta, delta};
        return poly_apply(lo, MPK_POLY_CHEBYSHEV, degree - 1, coef.data(), params, in, out, poly_flags, vec(L.poly),
                          L.poly_bytes, st);
    }

    // r = b - A x into Q_0 with FP64 values; returns ||r||^2
    mpk_status residual(const double* b, const double* x, double* rr) {
        mpk_status s_ = mpk_apply(hi, x, vec(L.t), n, 1, MPK_IO_PERMUTED, nullptr, 0, st);
        if (s_ != MPK_OK) return s_;
        hipLaunchKernelGGL(sub_kernel, dim3(grid_rows(n)), dim3(kThreads), 0, st, b, (const double*)vec(L.t), Q(0), n);
        s_ = hip(hipGetLastError(), "residual launch");
        if (s_ != MPK_OK) return s_;
        std::vector<double> g;
        s_ = gram(Q(0), 1, Q(0), 1, g);
        if (s_ == MPK_OK) *rr = g[0];
        return s_;
    }

    // One restart cycle from Q_0 = r / beta; adds s(A) Q y to x.  Returns the number of
    // Hessenberg columns built.
    mpk_status cycle(double beta, double target, double* x, int* cols_out) {
        std::vector<double> H;  // column-major, leading dimension m + 1
        const int ldh = m + 1;
        H.assign((size_t)ldh * m, 0.0);
        int c = 0;
        std::vector<double> rprev, G;
        for (;;) {
            const int sb = std::min(s, m - c);
            // Newton basis of the block (Sec. 4): W_k = (M - lambda_k I) W_{k-1} / sigma_k,
            // with the Chebyshev preconditioner one polynomial launch sequence per vector,
            // otherwise one blocked MPK of sb powers for the whole block (Alg. 3c)
            if (precond == MPK_PRECOND_CHEBYSHEV) {
                for (int k = 1; k <= sb; ++k) {
                    mpk_status s_ = newton_step(k == 1 ? Q(c) : W(k - 2), W(k - 1), lam[k - 1], sig[k - 1]);
                    if (s_ != MPK_OK) return s_;
                }
            } else if (precond == MPK_PRECOND_GS2) {  // one GS2 chain of sb powers, shifts at the closings
                mpk_status s_ = mpk::gs2_chain(lo, degree, Q(c), W(0), L.ld, sb, lam.data(), sig.data(), 0, poly_flags,
                                               vec(L.poly), L.poly_bytes, st);
                if (s_ != MPK_OK) return s_;
            } else if (precond == MPK_PRECOND_JACOBI && degree > 1) {  // one Jacobi chain of sb powers
                mpk_status s_ = mpk::jacobi_chain(lo, degree, Q(c), W(0), L.ld, sb, lam.data(), sig.data(), poly_flags,
                                                  vec(L.poly), L.poly_bytes, st);
                if (s_ != MPK_OK) return s_;
            } else {
                mpk_status s_ = sstep_basis(lo, sb, lam.data(), sig.data(), Q(c), V0(), L.ld, poly_flags, nullptr, 0,
                                            st);
                if (s_ != MPK_OK) return s_;
            }
            // BOrtho: R_prev = Q_{0..c}^T W, W' = W - Q R_prev
            mpk_status s_ = gram(Q(0), c + 1, W(0), sb, rprev);
            if (s_ != MPK_OK) return s_;
            std::vector<double> neg(rprev.size());
            for (size_t e = 0; e < rprev.size(); ++e) neg[e] = -rprev[e];
            s_ = lincomb(W(0), 1.0, Q(0), c + 1, neg, sb, W(0), 0);
            if (s_ != MPK_OK) return s_;
            // TSQR by Cholesky QR: G = W'^T W' = R^T R, truncated at a dependent column
            s_ = gram(W(0), sb, W(0), sb, G);
            if (s_ != MPK_OK) return s_;
            std::vector<double> R((size_t)sb * sb, 0.0);  // R[i*sb + j], upper
            int kk = sb;
            for (int j = 0; j < sb; ++j) {
                for (int i = 0; i < j; ++i) {
                    double t = G[i * sb + j];
                    for (int l = 0; l < i; ++l) t -= R[l * sb + i] * R[l * sb + j];
                    R[i * sb + j] = t / R[i * sb + i];
                }
                double piv2 = G[j * sb + j];
                for (int l = 0; l < j; ++l) piv2 -= R[l * sb + j] * R[l * sb + j];
                double wn2 = G[j * sb + j];
                for (int i = 0; i <= c; ++i) wn2 += rprev[i * sb + j] * rprev[i * sb + j];
                if (!(std::isfinite(piv2) && piv2 > kEta * kEta * wn2)) {
                    kk = j;
                    break;
                }
                R[j * sb + j] = std::sqrt(piv2);
            }
            const bool dep = kk < sb;
            if (kk > 0) {  // Q_{c+1..c+kk} = W'[:, :kk] R[:kk, :kk]^{-1}
                std::vector<double> Rinv((size_t)kk * kk, 0.0);
                for (int j = 0; j < kk; ++j) {
                    Rinv[j * kk + j] = 1.0 / R[j * sb + j];
                    for (int i = j - 1; i >= 0; --i) {
                        double t = 0.0;
                        for (int l = i + 1; l <= j; ++l) t += R[i * sb + l] * Rinv[l * kk + j];
                        Rinv[i * kk + j] = -t / R[i * sb + i];
                    }
                }
                s_ = lincomb(nullptr, 0.0, W(0), kk, Rinv, kk, Q(c + 1), 1);
                if (s_ != MPK_OK) return s_;
            }
            // Hessenberg columns c .. c + nh - 1 from M W_{0..nh-1} = W_{0..nh} B and
            // W_{0..nh} = Q_{0..rows-1} Rfull
            const int nh = kk + (dep ? 1 : 0), rows = c + kk + 1;
            std::vector<double> Rfull((size_t)rows * (nh + 1), 0.0);  // column-major, ld rows
            Rfull[c] = 1.0;
            for (int i = 1; i <= nh; ++i) {
                for (int r = 0; r <= c; ++r) Rfull[(size_t)i * rows + r] = rprev[r * sb + (i - 1)];
                const int top = std::min(i, kk);
                for (int r = 0; r < top; ++r) Rfull[(size_t)i * rows + c + 1 + r] = R[r * sb + (i - 1)];
            }
            std::vector<double> rhs((size_t)rows * nh, 0.0);  // Rfull B - [H_old Rk_top; 0]
            for (int col = 0; col < nh; ++col)
                for (int r = 0; r < rows; ++r)
                    rhs[(size_t)col * rows + r] =
                        Rfull[(size_t)col * rows + r] * lam[col] + Rfull[(size_t)(col + 1) * rows + r] * sig[col];
            if (c > 0)
                for (int col = 0; col < nh; ++col)
                    for (int r = 0; r <= c; ++r) {
                        double t = 0.0;
                        for (int l = 0; l < c; ++l) t += H[(size_t)l * ldh + r] * Rfull[(size_t)col * rows + l];
                        rhs[(size_t)col * rows + r] -= t;
                    }
            // X Rk_bot = rhs with Rk_bot = Rfull[c .. c+nh-1, 0 .. nh-1] upper triangular
            for (int r = 0; r < rows; ++r)
                for (int col = 0; col < nh; ++col) {
                    double t = rhs[(size_t)col * rows + r];
                    for (int l = 0; l < col; ++l) t -= H[(size_t)(c + l) * ldh + r] * Rfull[(size_t)col * rows + c + l];
                    H[(size_t)(c + col) * ldh + r] = t / Rfull[(size_t)col * rows + c + col];
                }
            c += nh;
            // least squares min ||beta e_0 - H y|| and its residual (Alg. 3c's check)
            const int hr = rows;
            std::vector<double> Hc((size_t)hr * c), e(hr, 0.0);
            for (int col = 0; col < c; ++col)
                for (int r = 0; r < hr; ++r) Hc[(size_t)col * hr + r] = H[(size_t)col * ldh + r];
            e[0] = beta;
            std::vector<double> y = least_squares(Hc, hr, c, e);
            double rho2 = 0.0;
            for (int r = 0; r < hr; ++r) {
                double t = e[r];
                for (int col = 0; col < c; ++col) t -= Hc[(size_t)col * hr + r] * y[col];
                rho2 += t * t;
            }
            if (dep || c >= m || std::sqrt(rho2) <= target) {
                // x += P^{-1} Q_{0..c-1} y with P^{-1} = s(A), I or D^{-1}
                if (c > 0 && precond == MPK_PRECOND_NONE) {
                    s_ = lincomb(x, 1.0, Q(0), c, y, 1, x, 2);
                    if (s_ != MPK_OK) return s_;
                } else if (c > 0) {
                    s_ = lincomb(nullptr, 0.0, Q(0), c, y, 1, vec(L.z), 2);
                    if (s_ != MPK_OK) return s_;
                    if (precond == MPK_PRECOND_GS2) {  // t = P^{-1} z, x += t
                        s_ = mpk::gs2_chain(lo, degree, vec(L.z), vec(L.t), L.ld, 1, nullptr, nullptr, 1, poly_flags,
                                            vec(L.poly), L.poly_bytes, st);
                        if (s_ != MPK_OK) return s_;
                        s_ = lincomb(x, 1.0, vec(L.t), 1, std::vector<double>{1.0}, 1, x, 3);
                        if (s_ != MPK_OK) return s_;
                    } else if (precond == MPK_PRECOND_JACOBI) {
                        // P^{-1} z = D^{-1} sum_{i<k} (I - B)^i z: a Newton polynomial in B with all
                        // shifts 1 and coefficients (-1)^i, then the diagonal
                        const double* zk = vec(L.z);
                        if (degree > 1) {
                            std::vector<double> c(degree), ones(degree - 1, 1.0);
                            for (int i = 0; i < degree; ++i) c[i] = (i % 2) ? -1.0 : 1.0;
                            s_ = poly_apply(lo, MPK_POLY_NEWTON, degree - 1, c.data(), ones.data(), vec(L.z),
                                            vec(L.t), poly_flags, vec(L.poly), L.poly_bytes, st);
                            if (s_ != MPK_OK) return s_;
                            zk = vec(L.t);
                        }
                        hipLaunchKernelGGL(add_div_kernel, dim3(grid_rows(n)), dim3(kThreads), 0, st, x, zk,
                                           (const double*)vec(L.diag), n);
                        s_ = hip(hipGetLastError(), "update launch");
                        if (s_ != MPK_OK) return s_;
                    } else {
                        s_ = precondition(vec(L.z), vec(L.t));
                        if (s_ != MPK_OK) return s_;
                        s_ = lincomb(x, 1.0, vec(L.t), 1, std::vector<double>{1.0}, 1, x, 3);
                        if (s_ != MPK_OK) return s_;
                    }
                }
                *cols_out = c;
                return MPK_OK;
            }
        }
    }
};

bool params_ok(int32_t s, int32_t m, int32_t degree) {
    return s >= 1 && s <= kMaxS && m >= s && m <= kMaxM && degree >= 0 && degree <= 4096;
}

// Bytes of the polynomial ring: the Chebyshev ring of poly_apply, or for a plan with
// lower-triangle masks (the GS2 preconditioner, degree = gamma) the GS2 ring.
mpk_status ring_bytes(mpk_plan_t lo, int32_t degree, size_t* bytes) {
    size_t pb = 0;
    mpk_status st = mpk_work_bytes(lo, MPK_CALL_POLY, std::max(degree, 1), MPK_IO_PERMUTED, &pb);
    if (st != MPK_OK) return st;
    if (mpk::plan_split_lower(lo)) {
        int64_t n = 0;
        st = mpk_plan_info(lo, &n, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
        if (st != MPK_OK) return st;
        const size_t gs2 = (size_t)(mpk::plan_p_block(lo) + std::min(degree, 16) + 2) * ((n + 31) / 32 * 32) * 8;
        pb = std::max(pb, gs2);
    }
    *bytes = pb;
    return MPK_OK;
}

}  // namespace

MPK_API mpk_status mpk_sstep_gmres_work_bytes(mpk_plan_t lo, int32_t s, int32_t m, int32_t degree, uint32_t flags,
                                              size_t* bytes) {
    if (!lo || !bytes) return mpk::set_error(MPK_ERR_ARG, "null argument");
    if (!params_ok(s, m, degree))
        return mpk::set_error(MPK_ERR_ARG, "need 1 <= s <= %d, s <= m <= %d, 1 <= degree <= 4096", kMaxS, kMaxM);
    int64_t n = 0;
    mpk_status st = mpk_plan_info(lo, &n, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    if (st != MPK_OK) return st;
    size_t pb = 0;
    st = ring_bytes(lo, degree, &pb);
    if (st != MPK_OK) return st;
    *bytes = layout(n, s, m, pb, flags & MPK_IO_PERMUTED).total;
    return MPK_OK;
}

MPK_API mpk_status mpk_sstep_gmres_ex(mpk_plan_t hi, mpk_plan_t lo, int32_t precond, int32_t s, int32_t m,
                                      int32_t degree, double lmin, double lmax, const double* b, double* x,
                                      double tol, int32_t max_cycles, uint32_t flags, void* work, size_t work_bytes,
                                      int32_t* iters_out, int32_t* cycles_out, double* relres_out, void* stream) {
    if (iters_out) *iters_out = 0;
    if (cycles_out) *cycles_out = 0;
    if (relres_out) *relres_out = 0.0;
    if (!hi || !lo) return mpk::set_error(MPK_ERR_ARG, "null plan");
    if (precond < MPK_PRECOND_CHEBYSHEV || precond > MPK_PRECOND_GS2)
        return mpk::set_error(MPK_ERR_ARG, "unknown preconditioner %d", precond);
    if (!mpk::plan_is_f64(hi) || mpk::plan_column_scaling(hi) != MPK_SCALE_NONE)
        return mpk::set_error(MPK_ERR_ARG, "hi must store the FP64 values of A");
    if (!mpk::plans_match(hi, lo))
        return mpk::set_error(MPK_ERR_ARG, "hi and lo must be plans of the same matrix with the same level order");
    if (mpk::plan_column_scaling(lo) != (precond == MPK_PRECOND_JACOBI ? MPK_SCALE_JACOBI : MPK_SCALE_NONE))
        return mpk::set_error(MPK_ERR_ARG, precond == MPK_PRECOND_JACOBI
                                               ? "lo must hold A D^{-1} (column_scaling = MPK_SCALE_JACOBI)"
                                               : "lo must hold A (column_scaling = MPK_SCALE_NONE)");
    if (!params_ok(s, m, degree) || (precond == MPK_PRECOND_CHEBYSHEV && degree < 1) ||
        (precond == MPK_PRECOND_GS2 && degree > 16) ||
        (precond == MPK_PRECOND_JACOBI && (degree < 1 || degree > 64)))
        return mpk::set_error(MPK_ERR_ARG, "need 1 <= s <= %d, s <= m <= %d, 1 <= degree <= 4096 (0 <= gamma <= 16 "
                                           "for GS2, 1 <= k <= 64 for Jacobi)", kMaxS, kMaxM);
    if (precond == MPK_PRECOND_GS2 && !mpk::plan_split_lower(lo))
        return mpk::set_error(MPK_ERR_ARG, "lo must be built with split_lower for the GS2 preconditioner");
    const bool ritz = flags & MPK_RITZ_SHIFTS;
    if (ritz && precond == MPK_PRECOND_CHEBYSHEV)
        return mpk::set_error(MPK_ERR_ARG, "MPK_RITZ_SHIFTS needs MPK_PRECOND_NONE, _JACOBI or _GS2");
    if (precond == MPK_PRECOND_CHEBYSHEV && !(lmin > 0.0))
        return mpk::set_error(MPK_ERR_ARG, "need 0 < lmin < lmax");
    if (!ritz && !(lmax > lmin)) return mpk::set_error(MPK_ERR_ARG, "need lmin < lmax");
    if (!(tol >= 0.0)) return mpk::set_error(MPK_ERR_ARG, "tol must be >= 0");
    if (max_cycles < 0) return mpk::set_error(MPK_ERR_ARG, "max_cycles must be >= 0");
    if (flags & ~(MPK_IO_PERMUTED | MPK_PLAIN | MPK_STAGED | MPK_RITZ_SHIFTS))
        return mpk::set_error(MPK_ERR_ARG, "unknown flag bits");
    int64_t n64 = 0;
    mpk_status st = mpk_plan_info(hi, &n64, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    if (st != MPK_OK) return st;
    if (n64 > 0 && (!b || !x)) return mpk::set_error(MPK_ERR_ARG, "b or x is null");
    size_t need = 0;
    st = mpk_sstep_gmres_work_bytes(lo, s, m, degree, flags, &need);
    if (st != MPK_OK) return st;
    if (!work || work_bytes < need)
        return mpk::set_error(MPK_ERR_ARG, "work buffer too small: %zu < %zu bytes", work_bytes, need);
    if (((uintptr_t)work) % 256) return mpk::set_error(MPK_ERR_ARG, "work must be 256-byte aligned");
    st = mpk::plan_uploaded(hi);
    if (st == MPK_OK) st = mpk::plan_uploaded(lo);
    if (st != MPK_OK) return st;
    if (n64 == 0) return MPK_OK;
    try {
        Solver S;
        S.hi = hi;
        S.lo = lo;
        S.n = (int32_t)n64;
        S.s = s;
        S.m = m;
        S.degree = degree;
        S.theta = 0.5 * (lmax + lmin);
        S.delta = 0.5 * (lmax - lmin);
        S.tcheb = precond == MPK_PRECOND_CHEBYSHEV ? std::cosh(degree * std::acosh(S.theta / S.delta)) : 1.0;
        S.poly_flags = MPK_IO_PERMUTED | (flags & (MPK_PLAIN | MPK_STAGED));
        S.precond = precond;
        size_t pb = 0;
        ring_bytes(lo, degree, &pb);
        const bool permuted = flags & MPK_IO_PERMUTED;
        S.L = layout(n64, s, m, pb, permuted);
        S.base = (double*)work;
        S.st = (hipStream_t)stream;
        // s: the Chebyshev interpolant of 1/lambda at the zeros of T_d (its residual
        // polynomial is T_d((theta - lambda)/delta) / T_d(theta/delta))
        S.coef.assign(std::max(degree, 1), 0.0);
        for (int j = 0; precond == MPK_PRECOND_CHEBYSHEV && j < degree; ++j) {
            const double ang = 3.14159265358979323846 * (j + 0.5) / degree;
            const double inv = 1.0 / (S.theta + S.delta * std::cos(ang));
            for (int k = 0; k < degree; ++k) S.coef[k] += std::cos(k * ang) * inv;
        }
        for (int k = 0; k < degree; ++k) S.coef[k] *= (k == 0 ? 1.0 : 2.0) / degree;
        // Newton shifts: the s Chebyshev points of the interval holding M's spectrum in Leja
        // order, columns scaled by half its half-width: [1 - eps, 1 + eps] with the Chebyshev
        // preconditioner (A's spectrum in [lmin, lmax]), else [lmin, lmax] itself
        const double eps = precond == MPK_PRECOND_CHEBYSHEV ? 1.0 / S.tcheb : 0.5 * (lmax - lmin);
        const double mid = precond == MPK_PRECOND_CHEBYSHEV ? 1.0 : 0.5 * (lmax + lmin);
        std::vector<double> pts(s);
        for (int i = 0; i < s; ++i) pts[i] = mid + eps * std::cos(3.14159265358979323846 * (2 * i + 1) / (2.0 * s));
        S.lam = leja(pts);
        S.sig.assign(s, 0.5 * eps);
        // level-order copies of b and x when the caller's vectors are in original order
        const double* bp = b;
        double* xp = x;
        if (!permuted) {
            double* io = S.vec(S.L.io);
            st = mpk_permute(hi, b, io, 0, stream);
            if (st == MPK_OK) st = mpk_permute(hi, x, io + S.L.ld, 0, stream);
            if (st != MPK_OK) return st;
            bp = io;
            xp = io + S.L.ld;
        }
        if (precond == MPK_PRECOND_JACOBI) {  // D in level order, from the FP64 plan
            st = mpk::plan_diagonal(hi, S.vec(S.L.diag), stream);
            if (st != MPK_OK) return st;
        }
        std::vector<double> g;
        st = S.gram(bp, 1, bp, 1, g);
        if (st != MPK_OK) return st;
        const double nb = std::sqrt(g[0]);
        int iters = 0, cyc = 0;
        double rel = 0.0;
        for (;; ++cyc) {
            double rr = 0.0;
            st = S.residual(bp, xp, &rr);
            if (st != MPK_OK) return st;
            const double beta = std::sqrt(rr);
            rel = nb > 0.0 ? beta / nb : beta;
            if (rel <= tol || cyc == max_cycles || beta == 0.0) break;
            std::vector<double> inv{1.0 / beta};
            st = S.lincomb(nullptr, 0.0, S.Q(0), 1, inv, 1, S.Q(0), 0);
            if (st != MPK_OK) return st;
            if (ritz && cyc == 0) {  // shifts from the first cycle's Arnoldi steps (R24)
                st = S.ritz_shifts();
                if (st != MPK_OK) return st;
            }
            int cols = 0;
            st = S.cycle(beta, tol * nb, xp, &cols);
            if (st != MPK_OK) return st;
            iters += cols;
        }
        if (!permuted) {
            st = mpk_permute(hi, xp, x, 1, stream);
            if (st != MPK_OK) return st;
        }
        // the coefficient staging vectors of the last copies are freed on return
        st = S.hip(hipStreamSynchronize(S.st), "synchronize");
        if (st != MPK_OK) return st;
        if (iters_out) *iters_out = iters;
        if (cycles_out) *cycles_out = cyc;
        if (relres_out) *relres_out = rel;
        return MPK_OK;
    } catch (const std::bad_alloc&) {
        return mpk::set_error(MPK_ERR_NOMEM, "out of host memory");
    }
}

MPK_API mpk_status mpk_ritz_values(const double* H, int64_t ldh, int32_t k, double* re, double* im) {
    if (k < 0 || k > 512) return mpk::set_error(MPK_ERR_ARG, "k must be in 0..512 (got %d)", k);
    if (k == 0) return MPK_OK;
    if (!H || !re || !im) return mpk::set_error(MPK_ERR_ARG, "null argument");
    if (ldh < k) return mpk::set_error(MPK_ERR_ARG, "ldh must be >= k");
    try {
        std::vector<cplx> A((size_t)k * k), ev;
        for (int j = 0; j < k; ++j)
            for (int i = 0; i <= std::min(j + 1, k - 1); ++i) A[(size_t)j * k + i] = H[(size_t)j * ldh + i];
        if (!hessenberg_eigenvalues(A, k, ev))
            return mpk::set_error(MPK_ERR_UNSUPPORTED, "the QR iteration did not converge");
        for (int i = 0; i < k; ++i) {
            re[i] = ev[i].real();
            im[i] = ev[i].imag();
        }
    } catch (const std::bad_alloc&) {
        return mpk::set_error(MPK_ERR_NOMEM, "out of host memory");
    }
    return MPK_OK;
}

MPK_API mpk_status mpk_sstep_gmres(mpk_plan_t hi, mpk_plan_t lo, int32_t s, int32_t m, int32_t degree, double lmin,
                                   double lmax, const double* b, double* x, double tol, int32_t max_cycles,
                                   uint32_t flags, void* work, size_t work_bytes, int32_t* iters_out,
                                   int32_t* cycles_out, double* relres_out, void* stream) {
    return mpk_sstep_gmres_ex(hi, lo, MPK_PRECOND_CHEBYSHEV, s, m, degree, lmin, lmax, b, x, tol, max_cycles, flags,
                              work, work_bytes, iters_out, cycles_out, relres_out, stream);
}
