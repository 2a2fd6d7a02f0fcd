"""FP64 CPU oracle for the matrix power kernel (MPK) -- TEST INFRASTRUCTURE ONLY.

Plain, single-threaded NumPy (plus pure-Python loops for tiny cases).  Only
``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may use it.  It shares no code with the HIP path.

Matrices are ``(n, rowptr, col, val)`` CSR tuples (0-based, columns sorted
and unique within a row), vectors are float64 NumPy arrays.

Parity status
-------------
pinned   spmv, mpk, round_values, round_values_bf16_rowscale, chebyshev_inverse_coeffs,
         refine_solve, newton_basis, poly_monomial, poly_newton, poly_chebyshev,
         leja_order, chebyshev_scale, newton_shifts, cholqr_truncated, sstep_cycle, sstep_gmres,
         diagonal, jacobi_precondition, jacobi_mpk, spmv_lower, gs2_precondition, gs2_mpk,
         gs2_smooth_residual,
         interval_shifts, sstep_gmres_precond, arnoldi, ritz_shifts,
         pattern_graph, bfs_levels, level_permutation, permute_symmetric,
         group_levels, wavefront_schedule, validate_schedule, run_schedule
         (pins: exact integer arithmetic, closed-form Laplacian eigenpairs,
         closed-form grid levels, scipy shortest paths, brute force on tiny
         inputs, special cases; see tests/test_oracle_pins.py)
unpinned the level grouping and the wavefront order (R14, R15) are readings of a
         passage that gives no rule; only their validity (coverage, read-after-write
         order, bitwise equality with the plain MPK) is pinned, not their identity
         with the paper's library.

How the GPU kernel hands out work (chunk ownership, units, the deadlock bound)
is a design choice of the HIP path, not a statement of the paper: it is
modelled on the test side (tests/schedule_model.py), not here.
"""
import math
from collections import deque

import numpy as np

# Readings taken where the paper is silent or garbled.  Each is implemented
# below exactly as stated; the HIP planner implements the same statements
# independently.
READINGS = {
    "R1": "BFS runs on the undirected graph of pattern(A) union pattern(A^T) without "
          "self-loops; explicitly stored zeros count as edges (Sec. 3: levels from "
          "the matrix graph; Sec. 5.1.2: levels come from A alone).",
    "R2": "Root of each connected component: George-Liu pseudo-peripheral node. Start "
          "at the component's lowest-index vertex r; BFS from r; among the last level "
          "take the vertex x of minimum degree (ties: lowest index); BFS from x; if "
          "ecc(x) > ecc(r) set r = x and repeat, else stop at r. An explicit root "
          "replaces this search for the component that contains it.",
    "R3": "Components are processed in order of their lowest vertex index; the levels "
          "of each component continue after the last level of the previous one.",
    "R4": "Within a level, rows keep ascending original index: perm[new] = old, "
          "iperm[old] = new.",
    "R8": "Newton basis: V_k = (A - lambda_k I) V_{k-1} / sigma_k, the product of distinct "
          "shifted factors (the printed powers (A - lambda_2 I)^2 ... are read as this "
          "product).",
    "R9": "Chebyshev polynomial on [theta - delta, theta + delta]: t_0 = x, "
          "t_1 = (A - theta I) x / delta, t_{k+1} = 2 (A - theta I) t_k / delta - t_{k-1}; "
          "result sum_k c_k t_k.",
    "R10": "Powers beyond one block of q are computed as consecutive blocks of q powers "
           "and a last block of the remaining r < q powers, each seeded with the last "
           "vector of the previous block (Sec. 3, p_opt and the remainder loop).",
    "R12": "Chebyshev polynomial preconditioner of degree d on [lmin, lmax] (the degree-d "
           "Chebyshev preconditioner of Sec. 5; the paper gives no formula): the "
           "polynomial s of degree d-1 with 1 - lam s(lam) = T_d((theta - lam)/delta) / "
           "T_d(theta/delta), theta = (lmax + lmin)/2, delta = (lmax - lmin)/2, expanded "
           "as sum_k c_k T_k((lam - theta)/delta) and applied with the recurrence of R9.",
    "R13": "Iterative refinement (beyond the paper, which is FP64 throughout): "
           "r_i = b - A x_i in FP64 with the unrounded matrix; stop when ||r_i|| <= tol "
           "||b||; else x_{i+1} = x_i + s(A~) r_i with s of R12 applied to the matrix "
           "whose values are stored in FP32 (R11).",
    "R14": "Level groups for a cache of C bytes and q powers (Sec. 3: groups from the "
           "level structure and the cache size): w(level) = sum over its rows of "
           "nnz_row * (value bytes + 4) + 4 + 16; budget B = floor(C / q); levels are "
           "taken in order and a new group starts before level l when the current "
           "group is non-empty, w(group) + w(l) > B and the group has at least "
           "min_group_rows rows.",
    "R15": "Wavefront execution of a block of q powers over groups g = [s_g, e_g], "
           "g = 0..G-1: task (k, g) computes power k on levels [lo, hi] with "
           "lo = max(0, s_g - (k - 1)) (0 for g = 0) and hi = e_g - (k - 1) (L - 1 for "
           "g = G - 1), empty when hi < lo, at stage g + k - 1; stages run in order, "
           "G + q - 1 of them.",
    "R16": "BF16 storage with a per-row scale (beyond the paper): a_ij ~ s_i q_ij with "
           "s_i = fl32(max_j |a_ij|) (1 for an all-zero row) and q_ij the BF16 value "
           "nearest (ties to even) to fl32(a_ij / s_i); the product is formed exactly in "
           "FP64 and the MPK is the FP64 MPK of the matrix of those products.",
    "R17": "s-step GMRES (Sec. 4, Alg. 3a/3c) with right polynomial preconditioning "
           "(Sec. 5): operator M = A s(A), s of R12, x = x_0 + s(A) Q y. A restart cycle "
           "starts from r = b - A x, q_0 = r / ||r||, and builds blocks of "
           "sb = min(s, m - c) vectors: Newton basis W_0 = q_c, W_k = (M - lambda_k I) "
           "W_{k-1} / sigma_k; BOrtho is one classical Gram-Schmidt sweep "
           "(R_prev = Q^T W, W' = W - Q R_prev); TSQR is Cholesky QR of W' (G = W'^T W' "
           "= R^T R, Q_new = W' R^{-1}); column j is dependent when its squared pivot is "
           "not above 2^-48 (||R_prev[:, j]||^2 + G_jj), and the block then keeps its "
           "first j columns and ends the cycle with a square Hessenberg matrix (the "
           "Krylov space is invariant to working accuracy). The Hessenberg columns come "
           "from M W_{0..sb-1} = W_{0..sb} B (B bidiagonal: lambda on the diagonal, "
           "sigma below) and the triangular change of basis W = Q R. After each block the "
           "least-squares residual of min ||beta e_0 - H y|| is compared with tol ||b|| "
           "(the convergence check of Alg. 3c); the cycle ends there, at a dependent "
           "column, or after m columns.",
    "R18": "Newton shifts: for A with spectrum in [lmin, lmax], M's spectrum lies in "
           "[1 - eps, 1 + eps], eps = 1 / T_d(theta / delta) (from R12). The paper takes "
           "the shifts from Ritz values of a few standard GMRES steps; here they are the "
           "s Chebyshev points 1 + eps cos(pi (2i + 1) / (2s)) of that interval in Leja "
           "order (first the largest modulus, then the largest product of distances to "
           "the points taken; ties to the lowest index), every column scaled by "
           "sigma = eps / 2, so no Arnoldi run is needed.",
    "R19": "The solve stops when the FP64 residual at the start of a cycle satisfies "
           "||b - A x|| <= tol ||b|| or after max_cycles cycles; with reduced-precision "
           "values (R11) only the basis and the preconditioner use the rounded matrix.",
    "R20": "Jacobi-preconditioned MPK (Sec. 5.1, right preconditioning of Sec. 5): "
           "w_j = A P^{-1} w_{j-1}, P^{-1} v the k-th Jacobi iterate z^k from z^0 = 0 "
           "(k = 1: P^{-1} = D^{-1}, the fused A D^{-1} of the paper; k > 1: the "
           "Neumann-series polynomial preconditioner the paper mentions). The two-stage "
           "Gauss-Seidel preconditioner is not covered.",
    "R21": "Two-stage Gauss-Seidel preconditioner (Sec. 5.1, Alg. 4a): the listing's "
           "superscripts are garbled and its update z^{k+1} = z^k + g_gamma is only "
           "consistent with g_0 = D^{-1}(v - U z^k) when z^k = 0; the paper states that "
           "one outer iteration from z^0 = 0 is the common use and that it then reduces to "
           "g_0 = D^{-1} v and z^1 = g_gamma. That is the form taken: g_j = g_0 - D^{-1} L "
           "g_{j-1}, j = 1..gamma, P^{-1} v = g_gamma, with L the strictly lower triangle "
           "in the original numbering; the MPK is w_j = A P^{-1} w_{j-1}.",
    "R22": "s-step GMRES without a preconditioner (M = A), with the diagonal Jacobi "
           "preconditioner from the right (M = A D^{-1}, x = x0 + D^{-1} Q y), or with GS2 "
           "(M = A P^{-1} of R21, x = x0 + P^{-1} Q y; Sec. 4 and 5.1): "
           "each block of s basis vectors is one Newton MPK of s powers (Alg. 3c's "
           "back-to-back SpMVs replaced by an MPK). The shifts are the s Chebyshev points of "
           "a caller-given interval [lmin, lmax] holding M's spectrum, in Leja order, each "
           "column scaled by (lmax - lmin)/4; the paper takes Ritz values instead.",
    "R11": "Reduced-precision matrix storage (the paper works in FP64 only): each stored "
           "value is rounded once to the nearest FP32 value (ties to even); vectors, "
           "products and sums stay FP64, so the result is the FP64 MPK of the rounded "
           "matrix.",
    "R24": "Newton shifts from Ritz values (Sec. 4: shifts from a few steps of standard "
           "GMRES): s steps of standard Arnoldi (Alg. 3b's one-vector-at-a-time subspace "
           "generation) on M from q0 = r0 / ||r0|| of the first cycle, stopped early if the "
           "Krylov space becomes invariant (a new vector's norm at most 2^-48 of ||M q_j||); "
           "the Ritz values are the eigenvalues of the square Hessenberg matrix. The shifts "
           "are their real parts (a complex pair gives its common real part twice, which keeps "
           "the basis real; the paper's shifts are real) in the Leja order of R18, repeated "
           "cyclically when fewer than s were found, kept for the whole solve; every column is "
           "scaled by a quarter of the spread of the shifts (the capacity of the interval they "
           "span; |shift| or 1 when they coincide).",
    "R23": "AMG pre-smoother fused with the residual (Sec. 5.3): nu outer GS2 sweeps on "
           "A x = b from a given x^0, then r = b - A x^nu. The paper names its GS2 listing "
           "the non-compact form of Gauss-Seidel, x^{k+1} = x^k + (D + L)^{-1}(b - A x^k), "
           "whose update x^{k+1} = x^k + g_gamma it prints; so for sweeps after the first "
           "g_0 is read as D^{-1}(b - A x^k) (the residual, which the printed "
           "D^{-1}(b - U x^k) equals only when x^k = 0), then g_j = g_0 - D^{-1} L g_{j-1}, "
           "j = 1..gamma, x^{k+1} = x^k + g_gamma. gamma = 0 is the Jacobi smoother "
           "x^{k+1} = x^k + D^{-1}(b - A x^k). With x^0 = 0 and nu = 1, x^1 is R21's "
           "P^{-1} b.",
}


# --------------------------------------------------------------------------- #
# Sec. 3, Alg. 1 and Alg. 2: the plain MPK
# --------------------------------------------------------------------------- #
def _arrays(A):
    n, rowptr, col, val = A
    return int(n), np.asarray(rowptr, dtype=np.int64), np.asarray(col, dtype=np.int64), \
        np.asarray(val, dtype=np.float64)


def spmv(A, x):
    """y = A x (Sec. 3, Alg. 1: one sparse matrix-vector product per power).

    y_i is the sum over row i's stored entries of a_ij * x_j: every product is
    rounded on its own (no fused multiply-add) and the sum runs over the
    entries in stored (ascending-column) order, starting from zero.  The
    products are formed elementwise and ``np.bincount`` then adds the weights
    of each output bin in input order, which is that sequential row sum.
    """
    n, rowptr, col, val = _arrays(A)
    x = np.asarray(x, dtype=np.float64)
    prod = val * x[col]
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    return np.bincount(rows, weights=prod, minlength=n)


def spmv_rows(A, x, r0, r1):
    """Rows r0..r1-1 of A x, with the same per-row summation order as ``spmv``."""
    n, rowptr, col, val = _arrays(A)
    a, b = rowptr[r0], rowptr[r1]
    prod = val[a:b] * np.asarray(x, dtype=np.float64)[col[a:b]]
    rows = np.repeat(np.arange(r1 - r0, dtype=np.int64), np.diff(rowptr[r0:r1 + 1]))
    return np.bincount(rows, weights=prod, minlength=r1 - r0)


def _bf16_rne(v32):
    """Rounds FP32 values to the nearest BF16 value (ties to even) on their bit
    patterns: keep the upper 16 bits after adding 0x7FFF plus the lowest kept bit."""
    b = np.asarray(v32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def round_values_bf16_rowscale(A):
    """Reading R16: a_ij ~ s_i q_ij with s_i = fl32(max_j |a_ij|) (1 for an all-zero
    row) and q_ij = bf16(fl32(a_ij / s_i)) (round to nearest even); the product
    s_i q_ij (8 + 24 significant bits) is exact in FP64.  Returns the matrix of
    those products."""
    n, rowptr, col, val = A
    rp = np.asarray(rowptr, dtype=np.int64)
    v = np.asarray(val, dtype=np.float64)
    rows = np.repeat(np.arange(int(n)), np.diff(rp))
    amax = np.zeros(int(n))
    np.maximum.at(amax, rows, np.abs(v))
    scale = np.where(amax > 0, amax, 1.0).astype(np.float32)
    q = _bf16_rne((v / scale[rows].astype(np.float64)).astype(np.float32))
    return type(A)(n, rowptr, col, scale[rows].astype(np.float64) * q.astype(np.float64))


def round_values(A, dtype=np.float32):
    """Reading R11: the matrix with every stored value rounded once to ``dtype``
    (round to nearest, ties to even, by NumPy's conversion) and widened back to
    FP64 exactly.  ``mpk(round_values(A), x, p)`` is the reduced-precision MPK."""
    n, rowptr, col, val = A
    return type(A)(n, rowptr, col, np.asarray(val, dtype=np.float64).astype(dtype).astype(np.float64))


def mpk(A, x, p):
    """Alg. 1: y_0 = x and y_k = A y_{k-1} for k = 1..p.  Returns Y with Y[k-1] = y_k."""
    y = np.asarray(x, dtype=np.float64)
    out = np.empty((p, y.size))
    for k in range(p):
        y = spmv(A, y)
        out[k] = y
    return out


# --------------------------------------------------------------------------- #
# Sec. 4 (Newton basis) and Sec. 5.2/5.3 (polynomials applied through the MPK)
# --------------------------------------------------------------------------- #
def newton_basis(A, v, lambdas, sigmas=None):
    """s-step basis with constant real shifts (Sec. 4; reading R8).

    V_0 = v and V_k = (A - lambda_k I) V_{k-1} / sigma_k for k = 1..s
    (sigma_k = 1 when ``sigmas`` is None; lambda_k = 0 gives the monomial basis).
    Returns an (s+1, n) array.
    """
    lambdas = np.asarray(lambdas, dtype=np.float64)
    s = lambdas.size
    V = np.empty((s + 1, np.asarray(v).size))
    V[0] = v
    for k in range(1, s + 1):
        w = spmv(A, V[k - 1]) - lambdas[k - 1] * V[k - 1]
        if sigmas is not None:
            w = w / sigmas[k - 1]
        V[k] = w
    return V


def poly_monomial(A, x, c):
    """Eq. (3): sum_{k=0..d} c_k A^k x with the powers from the plain MPK."""
    c = np.asarray(c, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    out = c[0] * x
    if c.size > 1:
        Y = mpk(A, x, c.size - 1)
        for k in range(1, c.size):
            out = out + c[k] * Y[k - 1]
    return out


def poly_newton(A, x, c, lambdas):
    """sum_{k=0..d} c_k phi_k with phi_0 = x, phi_k = (A - lambda_k I) phi_{k-1}."""
    c = np.asarray(c, dtype=np.float64)
    V = newton_basis(A, x, np.asarray(lambdas, dtype=np.float64)[: c.size - 1])
    out = c[0] * V[0]
    for k in range(1, c.size):
        out = out + c[k] * V[k]
    return out


def poly_chebyshev(A, x, c, theta, delta):
    """sum_{k=0..d} c_k t_k with the Chebyshev three-term recurrence (reading R9)."""
    c = np.asarray(c, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    out = c[0] * x
    if c.size == 1:
        return out
    t_prev = x
    t = (spmv(A, x) - theta * x) / delta
    out = out + c[1] * t
    for k in range(2, c.size):
        t_next = 2.0 * (spmv(A, t) - theta * t) / delta - t_prev
        out = out + c[k] * t_next
        t_prev, t = t, t_next
    return out


def chebyshev_inverse_coeffs(d, lmin, lmax):
    """Reading R12.  1 - lam s(lam) vanishes where T_d((theta - lam)/delta) does, i.e. at
    the d Chebyshev points lam_j = theta + delta u_j, u_j = cos(pi (j + 1/2) / d), so s
    (degree d - 1) is the interpolant of 1/lam at those points.  Its coefficients in the
    basis T_k(u) follow from the discrete orthogonality of T_k at the u_j:
    c_k = (2 - [k = 0]) / d * sum_j T_k(u_j) / lam_j.  Returns (c, theta, delta)."""
    if d < 1 or not (0 < lmin < lmax):
        raise ValueError("need d >= 1 and 0 < lmin < lmax")
    theta, delta = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    j = np.arange(d)
    u = np.cos(np.pi * (j + 0.5) / d)
    lam = theta + delta * u
    k = np.arange(d)[:, None]
    Tk = np.cos(k * np.arccos(u)[None, :])
    c = (2.0 / d) * (Tk / lam[None, :]).sum(axis=1)
    c[0] *= 0.5
    return c, theta, delta


def refine_solve(A, b, x0, d, lmin, lmax, tol, max_iter, values=np.float32):
    """Reading R13: FP64 residuals with A, corrections s(A~) r with A~ = round_values(A)
    (or A itself when ``values`` is None).  Returns (x, relative residual history)."""
    Alo = A if values is None else round_values(A, values)
    c, theta, delta = chebyshev_inverse_coeffs(d, lmin, lmax)
    b = np.asarray(b, dtype=np.float64)
    x = np.array(x0, dtype=np.float64)
    nb = np.linalg.norm(b)
    hist = []
    for it in range(max_iter + 1):
        r = b - spmv(A, x)
        hist.append(np.linalg.norm(r) / nb)
        if hist[-1] <= tol or it == max_iter:
            break
        x = x + poly_chebyshev(Alo, r, c, theta, delta)
    return x, hist


# --------------------------------------------------------------------------- #
# Sec. 4 (s-step GMRES, Alg. 3a and 3c) with the right polynomial
# preconditioner of Sec. 5 (readings R17-R19)
# --------------------------------------------------------------------------- #
def leja_order(points):
    """Reading R18: Leja order.  The first point has the largest modulus; each next
    one maximises the product of its distances to the points already taken.  Ties go
    to the lowest index.  Returns the reordered array."""
    pts = [float(v) for v in points]
    left = list(range(len(pts)))
    out = []
    while left:
        best, best_val = None, -1.0
        for i in left:
            if out:
                val = 1.0
                for z in out:
                    val *= abs(pts[i] - z)
            else:
                val = abs(pts[i])
            if val > best_val:
                best, best_val = i, val
        out.append(pts[best])
        left.remove(best)
    return np.array(out)


def chebyshev_scale(d, lmin, lmax):
    """T_d(theta/delta) for theta, delta of [lmin, lmax] (theta/delta > 1):
    cosh(d arccosh(theta/delta))."""
    theta, delta = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    return math.cosh(d * math.acosh(theta / delta))


def newton_shifts(s, d, lmin, lmax):
    """Reading R18: the spectrum of M = A s(A) (s of R12, A SPD with spectrum in
    [lmin, lmax]) lies in [1 - eps, 1 + eps], eps = 1 / T_d(theta/delta).  The shifts
    are the s Chebyshev points 1 + eps cos(pi (2i + 1) / (2s)) of that interval in Leja
    order, and every column is scaled by sigma = eps / 2.  Returns (lambdas, sigmas)."""
    eps = 1.0 / chebyshev_scale(d, lmin, lmax)
    i = np.arange(s)
    pts = 1.0 + eps * np.cos(np.pi * (2 * i + 1) / (2 * s))
    return leja_order(pts), np.full(s, 0.5 * eps)


def cholqr_truncated(G, wnorm2, eta=2.0 ** -24):
    """Reading R17, TSQR as Cholesky QR: the upper triangular R with G = R^T R, column
    by column.  Column j is dependent when its squared pivot G_jj - sum_{l<j} R_lj^2 is
    not above eta^2 * wnorm2[j] (or not finite); then R's column j holds its rows
    0..j-1 only and the factorisation stops.  Returns (R, kept columns)."""
    s = G.shape[0]
    R = np.zeros((s, s))
    for j in range(s):
        for i in range(j):
            R[i, j] = (G[i, j] - sum(R[l, i] * R[l, j] for l in range(i))) / R[i, i]
        piv2 = G[j, j] - sum(R[l, j] ** 2 for l in range(j))
        if not (math.isfinite(piv2) and piv2 > eta * eta * wnorm2[j]):
            return R, j
        R[j, j] = math.sqrt(piv2)
    return R, s


def sstep_cycle(apply_M, q0, m, s, lambdas, sigmas, beta, target):
    """One restart cycle of s-step GMRES (Alg. 3c, reading R17) on the operator
    ``apply_M``, from the unit vector q0 = r / beta.  Blocks of sb = min(s, m - c)
    vectors: W_0 = q_c, W_k = (M - lambda_k I) W_{k-1} / sigma_k (the Newton basis of
    Sec. 4); BOrtho, one classical Gram-Schmidt sweep R_prev = Q^T W, W' = W - Q R_prev;
    TSQR, Cholesky QR of W' with truncation at a dependent column; the new Hessenberg
    columns from the change of basis; the least-squares residual is checked after every
    block (Alg. 3c's convergence check) against ``target``.
    Returns (Q, H, y, rho): Q (k+1 or k vectors), H, the least-squares solution y of
    min ||beta e_0 - H y|| and its residual rho."""
    n = q0.size
    Q = [np.asarray(q0, dtype=np.float64)]
    H = np.zeros((1, 0))
    c = 0
    while True:
        sb = min(s, m - c)
        W = [Q[c]]
        for k in range(1, sb + 1):
            W.append((apply_M(W[k - 1]) - lambdas[k - 1] * W[k - 1]) / sigmas[k - 1])
        Qm = np.array(Q)                      # (c+1, n)
        Wm = np.array(W[1:])                  # (sb, n)
        R_prev = Qm @ Wm.T                    # BOrtho: (c+1, sb)
        Wp = Wm - R_prev.T @ Qm
        G = Wp @ Wp.T                         # TSQR by Cholesky QR
        wnorm2 = (R_prev ** 2).sum(axis=0) + np.diag(G)
        R_new, kk = cholqr_truncated(G, wnorm2)
        dep = kk < sb
        for j in range(kk):                   # Q_new = W'[:, :kk] R_new[:kk, :kk]^{-1}
            v = Wp[j] - sum(R_new[i, j] * Q[c + 1 + i] for i in range(j))
            Q.append(v / R_new[j, j])
        nh = kk + (1 if dep else 0)           # new Hessenberg columns
        rows = c + kk + 1                     # Q vectors now held
        # W_0..W_nh in the basis Q_0..Q_{rows-1}
        Rfull = np.zeros((rows, nh + 1))
        Rfull[c, 0] = 1.0
        for i in range(1, nh + 1):
            Rfull[: c + 1, i] = R_prev[:, i - 1]
            top = min(i, kk)
            Rfull[c + 1: c + 1 + top, i] = R_new[:top, i - 1]
        B = np.zeros((nh + 1, nh))            # M W_{0..nh-1} = W_{0..nh} B
        for i in range(nh):
            B[i, i] = lambdas[i]
            B[i + 1, i] = sigmas[i]
        Rk_top = Rfull[:c, :nh]
        Rk_bot = Rfull[c: c + nh, :nh]
        rhs = Rfull @ B
        if c > 0:
            rhs[: c + 1] -= H[: c + 1, :c] @ Rk_top
        Hnew = np.zeros((rows, c + nh))
        Hnew[: H.shape[0], :c] = H[:, :c]
        Hnew[:, c:] = np.linalg.solve(Rk_bot.T, rhs.T).T
        H = Hnew
        c += nh
        e0 = np.zeros(H.shape[0])
        e0[0] = beta
        y = np.linalg.lstsq(H, e0, rcond=None)[0] if c > 0 else np.zeros(0)
        rho = float(np.linalg.norm(e0 - H @ y)) if c > 0 else beta
        if dep or c >= m or rho <= target:
            return Q[:max(c, 1)], H, y, rho


def arnoldi(apply_M, q0, k):
    """Standard Arnoldi on ``apply_M`` from the unit vector q0 (the one-vector-at-a-time
    subspace generation of Alg. 3b, modified Gram-Schmidt), k steps, stopped when the
    Krylov space becomes invariant (reading R24).  Returns (Q, H) with Q the j + 1
    orthonormal vectors (rows) and H the (j + 1) x j Hessenberg matrix, M Q[:j] = Q H; on an
    early stop H is j x j (M Q = Q H) and Q holds j vectors."""
    Q = [np.asarray(q0, dtype=np.float64)]
    H = np.zeros((k + 1, k))
    for j in range(k):
        w = apply_M(Q[j])
        wn = float(np.linalg.norm(w))
        for i in range(j + 1):
            H[i, j] = float(Q[i] @ w)
            w = w - H[i, j] * Q[i]
        H[j + 1, j] = float(np.linalg.norm(w))
        if not H[j + 1, j] > 2.0 ** -48 * wn:
            return np.array(Q), H[: j + 1, : j + 1]
        Q.append(w / H[j + 1, j])
    return np.array(Q), H


def ritz_shifts(apply_M, q0, s):
    """Reading R24: Newton shifts from the Ritz values of s Arnoldi steps on M from q0:
    the real parts of the eigenvalues of the square Hessenberg matrix in Leja order (R18),
    repeated cyclically up to s, each column scaled by a quarter of their spread.
    Returns (lambdas, sigmas)."""
    Q, H = arnoldi(apply_M, q0, s)
    k = H.shape[1]
    theta = np.linalg.eigvals(H[:k, :k])
    lam = leja_order(np.real(theta))
    lam = np.array([lam[i % lam.size] for i in range(s)])
    spread = float(lam.max() - lam.min())
    sig = spread / 4.0 if spread > 0.0 else (abs(float(lam[0])) if lam[0] != 0.0 else 1.0)
    return lam, np.full(s, sig)


def interval_shifts(s, lo, hi):
    """Reading R22: Newton shifts for an operator whose spectrum lies in [lo, hi]: the s
    Chebyshev points of the interval in Leja order, every column scaled by a quarter of
    the interval's width (half its half-width, as in R18)."""
    c, h = 0.5 * (hi + lo), 0.5 * (hi - lo)
    i = np.arange(s)
    return leja_order(c + h * np.cos(np.pi * (2 * i + 1) / (2 * s))), np.full(s, 0.5 * h)


def sstep_gmres_precond(A, b, x0, s, m, precond, lmin, lmax, tol, max_cycles, values=None, gamma=1, ksweeps=1):
    """Reading R22: s-step GMRES (Alg. 3a/3c) without a preconditioner (M = A, x = x0 + Q y),
    with the diagonal (one-sweep Jacobi) preconditioner from the right (M = A D^{-1},
    x = x0 + D^{-1} Q y, Sec. 5.1), or with the GS2 preconditioner of gs2_precondition
    (M = A P^{-1}, x = x0 + P^{-1} Q y, ``gamma`` inner sweeps); with ``ksweeps`` > 1 the
    Jacobi preconditioner is k sweeps (R20), applied through B = A D^{-1} whose diagonal is
    one: M = jacobi_mpk(B) = I - (I - B)^k and x = x0 + D^{-1} jacobi_precondition(B, Q y).
    [lmin, lmax] holds the
    spectrum of M, the shifts are those of interval_shifts, and the cycle is sstep_cycle;
    with lmin = lmax = None the shifts are ritz_shifts of the first cycle's q0 (R24).
    With ``values`` the basis and the preconditioner use the rounded matrix.
    Returns (x, history, iters)."""
    if precond not in ("none", "jacobi", "gs2"):
        raise ValueError("precond must be 'none', 'jacobi' or 'gs2'")
    d = diagonal(A) if precond == "jacobi" else None
    if precond == "jacobi":
        n, rp, c, v = _arrays(A)
        Mmat = type(A)(n, rp, c, v / d[c]) if hasattr(type(A), "_fields") else (n, rp, c, v / d[c])
    else:
        Mmat = A
    Mlo = Mmat if values is None else round_values(Mmat, values)
    if precond == "gs2":
        def apply_M(w):
            return spmv(Mlo, gs2_precondition(Mlo, w, gamma))
    elif precond == "jacobi" and ksweeps > 1:
        def apply_M(w):
            return jacobi_mpk(Mlo, w, 1, ksweeps)[0]
    else:
        def apply_M(w):
            return spmv(Mlo, w)
    ritz = lmin is None and lmax is None
    lambdas, sigmas = (None, None) if ritz else interval_shifts(s, lmin, lmax)
    b = np.asarray(b, dtype=np.float64)
    x = np.array(x0, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    hist, iters = [], 0
    for cyc in range(max_cycles + 1):
        r = b - spmv(A, x)
        beta = float(np.linalg.norm(r))
        hist.append(beta / nb if nb > 0 else beta)
        if hist[-1] <= tol or cyc == max_cycles or beta == 0.0:
            break
        if lambdas is None:
            lambdas, sigmas = ritz_shifts(apply_M, r / beta, s)
        Q, H, y, rho = sstep_cycle(apply_M, r / beta, m, s, lambdas, sigmas, beta, tol * nb)
        iters += H.shape[1]
        z = np.zeros_like(x)
        for j in range(y.size):
            z = z + y[j] * Q[j]
        if precond == "gs2":
            z = gs2_precondition(Mlo, z, gamma)
        elif precond == "jacobi" and ksweeps > 1:
            z = jacobi_precondition(Mlo, z, ksweeps)
        x = x + (z / d if d is not None else z)
    return x, hist, iters


def sstep_gmres(A, b, x0, s, m, d, lmin, lmax, tol, max_cycles, values=None):
    """s-step GMRES (Alg. 3a with Alg. 3c, Sec. 4) on A s(A) u = b, x = s(A) u (right
    preconditioning, Sec. 5), s the degree d - 1 Chebyshev polynomial of R12, so one
    application of the operator costs d powers.  Restart length m (blocks of s);
    shifts of R18; each cycle starts from the FP64 residual r = b - A x with the
    unrounded matrix and stops the solve when ||r|| <= tol ||b|| or after max_cycles
    cycles (reading R19).  With ``values`` (e.g. np.float32) the basis and the
    preconditioner use the matrix rounded to that type (R11).
    Returns (x, true relative residual at the start of every cycle and at the end,
    number of Hessenberg columns built)."""
    Alo = A if values is None else round_values(A, values)
    c, theta, delta = chebyshev_inverse_coeffs(d, lmin, lmax)
    lambdas, sigmas = newton_shifts(s, d, lmin, lmax)

    def apply_M(v):                          # A P^{-1} v
        return spmv(Alo, poly_chebyshev(Alo, v, c, theta, delta))

    b = np.asarray(b, dtype=np.float64)
    x = np.array(x0, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    hist, iters = [], 0
    for cyc in range(max_cycles + 1):
        r = b - spmv(A, x)
        beta = float(np.linalg.norm(r))
        hist.append(beta / nb if nb > 0 else beta)
        if hist[-1] <= tol or cyc == max_cycles or beta == 0.0:
            break
        Q, H, y, rho = sstep_cycle(apply_M, r / beta, m, s, lambdas, sigmas, beta, tol * nb)
        iters += H.shape[1]
        z = np.zeros_like(x)
        for j in range(y.size):
            z = z + y[j] * Q[j]
        x = x + poly_chebyshev(Alo, z, c, theta, delta)
    return x, hist, iters


# --------------------------------------------------------------------------- #
# Sec. 5.1 (Jacobi preconditioner): the preconditioned MPK (A P^{-1})^j x
# --------------------------------------------------------------------------- #
def diagonal(A):
    """The stored diagonal of A; raises ValueError if an entry is missing or zero."""
    n, rp, c, v = _arrays(A)
    d = np.zeros(n)
    for i in range(n):
        hit = np.nonzero(c[rp[i]:rp[i + 1]] == i)[0]
        if hit.size == 0 or v[rp[i] + hit[0]] == 0.0:
            raise ValueError(f"row {i} has no nonzero diagonal entry")
        d[i] = v[rp[i] + hit[0]]
    return d


def jacobi_precondition(A, v, k):
    """Sec. 5.1, the Jacobi iteration z^{i+1} = D^{-1} v - D^{-1} (L + U) z^i from z^0 = 0,
    k iterations: z^k ~ A^{-1} v (k = 1 is the diagonal scaling D^{-1} v)."""
    d = diagonal(A)
    v = np.asarray(v, dtype=np.float64)
    z = np.zeros_like(v)
    for _ in range(k):
        offdiag = spmv(A, z) - d * z          # (L + U) z
        z = v / d - offdiag / d
    return z


def jacobi_mpk(A, x, p, k):
    """Reading R20: the Jacobi-preconditioned MPK of Sec. 5 with right preconditioning,
    w_0 = x, w_j = A P^{-1} w_{j-1} for j = 1..p, P^{-1} the k-sweep Jacobi iteration of
    jacobi_precondition.  Returns W with W[j-1] = w_j."""
    w = np.asarray(x, dtype=np.float64)
    out = np.empty((p, w.size))
    for j in range(p):
        w = spmv(A, jacobi_precondition(A, w, k))
        out[j] = w
    return out


def spmv_lower(A, x):
    """(L x)_i = sum over the stored entries a_ij with j < i (the strictly lower triangle in
    the original numbering), in stored order."""
    n, rp, c, v = _arrays(A)
    x = np.asarray(x, dtype=np.float64)
    y = np.zeros(n)
    for i in range(n):
        s = 0.0
        for e in range(rp[i], rp[i + 1]):
            if c[e] < i:
                s += v[e] * x[c[e]]
        y[i] = s
    return y


def gs2_precondition(A, v, gamma):
    """Reading R21, the two-stage Gauss-Seidel preconditioner of Sec. 5.1 (Alg. 4a) in the
    form the paper uses it: one outer iteration from z^0 = 0, so that g_0 = D^{-1} v,
    g_j = g_0 - D^{-1} L g_{j-1} for j = 1..gamma (inner Jacobi-Richardson sweeps for
    (D + L) g = v), and P^{-1} v = z^1 = g_gamma."""
    d = diagonal(A)
    g0 = np.asarray(v, dtype=np.float64) / d
    g = g0
    for _ in range(gamma):
        g = g0 - spmv_lower(A, g) / d
    return g


def gs2_mpk(A, x, p, gamma):
    """Reading R21: the GS2-preconditioned MPK, w_j = A P^{-1} w_{j-1} for j = 1..p with
    P^{-1} of gs2_precondition (gamma + 2 sub-powers per power: D^{-1}, gamma sweeps with
    L, then A).  Returns W with W[j-1] = w_j."""
    w = np.asarray(x, dtype=np.float64)
    out = np.empty((p, w.size))
    for j in range(p):
        w = spmv(A, gs2_precondition(A, w, gamma))
        out[j] = w
    return out


def gs2_smooth_residual(A, b, x0, sweeps, gamma):
    """Reading R23, the pre-smoothing step of an AMG cycle (Sec. 5.3) with the GS2 smoother
    of Sec. 5.1 and the residual that the cycle needs next: `sweeps` outer iterations of the
    non-compact form, each g_0 = D^{-1}(b - A x), g_j = g_0 - D^{-1} L g_{j-1} (j = 1..gamma),
    x = x + g_gamma; then r = b - A x.  Returns (x, r)."""
    d = diagonal(A)
    b = np.asarray(b, dtype=np.float64)
    x = np.array(x0, dtype=np.float64)
    for _ in range(sweeps):
        g0 = (b - spmv(A, x)) / d
        g = g0
        for _ in range(gamma):
            g = g0 - spmv_lower(A, g) / d
        x = x + g
    return x, b - spmv(A, x)


def chebyshev_basis(A, x, d, theta, delta):
    """The vectors t_0..t_d of reading R9 (used by tests)."""
    T = np.empty((d + 1, np.asarray(x).size))
    T[0] = x
    if d >= 1:
        T[1] = (spmv(A, T[0]) - theta * T[0]) / delta
    for k in range(2, d + 1):
        T[k] = 2.0 * (spmv(A, T[k - 1]) - theta * T[k - 1]) / delta - T[k - 2]
    return T


# --------------------------------------------------------------------------- #
# Sec. 3: level structure from a BFS of the matrix graph (readings R1-R4)
# --------------------------------------------------------------------------- #
def pattern_graph(A):
    """Undirected adjacency of pattern(A) union pattern(A^T) without self-loops (R1).

    Returns (ptr, adj) with adj[ptr[i]:ptr[i+1]] the sorted neighbours of i.
    """
    n, rowptr, col, _ = _arrays(A)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    r = np.concatenate([rows, col])
    c = np.concatenate([col, rows])
    keep = r != c
    key = np.unique(r[keep] * max(n, 1) + c[keep])
    r, c = key // max(n, 1), key % max(n, 1)
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=n), out=ptr[1:])
    return ptr, c


def _neighbours(ptr, adj, frontier):
    starts = ptr[frontier]
    lens = ptr[frontier + 1] - starts
    total = int(lens.sum())
    if total == 0:
        return np.zeros(0, dtype=np.int64)
    offs = np.repeat(starts - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens)
    return adj[offs + np.arange(total)]


def bfs_layers(ptr, adj, root, dist):
    """Breadth-first search from ``root``: layer d holds the vertices at distance d.

    ``dist`` (int64, -1 = unvisited) is updated in place; returns the list of
    layers, each sorted ascending.
    """
    frontier = np.array([root], dtype=np.int64)
    dist[root] = 0
    layers = [frontier]
    d = 0
    while True:
        nb = np.unique(_neighbours(ptr, adj, frontier))
        nb = nb[dist[nb] < 0]
        if nb.size == 0:
            return layers
        d += 1
        dist[nb] = d
        layers.append(nb)
        frontier = nb


def bfs_layers_queue(ptr, adj, root, n):
    """Textbook FIFO-queue BFS (pure Python, small graphs): distance of every vertex."""
    dist = [-1] * n
    dist[root] = 0
    q = deque([root])
    while q:
        u = q.popleft()
        for v in adj[ptr[u]:ptr[u + 1]]:
            if dist[v] < 0:
                dist[v] = dist[u] + 1
                q.append(int(v))
    return dist


def pseudo_peripheral_root(ptr, adj, start, n):
    """George-Liu pseudo-peripheral node search from ``start`` (reading R2).

    Returns (root, layers of the BFS from root).
    """
    r = int(start)
    layers_r = bfs_layers(ptr, adj, r, np.full(n, -1, dtype=np.int64))
    while True:
        last = layers_r[-1]
        deg = ptr[last + 1] - ptr[last]
        x = int(last[int(np.argmin(deg))])  # first minimum = lowest index (layers are sorted)
        layers_x = bfs_layers(ptr, adj, x, np.full(n, -1, dtype=np.int64))
        if len(layers_x) > len(layers_r):
            r, layers_r = x, layers_x
            continue
        return r, layers_r


def bfs_levels(A, root=None):
    """Level of every row (readings R1-R3).

    Returns (level, nlevels, roots) where ``roots`` lists the BFS root chosen
    for each component in processing order.
    """
    n = int(A[0])
    ptr, adj = pattern_graph(A)
    level = np.full(n, -1, dtype=np.int64)
    seen = np.zeros(n, dtype=bool)
    base = 0
    roots = []
    for v in range(n):
        if seen[v]:
            continue
        # the component of the lowest-index unvisited vertex
        comp_dist = np.full(n, -1, dtype=np.int64)
        comp = np.concatenate(bfs_layers(ptr, adj, v, comp_dist))
        if root is not None and comp_dist[int(root)] >= 0:
            r = int(root)
            layers = bfs_layers(ptr, adj, r, np.full(n, -1, dtype=np.int64))
        else:
            r, layers = pseudo_peripheral_root(ptr, adj, v, n)
        for d, layer in enumerate(layers):
            level[layer] = base + d
        seen[comp] = True
        base += len(layers)
        roots.append(r)
    return level, base, roots


def level_permutation(level, nlevels):
    """perm sorts rows by (level, original index) (R4).  Returns perm, iperm, level_ptr."""
    level = np.asarray(level, dtype=np.int64)
    n = level.size
    perm = np.lexsort((np.arange(n), level)).astype(np.int64)
    iperm = np.empty(n, dtype=np.int64)
    iperm[perm] = np.arange(n)
    level_ptr = np.zeros(nlevels + 1, dtype=np.int64)
    np.cumsum(np.bincount(level, minlength=nlevels), out=level_ptr[1:])
    return perm, iperm, level_ptr


def group_levels(A, level_ptr, perm, cache_bytes, q, value_bytes=8, min_group_rows=0):
    """Reading R14.  ``level_ptr`` and ``perm`` from ``level_permutation``; row
    weights use the original rows' entry counts.  Returns group_ptr (G + 1
    level indices): group g holds levels group_ptr[g] .. group_ptr[g+1]-1."""
    n, rowptr, _, _ = _arrays(A)
    nnz_row = np.diff(rowptr)[np.asarray(perm, dtype=np.int64)]
    budget = cache_bytes // q
    L = len(level_ptr) - 1
    group_ptr = [0]
    w_group, rows_group = 0, 0
    for lev in range(L):
        a, b = int(level_ptr[lev]), int(level_ptr[lev + 1])
        w = int(nnz_row[a:b].sum()) * (value_bytes + 4) + (b - a) * (4 + 16)
        if rows_group > 0 and w_group + w > budget and rows_group >= min_group_rows:
            group_ptr.append(lev)
            w_group, rows_group = 0, 0
        w_group += w
        rows_group += b - a
    group_ptr.append(L)
    return np.array(group_ptr, dtype=np.int64)


def wavefront_schedule(group_ptr, q):
    """Reading R15.  Returns the tasks of one block of q powers as a list of
    (stage, k, level_lo, level_hi), k = 1..q, in stage order (then k), empty
    tasks left out."""
    G = len(group_ptr) - 1
    L = int(group_ptr[-1])
    tasks = []
    for stage in range(G + q - 1):
        for k in range(1, q + 1):
            g = stage - (k - 1)
            if not (0 <= g < G):
                continue
            lo = 0 if g == 0 else max(0, int(group_ptr[g]) - (k - 1))
            hi = L - 1 if g == G - 1 else int(group_ptr[g + 1]) - 1 - (k - 1)
            if hi >= lo:
                tasks.append((stage, k, lo, hi))
    return tasks


def validate_schedule(B, level_ptr, tasks, q):
    """Checks a block schedule on the permuted matrix B: every (k, row) is covered
    exactly once; every read of y_{k-1}[j] (j a column of a row of the task)
    happens at a stage strictly later than the write of y_{k-1}[j] (k >= 2); a
    stage has at most one task per k.  Raises AssertionError on a violation."""
    n, rowptr, col, _ = _arrays(B)
    written = np.full((q + 1, n), -1, dtype=np.int64)  # stage that wrote y_k[row]
    written[0, :] = -(1 << 40)                        # y_0 = x exists before the block
    seen = set()
    for stage, k, lo, hi in tasks:
        assert (stage, k) not in seen, f"two tasks for power {k} in stage {stage}"
        seen.add((stage, k))
        r0, r1 = int(level_ptr[lo]), int(level_ptr[hi + 1])
        assert np.all(written[k, r0:r1] == -1), f"rows of power {k} covered twice"
        cols = col[rowptr[r0]:rowptr[r1]]
        assert np.all(written[k - 1, cols] < stage) and np.all(written[k - 1, cols] != -1), \
            f"power {k} in stage {stage} reads y_{k - 1} before it is written"
        written[k, r0:r1] = stage
    assert np.all(written[1:] >= 0), "some (power, row) is never computed"


def run_schedule(B, x, p, q, level_ptr, tasks_for, kind=None):
    """Executes p powers on the permuted matrix B block by block (R10), each
    block as the task list ``tasks_for(qb)`` in stage order, row by row with
    the row sums of ``spmv_rows``.  ``kind`` as in ``simulate_blocked_mpk``."""
    n = int(B[0])
    Y = np.full((p + 1, n), np.nan)
    Y[0] = np.asarray(x, dtype=np.float64)
    base = 0
    while base < p:
        qb = min(q, p - base)
        for _, k, lo, hi in tasks_for(qb):
            gk = base + k
            r0, r1 = int(level_ptr[lo]), int(level_ptr[hi + 1])
            acc = spmv_rows(B, Y[gk - 1], r0, r1)
            if kind is None:
                Y[gk, r0:r1] = acc
            else:
                prev2 = Y[gk - 2, r0:r1] if gk >= 2 else None
                Y[gk, r0:r1] = kind(gk, acc, Y[gk - 1, r0:r1], prev2)
        base += qb
    return Y[1:]


def permute_symmetric(A, perm, iperm):
    """B = P A P^T: B[i, j] = A[perm[i], perm[j]], columns re-sorted within each row."""
    n, rowptr, col, val = _arrays(A)
    lens = np.diff(rowptr)[perm]
    bptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=bptr[1:])
    # entry positions of old row perm[i], laid out row after row
    src = np.repeat(rowptr[perm] - bptr[:-1], lens) + np.arange(bptr[-1], dtype=np.int64)
    bcol = iperm[col[src]]
    bval = val[src]
    rows = np.repeat(np.arange(n, dtype=np.int64), lens)
    order = np.lexsort((bcol, rows))
    return (n, bptr, bcol[order], bval[order])
