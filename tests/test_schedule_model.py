"""Checks of the blocked kernel's work hand-out design (tests/schedule_model.py):
chunk ownership, dependency lists, units, the deadlock bound, and that the
design's execution order completes and reproduces the oracle's plain MPK
bitwise.  These test a design choice of the HIP path, not the paper."""
import numpy as np
import pytest

import oracle as O
import synth as S
import schedule_model as SM


def dense(A):
    n, rp, c, v = A
    D = np.zeros((n, n))
    for i in range(n):
        D[i, c[rp[i]:rp[i + 1]]] = v[rp[i]:rp[i + 1]]
    return D


def _schedule(A, chunk_rows, nparts):
    level, nl, _ = O.bfs_levels(A)
    perm, iperm, level_ptr = O.level_permutation(level, nl)
    B = O.permute_symmetric(A, perm, iperm)
    lnew = level[perm]
    owner = SM.chunk_owner(level_ptr, lnew, A.n, chunk_rows, nparts)
    deps = SM.chunk_dependencies(B, chunk_rows)
    clev = lnew[np.arange(len(deps)) * chunk_rows]
    return B, perm, owner, deps, clev


def test_chunk_owner_and_deps_on_grid():
    A = S.laplacian_2d(20, 20)
    B, perm, owner, deps, clev = _schedule(A, 8, 4)
    assert owner.min() >= 0 and owner.max() <= 3
    # one hop from every chunk reaches the level before it
    b1 = SM.hop_min(deps, np.arange(len(deps)), 1)
    assert np.all(b1[1:] < np.arange(1, len(deps)))
    # brute force: chunk c waits on c' iff some row of c touches a row of c'
    Bd = dense(B) != 0
    Bd = Bd | Bd.T
    for c in range(len(deps)):
        touch = Bd[c * 8:(c + 1) * 8].any(axis=0)
        want = sorted({j // 8 for j in np.nonzero(touch)[0]} - {c})
        assert list(deps[c]) == want


def test_chunk_owner_fraction_rule():
    # the level sizes of a 1D chain are all 1: every chunk belongs to partition 0
    A = S.laplacian_1d(40)
    _, _, owner, _, _ = _schedule(A, 4, 8)
    assert np.all(owner == 0)
    # star with centre 0 and leaves 1..16: George-Liu moves the root to leaf 1
    # (ecc 2 > 1), so the levels are {1}, {0}, {2..16}; the last level of 15 rows
    # is cut into 8 partitions by position
    M = np.eye(17)
    M[0, 1:] = 1
    A = S.from_dense(M + M.T)
    level, nl, roots = O.bfs_levels(A)
    assert roots == [1] and list(np.bincount(level)) == [1, 1, 15]
    perm, iperm, lp = O.level_permutation(level, nl)
    own = SM.chunk_owner(lp, level[perm], 17, 1, 8)
    assert list(own) == [0, 0] + [(8 * i) // 15 for i in range(15)]


@pytest.mark.parametrize("group", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("mk,cr,parts,q,p", [
    (lambda: S.laplacian_2d(16, 16), 8, 4, 3, 7),
    (lambda: S.laplacian_3d(6, 6, 6), 16, 8, 4, 4),
    (lambda: S.random_pattern(200, 3, 5), 8, 2, 2, 5),
    (lambda: S.block_diagonal(S.laplacian_2d(9, 7), S.identity(5), S.laplacian_1d(30)), 4, 8, 4, 9),
])
def test_blocked_schedule_equals_plain_mpk(mk, cr, parts, q, p, group):
    # with the fewest workers that meet the window condition, the blocked order
    # completes and gives bitwise the plain powers of the permuted matrix
    A = mk()
    B, perm, owner, deps, clev = _schedule(A, cr, parts)
    x = S.uniform_vector(A.n, 3)
    w = SM.min_workers(owner, deps, group, q)
    Y = SM.simulate_blocked_mpk(B, x[perm], p, q, cr, owner, deps, w, group=group)
    assert not np.isnan(Y).any()
    assert np.array_equal(Y, O.mpk(B, x[perm], p))


def test_units_reduce_to_chunks_for_group_one():
    A = S.laplacian_2d(14, 11)
    B, perm, owner, deps, clev = _schedule(A, 4, 3)
    units, upart = SM.worker_units(owner, 1)
    assert [int(u[0]) for u in units] == [int(c) for x in range(3) for c in np.nonzero(owner == x)[0]]
    udeps = SM.unit_dependencies(units, deps, len(deps))
    unit_of = {int(u[0]): i for i, u in enumerate(units)}
    for c in range(len(deps)):
        assert sorted(int(units[v][0]) for v in udeps[unit_of[c]]) == list(deps[c])


def test_blocked_schedule_deadlocks_when_window_too_small():
    # a 1D chain with single-row chunks and one worker: power 2 of chunk 0 waits on
    # chunk 1, which that same worker only starts after finishing chunk 0
    A = S.laplacian_1d(12)
    B, perm, owner, deps, clev = _schedule(A, 1, 1)
    first = np.arange(12)
    bmin = SM.hop_min(deps, first, 2)
    assert list(bmin) == [max(0, c - 2) for c in range(12)]
    assert not SM.window_ok(first, 1, bmin)
    with pytest.raises(RuntimeError):
        SM.simulate_blocked_mpk(B, np.ones(12), 3, 3, 1, owner, deps, 1)
    assert not SM.window_ok(first, 2, bmin) and SM.window_ok(first, 3, bmin)
    assert SM.min_workers(owner, deps, 1, 3) == 3
    Y = SM.simulate_blocked_mpk(B, np.ones(12), 3, 3, 1, owner, deps, 3)
    assert np.array_equal(Y, O.mpk(B, np.ones(12), 3))
    # units of two chunks: unit j waits on units j-1, j+1; two hops reach unit j-2
    assert SM.min_workers(owner, deps, 2, 3) == 3
    with pytest.raises(RuntimeError):
        SM.simulate_blocked_mpk(B, np.ones(12), 3, 3, 1, owner, deps, 2, group=2)
    Y = SM.simulate_blocked_mpk(B, np.ones(12), 3, 3, 1, owner, deps, 3, group=2)
    assert np.array_equal(Y, O.mpk(B, np.ones(12), 3))


@pytest.mark.parametrize("seed", range(6))
def test_window_condition_holds_with_fewer_active_workers(seed):
    # units are handed out in order, so workers that never run cannot stall the
    # others: launching many but running only the bound's number still completes
    rng = np.random.default_rng(100 + seed)
    A = S.random_pattern(int(rng.integers(300, 700)), 2.5, seed) if seed % 2 else \
        S.laplacian_3d(7, 6, int(rng.integers(4, 8)))
    B, perm, owner, deps, clev = _schedule(A, 4, 3)
    q = int(rng.integers(2, 5))
    g = int(rng.choice([1, 2]))
    w = SM.min_workers(owner, deps, g, q)
    Y = SM.simulate_blocked_mpk(B, np.ones(A.n), 2 * q, q, 4, owner, deps, 3 * w, group=g, active=w)
    assert np.array_equal(Y, O.mpk(B, np.ones(A.n), 2 * q))


@pytest.mark.parametrize("seed", range(8))
def test_early_claim_keeps_the_window_condition_sufficient(seed):
    # claiming the next unit during the last power, only once the partition's
    # next position is at least W beyond the current one, never deadlocks
    rng = np.random.default_rng(200 + seed)
    A = S.random_pattern(int(rng.integers(300, 800)), 2.5, seed) if seed % 2 else \
        S.laplacian_2d(int(rng.integers(12, 24)), int(rng.integers(12, 24)))
    B, perm, owner, deps, clev = _schedule(A, 4, 2)
    q = int(rng.integers(2, 5))
    g = int(rng.choice([1, 2]))
    w = SM.min_workers(owner, deps, g, q)
    for active in (w, 2 * w):
        Y = SM.simulate_blocked_mpk(B, np.ones(A.n), 2 * q + 1, q, 4, owner, deps, active, group=g,
                                   early=w)
        assert np.array_equal(Y, O.mpk(B, np.ones(A.n), 2 * q + 1))


def test_unrestricted_early_claim_can_deadlock():
    # without the distance rule, a worker may claim a unit that its own current
    # unit still waits on: a 1D chain, one worker, units of one chunk
    A = S.laplacian_1d(10)
    B, perm, owner, deps, clev = _schedule(A, 1, 1)
    with pytest.raises(RuntimeError):
        SM.simulate_blocked_mpk(B, np.ones(10), 2, 2, 1, owner, deps, 1, early=0)
    w = SM.min_workers(owner, deps, 1, 2)
    Y = SM.simulate_blocked_mpk(B, np.ones(10), 2, 2, 1, owner, deps, w, early=w)
    assert np.array_equal(Y, O.mpk(B, np.ones(10), 2))


@pytest.mark.parametrize("seed", range(4))
def test_window_condition_is_sufficient(seed):
    rng = np.random.default_rng(seed)
    A = S.laplacian_2d(int(rng.integers(8, 20)), int(rng.integers(8, 20)))
    B, perm, owner, deps, clev = _schedule(A, 4, 2)
    q = int(rng.integers(2, 5))
    g = int(rng.choice([1, 2, 3, 4, 5]))
    w = SM.min_workers(owner, deps, g, q)
    Y = SM.simulate_blocked_mpk(B, np.ones(A.n), q, q, 4, owner, deps, w, group=g)
    assert np.array_equal(Y, O.mpk(B, np.ones(A.n), q))


def test_blocked_schedule_operator_kinds():
    A = S.laplacian_2d(12, 10)
    B, perm, owner, deps, clev = _schedule(A, 8, 4)
    x = S.uniform_vector(A.n, 9)[perm]
    lam = [0.5, 1.0, 1.5, 2.0, 2.5]
    newton = lambda k, acc, prev, prev2: acc - lam[k - 1] * prev
    Y = SM.simulate_blocked_mpk(B, x, 5, 3, 8, owner, deps, 4, kind=newton, group=2)
    assert np.array_equal(Y, O.newton_basis(B, x, lam)[1:])
    th, de = 4.0, 4.0
    cheb = lambda k, acc, prev, prev2: ((acc - th * prev) / de if k == 1
                                        else 2.0 * (acc - th * prev) / de - prev2)
    Y = SM.simulate_blocked_mpk(B, x, 6, 4, 8, owner, deps, 4, kind=cheb)
    assert np.array_equal(Y, O.chebyshev_basis(B, x, 6, th, de)[1:])
