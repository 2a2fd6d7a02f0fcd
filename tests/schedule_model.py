"""Design model of the blocked kernel's work hand-out -- TEST-SIDE, NOT THE ORACLE.

The paper fixes what the MPK computes (Sec. 3, Alg. 1) but not how a GPU hands
out work; the rules below are this project's own design of the blocked kernel
(chunk ownership by XCD, units of G chunks handed out in order, the deadlock
bound on the number of resident workers).  They are modelled here so that the
host planner's tables can be cross-checked against an independent Python
statement of the same design, and so that the design's validity (coverage,
read-after-write order, deadlock freedom, bitwise equality with the plain MPK
of the oracle) can be tested on the CPU.  Equality with this model is a design
cross-check, not parity with the paper.

Design rules:
  D1  Rows are cut, in permuted order, into chunks of C consecutive rows (the
      last may be shorter); a chunk is the unit of work.
  D2  Chunk c is owned by partition x = floor(P (r0 - level_start) / level_size),
      r0 = C c its first row, level_start/level_size those of r0's level; each
      partition processes its chunks in ascending order.
  D3  Chunk c may compute power k once every chunk holding a row adjacent to c's
      rows in the symmetrised pattern has finished power k - 1.  Each
      partition's ascending chunk sequence is cut into units of G consecutive
      chunks; a worker takes the partition's next unit in sequence order,
      carries its chunks together through the q powers of a block, then takes
      the next.  With at least W active workers per partition this cannot
      deadlock when, for every unit position j >= W, the first chunk of unit
      j - W has a smaller index than the first chunk of every unit within q - 1
      unit-dependency hops of unit j (proof in ``window_ok``).
"""
import numpy as np

from oracle import pattern_graph, spmv_rows


def chunk_owner(level_ptr, level_of_new_row, n, chunk_rows, nparts):
    """Owner partition of every chunk (rule D2)."""
    nchunks = (n + chunk_rows - 1) // chunk_rows
    owner = np.empty(nchunks, dtype=np.int64)
    for c in range(nchunks):
        r0 = c * chunk_rows
        lv = int(level_of_new_row[r0])
        start, size = int(level_ptr[lv]), int(level_ptr[lv + 1] - level_ptr[lv])
        owner[c] = (nparts * (r0 - start)) // size
    return owner


def chunk_dependencies(B, chunk_rows):
    """For every chunk, the sorted other chunks holding a row adjacent to one of
    its rows in pattern(B) union pattern(B^T) (rule D3)."""
    n = int(B[0])
    ptr, adj = pattern_graph(B)
    nchunks = (n + chunk_rows - 1) // chunk_rows
    deps = []
    for c in range(nchunks):
        r0, r1 = c * chunk_rows, min(n, (c + 1) * chunk_rows)
        nb = adj[ptr[r0]:ptr[r1]] // chunk_rows
        nb = np.unique(nb)
        deps.append(nb[nb != c])
    return deps


def worker_units(owner, group):
    """Units of ``group`` consecutive chunks of each partition's ascending sequence
    (rule D3).  Returns (units, unit_part): a list of chunk-index arrays and the
    partition of each unit, units of partition 0 first, each partition in order."""
    owner = np.asarray(owner)
    nparts = int(owner.max()) + 1 if owner.size else 0
    units, part = [], []
    for x in range(nparts):
        seq = np.nonzero(owner == x)[0]
        for j in range(0, seq.size, group):
            units.append(seq[j:j + group])
            part.append(x)
    return units, np.asarray(part, dtype=np.int64)


def unit_dependencies(units, deps, nchunks):
    """Other units holding a chunk that some chunk of the unit waits on."""
    unit_of = np.empty(nchunks, dtype=np.int64)
    for u, ch in enumerate(units):
        unit_of[ch] = u
    out = []
    for u, ch in enumerate(units):
        d = np.unique(np.concatenate([unit_of[deps[c]] for c in ch])) if len(ch) else \
            np.zeros(0, dtype=np.int64)
        out.append(d[d != u])
    return out


def hop_min(udeps, first, hops):
    """B[u] = smallest first-chunk index among units within ``hops`` dependency hops
    of unit u (u included).  The relation is symmetric (it comes from a
    symmetrised pattern), so this is also the smallest first chunk of a unit from
    which u is reachable in ``hops``."""
    b = np.asarray(first, dtype=np.int64).copy()
    for _ in range(max(0, hops)):
        nb = b.copy()
        for u, dl in enumerate(udeps):
            if dl.size:
                nb[u] = min(nb[u], int(b[dl].min()))
        b = nb
    return b


def window_ok(first, workers, bmin):
    """Deadlock-freedom condition of rule D3 for one partition: ``first`` are the
    first-chunk indices of the partition's units in order, ``bmin`` their values of
    ``hop_min(..., q - 1)``.

    Proof sketch: in a deadlock every started unit waits; take the one whose
    first chunk c is smallest.  Its chain of waits has at most q-1 hops (powers
    drop by one per hop and power 1 never waits) and ends at a unit u that has
    not started.  If nobody holds u, units start in order, so the W busy
    workers of u's partition hold units at positions below u's, one of them at
    pos(u) - W or earlier, whose first chunk is below bmin[u] <= c.  If a worker
    claimed u early, it did so while on a unit at position <= pos(u) - W, whose
    first chunk is again below bmin[u] <= c.  Either way a waiting unit with a
    smaller first chunk exists: a contradiction.
    """
    first = np.asarray(first, dtype=np.int64)
    if first.size <= workers:
        return True
    return bool(np.all(first[:-workers] < np.asarray(bmin)[workers:]))


def min_workers(owner, deps, group, q):
    """Smallest W meeting ``window_ok`` in every partition (direct search)."""
    units, upart = worker_units(owner, group)
    udeps = unit_dependencies(units, deps, len(deps))
    first = np.array([u[0] for u in units], dtype=np.int64)
    bmin = hop_min(udeps, first, q - 1)
    parts = [np.nonzero(upart == x)[0] for x in range(int(upart.max()) + 1 if upart.size else 0)]
    for w in range(1, len(units) + 1):
        if all(window_ok(first[pu], w, bmin[pu]) for pu in parts):
            return w
    return max(1, len(units))


def simulate_blocked_mpk(B, x, p, q, chunk_rows, owner, deps, workers, kind=None, group=1,
                         active=None, early=None):
    """Execute the blocked MPK on permuted matrix B sequentially, in the worker
    order of rule D3, and return Y (p, n) in permuted space.

    Each partition hands out its units in sequence order to ``workers`` workers
    (``active`` of them actually run, default all).  A worker repeatedly tries to
    advance its current (unit, power): power k of all chunks of the unit is
    computed only when every chunk they wait on, outside the unit, has finished
    power k-1; an idle worker takes the partition's next unit.  ``early`` = W
    models a variant that the GPU kernel does not use: a worker about to compute
    the last power of the unit at position j first claims its next unit if the
    partition's next position is >= j + W (safe by the same condition, but a
    unit claimed this way cannot start until its holder finishes, which delays
    everything that waits on it).
    Values not yet computed are NaN, so a wrong order shows up as NaN in the
    result; a full sweep without progress raises (deadlock).  Powers are done
    in blocks of q (R10).  ``kind`` is None for plain powers, or a callable
    (k, acc, prev, prev2) -> y_k for the shifted and three-term forms, where
    acc = (A y_{k-1}) on the chunk's rows and prev/prev2 are y_{k-1}/y_{k-2} on
    the same rows.
    """
    n = int(B[0])
    nchunks = len(deps)
    Y = np.full((p + 1, n), np.nan)
    Y[0] = x
    units, upart = worker_units(owner, group)
    nparts = int(upart.max()) + 1 if upart.size else 0
    pu = [np.nonzero(upart == part)[0] for part in range(nparts)]
    inside = [set(u.tolist()) for u in units]
    nact = workers if active is None else active
    base = 0
    while base < p:
        qb = min(q, p - base)
        done = np.zeros(nchunks, dtype=np.int64)  # powers finished in this block
        ticket = [0] * nparts
        # worker: [partition, position of current unit or -1, power, claimed next position or -1]
        state = [[part, -1, 0, -1] for part in range(nparts) for _ in range(nact)]
        remaining = len(units) * qb
        while remaining:
            progress = False
            for st in state:
                part, pos, k, nxt = st
                if pos < 0:
                    if nxt >= 0:
                        pos, nxt = nxt, -1
                    elif ticket[part] < pu[part].size:
                        pos = ticket[part]
                        ticket[part] += 1
                    else:
                        continue
                    k = 1
                    st[1], st[2], st[3] = pos, k, nxt
                    progress = True
                u = int(pu[part][pos])
                if (early is not None and k == qb and nxt < 0 and ticket[part] < pu[part].size
                        and ticket[part] >= pos + early):
                    nxt = ticket[part]
                    ticket[part] += 1
                    st[3] = nxt
                    progress = True
                if k > 1 and any(done[d] < k - 1 for c in units[u] for d in deps[c]
                                 if int(d) not in inside[u]):
                    continue
                gk = base + k
                for c in units[u]:
                    r0, r1 = int(c) * chunk_rows, min(n, (int(c) + 1) * chunk_rows)
                    acc = spmv_rows(B, Y[gk - 1], r0, r1)
                    if kind is None:
                        Y[gk, r0:r1] = acc
                    else:
                        prev2 = Y[gk - 2, r0:r1] if gk >= 2 else None
                        Y[gk, r0:r1] = kind(gk, acc, Y[gk - 1, r0:r1], prev2)
                    done[c] = k
                remaining -= 1
                progress = True
                if k == qb:
                    st[1], st[2] = -1, 0
                else:
                    st[2] = k + 1
            if not progress:
                raise RuntimeError("blocked MPK schedule deadlocked")
        base += qb
    return Y[1:]
