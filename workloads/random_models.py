"""Random tiny kernel models for cross-checking the two oracle methods and,
later, the GPU path.  Domains stay small (at most a few hundred points per
access and tuple) so the pair double loop finishes quickly.

Expressions mix every operator of the language: affine terms, truncating
division and modulo by positive or negative constants and parameters, shifts,
min/max, comparisons and logical connectives, with optional guards, loops,
block/warp barrier-interval ids, 1-D to 3-D launches, several tuples, shared
and global arrays, all access kinds and scopes, and random caller masks.
"""
import numpy as np

from .expr import (E, c, param, tid, bid, bdim, gdim, loop, div, mod, shl, shr,
                   band, bor, bxor, emin, emax, lt, le, eq, ne, ge, gt, land,
                   lor, lnot, neg)
from .model import (Access, Array, Launch, Loop, Model, Workload, GLOBAL,
                    SHARED, READ, WRITE, ATOMIC, SCOPE_BLOCK, SCOPE_DEVICE)


def _coord(rng, n_loops_acc, loops_acc, allow_point=True):
    r = rng.integers(0, 10)
    if allow_point and r < 3:
        return tid(int(rng.integers(0, 3)))
    if allow_point and r < 5:
        return bid(int(rng.integers(0, 3)))
    if r < 6:
        return param(int(rng.integers(0, 2)))
    if r < 7:
        return bdim(int(rng.integers(0, 3))) if rng.random() < 0.5 else gdim(int(rng.integers(0, 3)))
    if n_loops_acc and r < 9:
        return loop(int(rng.choice(loops_acc)))
    return c(int(rng.integers(-3, 4)))


def rand_expr(rng, depth, loops_acc, allow_point=True, small=True):
    """A random expression over the variables visible to an access."""
    if depth <= 0 or rng.random() < 0.3:
        return _coord(rng, len(loops_acc), loops_acc, allow_point)
    a = rand_expr(rng, depth - 1, loops_acc, allow_point)
    r = rng.integers(0, 20)
    if r < 6:
        b = rand_expr(rng, depth - 1, loops_acc, allow_point)
        return a + b if r < 3 else a - b
    if r < 9:
        return a * int(rng.integers(-3, 4))
    if r < 11:
        d = int(rng.choice([1, 2, 3, 4, 5, -2, -3]))
        return div(a, d) if r == 9 else mod(a, d)
    if r == 11:
        return div(a, param(0)) if rng.random() < 0.5 else mod(a, param(0))
    if r == 12:
        return shl(a, int(rng.integers(0, 3)))
    if r == 13:
        return shr(a, int(rng.integers(0, 3)))
    b = rand_expr(rng, depth - 1, loops_acc, allow_point)
    op = [emin, emax, band, bor, bxor, lt, ne][int(rng.integers(0, 7))]
    return op(a, b)


def rand_guard(rng, loops_acc):
    r = rng.random()
    if r < 0.4:
        return None
    a = rand_expr(rng, 2, loops_acc)
    b = rand_expr(rng, 1, loops_acc)
    op = [lt, le, eq, ne, ge, gt][int(rng.integers(0, 6))]
    g = op(a, b)
    if rng.random() < 0.3:
        g2 = [lt, ge][int(rng.integers(0, 2))](rand_expr(rng, 1, loops_acc), rand_expr(rng, 1, loops_acc))
        g = land(g, g2) if rng.random() < 0.6 else lor(g, g2)
    if rng.random() < 0.1:
        g = lnot(g)
    return g


def rand_model(rng, n_acc=4):
    """One random small model with n_acc accesses on two arrays."""
    gx, gy, gz = [int(x) for x in rng.integers(1, 4, size=3)]
    if rng.random() < 0.5:
        gy = gz = 1
    bx = int(rng.choice([1, 2, 3, 4, 6, 8]))
    by = int(rng.choice([1, 1, 2, 3]))
    bz = int(rng.choice([1, 1, 2]))
    warp = int(rng.choice([1, 2, 4, 8, 32]))
    n_sets = int(rng.integers(1, 4))
    # params: p0 positive (used as a divisor), p1 any small value
    sets = [[int(rng.integers(1, 5)), int(rng.integers(-3, 6))] for _ in range(n_sets)]
    loops = [Loop(0, "lt", int(rng.integers(1, 4)), "add", 1),
             Loop(param(0), "gt", 0, "sub", 1),
             Loop(1, "le", 4, "shl", 1)]
    arrays = [Array(SHARED if rng.random() < 0.4 else GLOBAL, 64),
              Array(GLOBAL, 32)]
    accs = []
    for _ in range(n_acc):
        k = int(rng.integers(0, 3))
        loops_acc = sorted(int(x) for x in rng.choice(3, size=k, replace=False)) if k else []
        kind = [READ, WRITE, WRITE, ATOMIC][int(rng.integers(0, 4))]
        scope = SCOPE_BLOCK if rng.random() < 0.3 else SCOPE_DEVICE
        addr = rand_expr(rng, 3, loops_acc)
        guard = rand_guard(rng, loops_acc)
        bint = None
        wint = None
        if loops_acc and rng.random() < 0.3:
            bint = mod(loop(loops_acc[0]), 2) if rng.random() < 0.5 else loop(loops_acc[0])
        if rng.random() < 0.2:
            wint = c(int(rng.integers(0, 2)))
        arr = int(rng.integers(0, 2))
        accs.append(Access(arr, kind, addr, guard, loops_acc, bint, wint, scope))
    return Model(2, arrays, accs, Launch((gx, gy, gz), (bx, by, bz), warp), sets,
                 loops=loops, name="rand")


def rand_workload(seed, n_models=4, pairs_per_model=6):
    """Random tiny models and random pairs on the same array (plus a few
    self-pairs), with random caller masks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    models, pairs = [], []
    for mi in range(n_models):
        m = rand_model(rng)
        models.append(m)
        for _ in range(pairs_per_model):
            a = int(rng.integers(0, len(m.accesses)))
            if rng.random() < 0.25:
                b = a
            else:
                same = [k for k, x in enumerate(m.accesses)
                        if x.array == m.accesses[a].array]
                b = int(rng.choice(same))
            mask = 7 if rng.random() < 0.7 else int(rng.integers(0, 8))
            pairs.append((mi, a, b, mask))
    return Workload(models, pairs, name="rand%d" % seed)


def _sync_addr(rng, loops_acc):
    """A synchronisation address that often coincides between threads."""
    r = int(rng.integers(0, 8))
    if r == 0:
        return c(int(rng.integers(0, 2)))
    if r == 1:
        return mod(tid(0), 2)
    if r == 2:
        return bid(0)
    if r == 3:
        return mod(tid(0) + bid(0), 2)
    if r == 4 and loops_acc:
        return loop(int(rng.choice(loops_acc)))
    if r == 5:
        return div(tid(0), 2)
    return mod(rand_expr(rng, 1, loops_acc), 3)


def rand_sync_model(rng, n_acc=4):
    """A random small model whose accesses are guarded by random acquires
    and releases (section 6.5): locks, producer/consumer flags, mismatched
    pairs, block and device scopes, in a global and a shared lock array."""
    from .model import Sync
    m = rand_model(rng, n_acc)
    m.arrays = m.arrays + [Array(GLOBAL, 64), Array(SHARED, 32)]
    for a in m.accesses:
        r = rng.random()
        if r < 0.2:
            continue
        arr = int(rng.integers(2, 4))
        sc = lambda: SCOPE_BLOCK if rng.random() < 0.3 else SCOPE_DEVICE
        if r < 0.55:
            # a lock: acquire and release on one address
            e = _sync_addr(rng, a.loops)
            a.acq, a.rel = Sync(arr, e, sc()), Sync(arr, e, sc())
        else:
            if rng.random() < 0.75:
                a.acq = Sync(arr, _sync_addr(rng, a.loops), sc())
            if rng.random() < 0.75:
                arr2 = arr if rng.random() < 0.7 else 5 - arr
                a.rel = Sync(arr2, _sync_addr(rng, a.loops), sc())
    return m


def rand_sync_workload(seed, n_models=4, pairs_per_model=6):
    """Random tiny models with synchronisation, random pairs on one array."""
    rng = np.random.Generator(np.random.PCG64(seed))
    models, pairs = [], []
    for mi in range(n_models):
        m = rand_sync_model(rng)
        models.append(m)
        for _ in range(pairs_per_model):
            a = int(rng.integers(0, len(m.accesses)))
            if rng.random() < 0.25:
                b = a
            else:
                same = [k for k, x in enumerate(m.accesses)
                        if x.array == m.accesses[a].array]
                b = int(rng.choice(same))
            mask = 7 if rng.random() < 0.7 else int(rng.integers(0, 8))
            pairs.append((mi, a, b, mask))
    return Workload(models, pairs, name="randsync%d" % seed)
