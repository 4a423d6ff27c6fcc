"""Seeded synthetic workloads at the benchmark configurations.

The paper measures on 22 programs from public suites (section 7); none of
them is reproduced here.  These seeded workloads stand in for them, with the
access shapes the paper shows (affine 1-D/2-D indexing, thread-id division
and modulo, host-fixed parameters and launch extents, guards; section 4,
Figures 1-5).

Every generator is deterministic in its seed (numpy PCG64).  Races are
planted structurally (a non-injective thread-to-address map); race freedom is
planted by range separation or by an injective map.  Nothing here evaluates an
expression: the labels used by the tests come from the oracle.
"""
import numpy as np

from .expr import bid, bdim, tid, param, loop, c, lt, ge, emin, ne, eq
from .model import (Access, Array, Launch, Loop, Model, Workload, GLOBAL,
                    SHARED, READ, WRITE, ALL_CLASSES)


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------------------
# tiny plain config: one model, 64 pairs

def tiny(seed=1001, n_pairs=64):
    """One model, 64 access pairs, grid 4 x block 64 (1-D), warp 32,
    loop i in [0, 8), addr = c0 + c1*tid + c2*bid + c3*i + c4*N with every
    coefficient drawn from [-4, 4], N = 256, one tuple.

    Pairs: half on a shared array, half on a global one; 8 self-pairs
    (writes), the rest drawn from {W/W, W/R, R/W}.  16 pairs are racy by
    construction, 48 race-free by construction:
      * racy: both sides use the same coefficient vector with c1 = 0 (all
        threads of a block meet at one address in each iteration), or, for
        shared arrays, c1 != 0 and c3 != 0 (thread t at iteration i meets
        thread t' at iteration i' whenever c1*(t - t') = c3*(i' - i));
      * race-free cross pairs: |c4_i - c4_j| >= 3, so the address ranges
        (each within c4*256 +- 296) are disjoint;
      * race-free self-pairs: an injective thread map with c3 = 0
        (shared: c1 != 0; global: c1 = +-4 and c2 odd, so c1*t + c2*b is
        injective for b < 4).
    """
    rng = _rng(seed)
    G, B, I, N = 4, 64, 8, 256
    arrays = [Array(SHARED, 32), Array(GLOBAL, 32)]
    loops = [Loop(0, "lt", I, "add", 1)]
    accs, pairs, labels = [], [], []

    def coef():
        return [int(x) for x in rng.integers(-4, 5, size=5)]

    def mk(arr, kind, cf):
        c0, c1, c2, c3, c4 = cf
        addr = (c(c0) + c(c1) * tid(0) + c(c2) * bid(0) + c(c3) * loop(0)
                + c(c4) * param(0))
        accs.append(Access(arr, kind, addr, None, [0],
                           name="%s a%d %r" % (kind[0].upper(), arr, cf)))
        return len(accs) - 1

    def racy_cf(arr):
        cf = coef()
        if arr == 0 and rng.random() < 0.5:
            cf[1] = int(rng.choice([-4, -3, -2, -1, 1, 2, 3, 4]))
            cf[3] = int(rng.choice([-4, -3, -2, -1, 1, 2, 3, 4]))
        else:
            cf[1] = 0
        return cf

    def free_self_cf(arr):
        cf = coef()
        cf[3] = 0
        if arr == 0:
            cf[1] = int(rng.choice([-4, -3, -2, -1, 1, 2, 3, 4]))
        else:
            cf[1] = int(rng.choice([-4, 4]))
            cf[2] = int(rng.choice([-3, -1, 1, 3]))
        return cf

    # plan: per array 4 self-pairs (1 racy) and 28 cross pairs (7 racy)
    plan = []
    for arr in (0, 1):
        plan += [(arr, "self", True)] + [(arr, "self", False)] * 3
        plan += [(arr, "cross", True)] * 7 + [(arr, "cross", False)] * 21
    order = rng.permutation(len(plan))
    kinds = [(WRITE, WRITE), (WRITE, READ), (READ, WRITE)]
    for k in order:
        arr, form, racy = plan[k]
        if form == "self":
            cf = racy_cf(arr) if racy else free_self_cf(arr)
            a = mk(arr, WRITE, cf)
            pairs.append((0, a, a, ALL_CLASSES))
        else:
            ka, kb = kinds[int(rng.integers(0, 3))]
            if racy:
                cf = racy_cf(arr)
                a, b = mk(arr, ka, cf), mk(arr, kb, list(cf))
            else:
                ci = coef()
                while True:
                    cj = coef()
                    if abs(ci[4] - cj[4]) >= 3:
                        break
                a, b = mk(arr, ka, ci), mk(arr, kb, cj)
            pairs.append((0, a, b, ALL_CLASSES))
        labels.append(bool(racy))
    m = Model(1, arrays, accs, Launch((G, 1, 1), (B, 1, 1), 32), [[N]],
              loops=loops, name="tiny")
    return Workload([m], pairs[:n_pairs], name="tiny",
                    meta={"seed": seed, "planted_racy": labels[:n_pairs]})


# ---------------------------------------------------------------------------
# batched uneven config: 256 models x 16 pairs

def _log_uniform_int(rng, lo, hi):
    return int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))


def _host_widths(bx, gx, n):
    """At least n distinct candidate widths a host program derives: powers
    of two up to 128, then multiples of the block row width bx and the grid
    row width bx * gx."""
    out = [1, 2, 4, 8, 16, 32, 64, 128]
    k = 1
    while len(set(out)) < n or k <= 8:
        out += [bx * k, bx * gx * k]
        k += 1
    return sorted(set(out))


def batched(seed=2002, n_models=256, pairs_per_model=16, max_grid=1024,
            max_iters=64, max_sets=16, scale=1.0):
    """256 models x 16 pairs = 4096 queries of uneven size.

    Per model: grid log-uniform in [1, max_grid] blocks (1-D or 2-D), block
    of 32..256 threads (1-D or 2-D), one loop of 1..max_iters iterations,
    parameters (W, N) as joint tuples from a host-derived set of 1..16
    distinct values (W a power of two or a multiple of the row width, N derived from
    W: host class 3).  Address terms: tid/32, tid % W, row*W + col, affine
    in the global thread id and the loop variable.  Guards tid < N - k.
    int32 addresses.  Shared and global arrays alternate by model.  About
    30% of pairs are planted racy (non-injective maps or equal bases);
    labels come from the oracle.  ``scale`` shrinks the grids (for tests).
    """
    rng = _rng(seed)
    models, pairs = [], []
    for mi in range(n_models):
        two_d_grid = rng.random() < 0.4
        nblk = max(1, int(_log_uniform_int(rng, 1, max_grid) * scale))
        if two_d_grid and nblk >= 4:
            gx = 1 << int(rng.integers(1, max(2, int(np.log2(nblk)))))
            gx = min(gx, nblk)
            gy = max(1, nblk // gx)
        else:
            gx, gy = nblk, 1
        bt = int(rng.choice([32, 64, 128, 256]))
        two_d_block = rng.random() < 0.4 and bt >= 64
        if two_d_block:
            bx = int(rng.choice([16, 32]))
            by = bt // bx
        else:
            bx, by = bt, 1
        iters = max(1, _log_uniform_int(rng, 1, max_iters))
        space = SHARED if mi % 2 == 1 else GLOBAL
        nsets = int(rng.integers(1, max_sets + 1))
        # host-derived parameter set: nsets distinct W from powers of two and
        # multiples of the row width, N derived jointly from W (one host
        # variable feeds both)
        Ws = sorted(int(x) for x in rng.choice(
            _host_widths(bx, gx, max_sets), size=nsets, replace=False))
        sets = [[w, w * int(rng.integers(1, 5)) + bt // 2] for w in Ws]
        W, Np = param(0), param(1)
        row = bid(1) * bdim(1) + tid(1)
        col = bid(0) * bdim(0) + tid(0)
        tl = tid(0) + bdim(0) * tid(1)
        blin = bid(0) + c(gx) * bid(1)
        gid = blin * bt + tl
        i = loop(0)
        # per-block extent used to separate bases
        span_t = 2 * bt * iters + 4096
        accs = []
        arr = [Array(space, 32)]
        for p in range(pairs_per_model):
            racy = rng.random() < 0.30
            form = int(rng.integers(0, 4))
            selfp = rng.random() < 0.25
            k = int(rng.integers(0, 4))
            guard = lt(tl, Np - k) if rng.random() < 0.5 else None
            if space == SHARED:
                # shared memory is per block: addresses need not name the block
                if form == 0:
                    e_ok = tl * iters + i            # injective in (t, i)
                    e_bad = tl // 32 + i * 8        # 32 threads share
                elif form == 1:
                    e_ok = tl + bt * i
                    e_bad = tl % W + i             # W-periodic
                elif form == 2:
                    e_ok = tid(1) * (bx * iters) + tid(0) * iters + i
                    e_bad = tid(1) * W + tid(0)
                else:
                    e_ok = tl * 2 + i * (2 * bt)
                    e_bad = tl * 2 + i
            else:
                if form == 0:
                    e_ok = gid * iters + i
                    e_bad = gid // 32 + i * 4
                elif form == 1:
                    e_ok = gid + c(gx * gy * bt) * i
                    e_bad = tl % W + blin * W + i
                elif form == 2:
                    e_ok = (row * c(bx * gx) + col) * iters + i
                    e_bad = row * W + col
                else:
                    e_ok = blin * (bt * iters) + tl * iters + i
                    e_bad = tl + i * 16
            kinds = [(WRITE, WRITE), (WRITE, READ), (READ, WRITE)]
            ka, kb = kinds[int(rng.integers(0, 3))]
            if selfp:
                e = e_bad if racy else e_ok
                accs.append(Access(0, WRITE, e, guard, [0]))
                a = len(accs) - 1
                pairs.append((mi, a, a, ALL_CLASSES))
                continue
            if racy:
                ea, eb = e_bad, e_bad
                base_b = 0
            else:
                ea, eb = e_ok, e_ok
                base_b = int(rng.integers(2, 6)) * (span_t * max(1, gx * gy) + (1 << 16))
                if space == SHARED:
                    base_b = int(rng.integers(2, 6)) * span_t
            accs.append(Access(0, ka, ea, guard, [0]))
            accs.append(Access(0, kb, eb + base_b, guard, [0]))
            pairs.append((mi, len(accs) - 2, len(accs) - 1, ALL_CLASSES))
        models.append(Model(2, arr, accs, Launch((gx, gy, 1), (bx, by, 1), 32),
                            sets, loops=[Loop(0, "lt", iters, "add", 1)],
                            name="batched%d" % mi))
    return Workload(models, pairs, name="batched",
                    meta={"seed": seed, "scale": scale})


# ---------------------------------------------------------------------------
# race-free throughput stress: 128 pairs, 2^30 points per access, int64

def stress(seed=3003, n_pairs=128, grid=1 << 16, block=256, iters=64):
    """128 write/write or write/read pairs on 64-bit global arrays, each
    access with grid * block * iters points (2^16 * 256 * 64 = 2^30 by
    default), race-free by construction, no early exit possible:

      * strided-disjoint: A_i = base + 2 f, A_j = base + 2 f + 1 with
        f = (global thread id) * iters + i injective: one side even, the
        other odd, every address one away from an address of the other side;
      * blocked-disjoint: with K = block * iters, A_i covers
        [base + 2Kb, base + 2Kb + K) and A_j [base + 2Kb + K, base + 2K(b+1))
        for block b: adjacent ranges, edges one element apart.

    Bases are >= 2^40.  Every pair's verdict is 0 and count 0 by
    construction.
    """
    rng = _rng(seed)
    B, I = block, iters
    K = B * I
    g = bid(0) * bdim(0) + tid(0)
    f = g * I + loop(0)
    accs, pairs = [], []
    for p in range(n_pairs):
        base = (1 << 40) + int(rng.integers(0, 1 << 20)) * (1 << 24)
        kind_b = WRITE if rng.random() < 0.5 else READ
        if p % 2 == 0:
            ea = c(base) + f * 2
            eb = c(base) + f * 2 + 1
        else:
            ea = c(base) + bid(0) * (2 * K) + tid(0) * I + loop(0)
            eb = c(base) + bid(0) * (2 * K) + K + tid(0) * I + loop(0)
        accs.append(Access(0, WRITE, ea, None, [0], name="stress a%d" % p))
        accs.append(Access(0, kind_b, eb, None, [0], name="stress b%d" % p))
        pairs.append((0, 2 * p, 2 * p + 1, ALL_CLASSES))
    m = Model(0, [Array(GLOBAL, 64)], accs, Launch((grid, 1, 1), (B, 1, 1), 32),
              [[]], loops=[Loop(0, "lt", I, "add", 1)], name="stress")
    return Workload([m], pairs, name="stress",
                    meta={"seed": seed, "race_free": True,
                          "points_per_access": grid * B * I})


# ---------------------------------------------------------------------------
# sparse witnesses: one conflicting block pair out of G*G

def sparse(seed=4004, n_queries=16384, G=256, B=256, racy_frac=0.5,
           queries_per_model=64):
    """Queries whose only conflicts sit in a single (block of a, block of b)
    pair out of G * G: access a writes base + g, access b writes
    base + g + D + K * (bid != c_b) with g the global thread id; K moves
    every block of b except block c_b far away, and D shifts block c_b so
    that it lands on block c_a of a (D = B * (c_a - c_b)).  Race-free
    queries use D = G * B (a near miss: one past a's range), so no block
    pair meets.  Global int32 arrays, one tuple, no loops.
    """
    rng = _rng(seed)
    models, pairs = [], []
    for q0 in range(0, n_queries, queries_per_model):
        accs = []
        nq = min(queries_per_model, n_queries - q0)
        for k in range(nq):
            racy = rng.random() < racy_frac
            ca = int(rng.integers(0, G))
            cb = int(rng.integers(0, G))
            if cb == ca:  # same block, same thread: would not conflict
                cb = (ca + 1) % G
            base = int(rng.integers(0, 1 << 20)) * 4
            Kf = 4 * G * B
            g = bid(0) * bdim(0) + tid(0)
            D = B * (ca - cb) if racy else G * B
            ea = c(base) + g
            eb = c(base) + g + D + c(Kf) * ne(bid(0), cb)
            accs.append(Access(0, WRITE, ea, name="sparse a"))
            accs.append(Access(0, WRITE, eb, name="sparse b"))
            pairs.append((len(models), 2 * k, 2 * k + 1, ALL_CLASSES))
        models.append(Model(0, [Array(GLOBAL, 32)], accs,
                            Launch((G, 1, 1), (B, 1, 1), 32), [[]],
                            name="sparse%d" % len(models)))
    return Workload(models, pairs, name="sparse", meta={"seed": seed, "G": G})


def sparse_overlap(seed=4004, n_queries=16384, G=256, B=256, racy_frac=0.5,
                   queries_per_model=64):
    """Sparse witnesses among many overlapping tiles: the ranking problem of
    the learned tile order.  Access a writes base + 2 B bid + 2 tid (even
    addresses, block b1 covers [2 B b1, 2 B b1 + 2 B - 2]); access b writes
    base + 2 B bid + 2 tid + 1 (odd addresses interleaved with block bid of
    a: G tiles whose address ranges overlap but hold no conflict).  In a
    racy query one block c_b of b is moved onto block c_a of a with even
    addresses (its block term gains eq(bid, c_b) * (2 B (c_a - c_b) - 1)),
    so exactly one tile out of G * G conflicts (B conflicting thread pairs,
    inter-block), and it overlaps as the others do.  Global int32 arrays,
    one tuple, no loops.
    """
    rng = _rng(seed)
    models, pairs = [], []
    for q0 in range(0, n_queries, queries_per_model):
        accs = []
        nq = min(queries_per_model, n_queries - q0)
        for k in range(nq):
            racy = rng.random() < racy_frac
            ca = int(rng.integers(0, G))
            cb = int(rng.integers(0, G))
            if cb == ca:
                cb = (ca + 1) % G
            base = int(rng.integers(0, 1 << 20)) * 4
            ea = c(base) + bid(0) * (2 * B) + tid(0) * 2
            eb = c(base) + bid(0) * (2 * B) + tid(0) * 2 + 1
            if racy:
                eb = eb + eq(bid(0), cb) * (2 * B * (ca - cb) - 1)
            accs.append(Access(0, WRITE, ea, name="overlap a"))
            accs.append(Access(0, WRITE, eb, name="overlap b"))
            pairs.append((len(models), 2 * k, 2 * k + 1, ALL_CLASSES))
        models.append(Model(0, [Array(GLOBAL, 32)], accs,
                            Launch((G, 1, 1), (B, 1, 1), 32), [[]],
                            name="overlap%d" % len(models)))
    return Workload(models, pairs, name="sparse_overlap", meta={"seed": seed, "G": G})


# ---------------------------------------------------------------------------
# mixed: many queries of log-uniform domain size

def mixed(seed=5005, n_queries=100000, log2_min=8, log2_max=28, racy_frac=0.10,
          queries_per_model=16, max_sets=64, self_frac=0.125):
    """Queries whose domain (points of one access over all its tuples) is
    log-uniform in [2^log2_min, 2^log2_max] (mean about 1.94e7 points for
    2^8..2^28, so about 3.9e12 evals for 100 000 queries); 2-D and 3-D
    launches; global and shared arrays half and half (a quarter of the global
    models on 64-bit arrays with bases of 2^33 and more); 1..max_sets
    distinct parameter tuples (W, N) per model derived from one host
    variable.  About racy_frac of the pairs are planted racy (a
    non-injective map on both sides); the others are race-free in one of
    three ways, a third each:

      * near miss by range: the second access is the first shifted by the
        exact size of its range (adjacent ranges, one element apart);
      * interleaved: 2 f and 2 f + 1 for an injective f (ranges overlap,
        residues differ);
      * own element: both accesses (or a self-pair) use the same injective
        map, so every address is reached by one point only and only a
        thread meets itself; no range or residue test decides these, the
        join has to run down to the thread level.

    Address forms are those of ``batched`` over the linear thread id, the
    linear block id and the loop variable.  Labels come from the oracle.
    meta["evals"] holds each pair's evals (box points of both sides over
    all tuples, a self-pair twice), known here from the launch constants.
    """
    rng = _rng(seed)
    models, pairs, evals = [], [], []
    lo, hi = np.log(2.0 ** log2_min), np.log(2.0 ** log2_max)
    q = 0
    while q < n_queries:
        nsets = int(rng.integers(1, max_sets + 1))
        D = float(np.exp(rng.uniform(lo, hi)))      # points per access, all tuples
        space = SHARED if len(models) % 2 == 1 else GLOBAL
        wide = space == GLOBAL and rng.random() < 0.25
        # block: 2-D or 3-D, 8..1024 threads
        bx = int(rng.choice([8, 16, 32, 64]))
        by = int(rng.choice([1, 2, 4, 8]))
        bz = int(rng.choice([1, 2, 4])) if rng.random() < 0.4 else 1
        while bx * by * bz > 1024:
            bz = max(1, bz // 2)
            by = max(1, by // 2)
        bt = bx * by * bz
        per_set = max(1.0, D / nsets)
        imax = int(np.clip(np.floor(np.log2(max(1.0, per_set / bt))), 0, 6))
        iters = 1 << int(rng.integers(0, imax + 1))
        nblk = max(1, int(round(per_set / (bt * iters))))
        three = rng.random() < 0.3 and nblk >= 8
        if three:
            gz = 1 << int(rng.integers(1, 3))
            gx = 1 << int(rng.integers(0, max(1, int(np.log2(nblk // gz)))))
            gy = max(1, int(round(nblk / (gx * gz))))
        elif rng.random() < 0.5 and nblk >= 4:
            gx = 1 << int(rng.integers(1, max(2, int(np.log2(nblk)))))
            gx = min(gx, nblk)
            gy, gz = max(1, int(round(nblk / gx))), 1
        else:
            gx, gy, gz = nblk, 1, 1
        nb = gx * gy * gz
        Ws = sorted(int(x) for x in rng.choice(
            _host_widths(bx, gx, max_sets), size=nsets, replace=False))
        sets = [[w, w * int(rng.integers(1, 5)) + bt // 2] for w in Ws]
        W, Np = param(0), param(1)
        tl = tid(0) + bdim(0) * (tid(1) + bdim(1) * tid(2))
        blin = bid(0) + c(gx) * (bid(1) + c(gy) * bid(2))
        gid = blin * bt + tl
        i = loop(0)
        rng_size = (nb if space == GLOBAL else 1) * bt * iters  # range of e_ok
        base = (1 << 33) + int(rng.integers(0, 1 << 20)) * (1 << 24) if wide else 0
        box = nb * bt * iters
        accs = []
        nq = min(queries_per_model, n_queries - q)
        for k in range(nq):
            racy = rng.random() < racy_frac
            selfp = rng.random() < self_frac
            form = int(rng.integers(0, 3))
            how = int(rng.integers(0, 3))
            guard = lt(tl, Np - int(rng.integers(0, 4))) if rng.random() < 0.3 else None
            if space == SHARED:
                e_ok = [tl * iters + i, tl + bt * i, tl * 2 + i * (2 * bt)][form]
                e_bad = [tl // 32 + i * 8, tl % W + i, tl * 2 + i][form]
            else:
                e_ok = [gid * iters + i, gid + c(nb * bt) * i,
                        blin * (bt * iters) + tl * iters + i][form]
                e_bad = [gid // 32 + i * 4, tl % W + blin * W + i, tl + i * 16][form]
            if base:
                e_ok, e_bad = c(base) + e_ok, c(base) + e_bad
            kinds = [(WRITE, WRITE), (WRITE, READ), (READ, WRITE)]
            ka, kb = kinds[int(rng.integers(0, 3))]
            if selfp:
                accs.append(Access(0, WRITE, e_bad if racy else e_ok, guard, [0]))
                a = len(accs) - 1
                pairs.append((len(models), a, a, ALL_CLASSES))
                evals.append(2 * nsets * box)
                continue
            if racy:
                ea, eb = e_bad, e_bad
            elif how == 0:
                ea, eb = e_ok, e_ok + rng_size
            elif how == 1:
                ea, eb = e_ok * 2 - c(base), e_ok * 2 - c(base) + 1
            else:
                ea, eb = e_ok, e_ok
            accs.append(Access(0, ka, ea, guard, [0]))
            accs.append(Access(0, kb, eb, guard, [0]))
            pairs.append((len(models), len(accs) - 2, len(accs) - 1, ALL_CLASSES))
            evals.append(2 * nsets * box)
        q += nq
        models.append(Model(2, [Array(space, 64 if wide else 32)], accs,
                            Launch((gx, gy, gz), (bx, by, bz), 32), sets,
                            loops=[Loop(0, "lt", iters, "add", 1)],
                            name="mixed%d" % len(models)))
    return Workload(models, pairs, name="mixed",
                    meta={"seed": seed, "log2": (log2_min, log2_max),
                          "evals": evals})


# ---------------------------------------------------------------------------
# synchronised workload: the mixed queries with acquire/release around them

def synced(seed=6006, n_queries=4000, log2_min=8, log2_max=22):
    """The mixed workload's queries (domains log-uniform in
    [2^log2_min, 2^log2_max] points per access) with each access guarded by
    one of the acquire/release patterns of section 6.5 (Figure 9) and
    appendix A, drawn per access:

      * a global lock L[0] at device scope (orders every pair);
      * a lock per block L[blockIdx.x] (orders pairs inside a block);
      * a lock by thread parity L[threadIdx.x % 2];
      * a block-scoped lock L[0] (too narrow for inter-block pairs);
      * a lock word in shared memory (one per block);
      * producer/consumer: a write releases flag F[blockIdx.x], a read
        acquires F[blockIdx.x] (or, one time in four, F[blockIdx.x + 1]);
      * nothing (a fifth of the accesses).

    Locks and flags live in two extra arrays of each model (global 64-bit,
    shared 32-bit).  meta["evals"] is the mixed workload's.
    """
    from .model import Sync
    from .expr import mod
    wl = mixed(seed=seed, n_queries=n_queries, log2_min=log2_min, log2_max=log2_max)
    rng = _rng(seed + 1)
    for m in wl.models:
        gl, sh = len(m.arrays), len(m.arrays) + 1
        m.arrays = m.arrays + [Array(GLOBAL, 64), Array(SHARED, 32)]
        for a in m.accesses:
            k = int(rng.integers(0, 8))
            dev, blk = "device", "block"
            lock = lambda arr, e, sc=dev: (Sync(arr, e, sc), Sync(arr, e, sc))
            if k == 0:
                a.acq, a.rel = lock(gl, c(0))
            elif k == 1:
                a.acq, a.rel = lock(gl, bid(0))
            elif k == 2:
                a.acq, a.rel = lock(gl, mod(tid(0), 2))
            elif k == 3:
                a.acq, a.rel = lock(gl, c(0), blk)
            elif k == 4:
                a.acq, a.rel = lock(sh, c(0), blk)
            elif k in (5, 6):
                off = 1 if rng.random() < 0.25 else 0
                if a.kind == WRITE:
                    a.rel = Sync(gl, bid(0), dev)
                else:
                    a.acq = Sync(gl, bid(0) + off, dev)
    wl.name = "synced"
    return wl
