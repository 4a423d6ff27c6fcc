"""Pins of the oracle's synchronisation-aware query (section 6.5, Figure 9,
Table 2's highlighted constraint; appendix A, Figure 10) to closed forms
derived by hand.

Launch: G blocks of B threads, warp w, one tuple.  Without synchronisation,
every thread writing one address gives, in ordered pairs of distinct threads,
    inter = G (G - 1) B^2,  intra-block = G B (B - w),  intra-warp = G B (w - 1).
Each case below states which of these pairs the acquire/release removes.
"""
import copy

import pytest

import oracle
from workloads import (c, tid, bid, loop, mod, eq, lor, Model, Workload, Access,
                       Sync, Array, Launch, Loop, GLOBAL, SHARED, READ, WRITE,
                       ATOMIC, SCOPE_BLOCK, SCOPE_DEVICE, INTRA_WARP)
from workloads.random_models import rand_sync_workload

DEV, BLK = SCOPE_DEVICE, SCOPE_BLOCK
# arrays: 0 data (global), 1 locks and flags (global), 2 locks (shared)
ARRAYS = [Array(GLOBAL, 64), Array(GLOBAL, 64), Array(SHARED, 32)]


def both(wl):
    ra = oracle.check_pairs(wl, "A", threads=4)[0]
    rb = oracle.check_pairs(wl, "B", threads=4)[0]
    assert ra == rb
    return ra


def run(accs, pairs, G, B, w, loops=()):
    m = Model(0, ARRAYS, accs, Launch((G, 1, 1), (B, 1, 1), w), [[]], loops=loops)
    return both(Workload([m], [(0, a, b, 7) for (a, b) in pairs]))


def full(G, B, w):
    return [G * (G - 1) * B * B, G * B * (B - w), G * B * (w - 1)]


def lock(addr, arr=1, sa=DEV, sr=DEV):
    return dict(acq=Sync(arr, addr, sa), rel=Sync(arr, addr, sr))


GBW = [(4, 16, 4), (3, 8, 2), (2, 32, 8)]


@pytest.mark.parametrize("G,B,w", GBW)
def test_global_lock_removes_every_race(G, B, w):
    """lock(L[0]) at device scope around A[0] = ...: syn is the lock for
    every thread, one address, so no pair races."""
    r = run([Access(0, WRITE, c(0)), Access(0, WRITE, c(0), **lock(c(0)))],
            [(0, 0), (1, 1)], G, B, w)
    assert r[0]["by_class"] == full(G, B, w)
    assert r[1]["by_class"] == [0, 0, 0] and r[1]["verdict"] == 0
    assert r[1]["witness"] == (-1,) * 7


@pytest.mark.parametrize("G,B,w", GBW)
def test_block_scoped_lock_leaves_inter_block_races(G, B, w):
    """A block-scoped lock: device scope is required for an inter-block
    conflict, so those all remain; intra-block and intra-warp go."""
    r = run([Access(0, WRITE, c(0), **lock(c(0), sa=BLK, sr=BLK))], [(0, 0)], G, B, w)
    assert r[0]["by_class"] == [G * (G - 1) * B * B, 0, 0]


@pytest.mark.parametrize("G,B,w", GBW)
def test_per_block_lock(G, B, w):
    """lock(L[blockIdx]): threads of two blocks take different locks."""
    r = run([Access(0, WRITE, c(0), **lock(bid()))], [(0, 0)], G, B, w)
    assert r[0]["by_class"] == [G * (G - 1) * B * B, 0, 0]


@pytest.mark.parametrize("G,B,w", GBW)
def test_shared_memory_lock_is_per_block(G, B, w):
    """A lock word in shared memory exists once per block: at device scope it
    still orders nothing across blocks."""
    r = run([Access(0, WRITE, c(0), **lock(c(0), arr=2))], [(0, 0)], G, B, w)
    assert r[0]["by_class"] == [G * (G - 1) * B * B, 0, 0]


@pytest.mark.parametrize("G,B,w", GBW)
def test_lock_by_thread_parity(G, B, w):
    """lock(L[tid % 2]) with B and w even: exactly the pairs of different
    parity race.  For a thread, half of the B threads of another block, half
    of the B - w threads of the other warps and w / 2 threads of its own warp
    have the other parity."""
    r = run([Access(0, WRITE, c(0), **lock(mod(tid(), 2)))], [(0, 0)], G, B, w)
    assert r[0]["by_class"] == [G * (G - 1) * B * B // 2, G * B * (B - w) // 2,
                                G * B * w // 2]


@pytest.mark.parametrize("G,B,w,n", [(2, 8, 4, 3), (3, 4, 2, 2)])
def test_lock_per_iteration(G, B, w, n):
    """Every thread writes A[0] in each of n iterations under lock(L[i]):
    two points race exactly when their iterations differ, n (n - 1) of the
    n^2 ordered iteration pairs of two threads."""
    r = run([Access(0, WRITE, c(0), loops=[0], **lock(loop(0)))], [(0, 0)], G, B, w,
            loops=[Loop(0, "lt", n)])
    assert r[0]["by_class"] == [x * n * (n - 1) for x in full(G, B, w)]


@pytest.mark.parametrize("G,B,w", GBW)
def test_producer_consumer(G, B, w):
    """Thread 0 of each block writes X[b] then releases F[b]; every thread
    acquires a flag then reads X[b].  Without synchronisation the writer
    conflicts with the B - 1 readers of its block (w - 1 in its warp).  A
    reader acquiring F[b] removes all; one acquiring F[0] only block 0's.
    Witness then: p = writer of block 1, q = its thread 1, intra-warp."""
    W = Access(0, WRITE, bid(), guard=eq(tid(), 0), rel=Sync(1, bid(), DEV))
    R_ok = Access(0, READ, bid(), acq=Sync(1, bid(), DEV))
    R_bad = Access(0, READ, bid(), acq=Sync(1, c(0), DEV))
    R_none = Access(0, READ, bid())
    r = run([W, R_ok, R_bad, R_none], [(0, 1), (0, 2), (0, 3)], G, B, w)
    assert r[2]["by_class"] == [0, G * (B - w), G * (w - 1)]
    assert r[0]["by_class"] == [0, 0, 0]
    assert r[1]["by_class"] == [0, (G - 1) * (B - w), (G - 1) * (w - 1)]
    assert r[1]["witness"] == (0, 1, 0, 0, 1, 1, 0)
    assert r[1]["w_addr"] == 1 and r[1]["witness_class"] == INTRA_WARP


@pytest.mark.parametrize("G,B,w", GBW)
def test_mismatched_acquire_release(G, B, w):
    """A write between acquire F[b] and release F[b + 1] is no lock (the
    addresses differ), so its syn is the release F[b + 1]: a reader that
    acquires F[b + 1] is ordered after it, one that acquires F[b] is not."""
    W = Access(0, WRITE, bid(), guard=eq(tid(), 0), acq=Sync(1, bid(), DEV),
               rel=Sync(1, bid() + 1, DEV))
    R1 = Access(0, READ, bid(), acq=Sync(1, bid() + 1, DEV))
    R2 = Access(0, READ, bid(), acq=Sync(1, bid(), DEV))
    r = run([W, R1, R2], [(0, 1), (0, 2)], G, B, w)
    assert r[0]["by_class"] == [0, 0, 0]
    assert r[1]["by_class"] == [0, G * (B - w), G * (w - 1)]


@pytest.mark.parametrize("G,B,w", GBW)
def test_atomic_needs_a_lock(G, B, w):
    """An atomic is neither producer nor consumer: only a matching lock
    gives it a syn.  With acquire L[0] and release L[1] every pair with the
    locked write races; with lock(L[0]) none does."""
    Wl = Access(0, WRITE, c(0), **lock(c(0)))
    At_bad = Access(0, ATOMIC, c(0), acq=Sync(1, c(0), DEV), rel=Sync(1, c(1), DEV))
    At_ok = Access(0, ATOMIC, c(0), **lock(c(0)))
    r = run([Wl, At_bad, At_ok], [(0, 1), (0, 2)], G, B, w)
    assert r[0]["by_class"] == full(G, B, w)
    assert r[1]["by_class"] == [0, 0, 0]


@pytest.mark.parametrize("G,B,w", GBW)
def test_scope_filter_before_the_lock_test(G, B, w):
    """Acquire at device scope, release at block scope (appendix A, Figure
    10: an operation narrower than the required scope is not seen).  For an
    inter-block conflict only the acquire is seen: the write has no syn and
    races, the read's syn is the acquire.  At block scope both are seen and
    form a lock, so intra-block and intra-warp conflicts go."""
    kw = lock(c(0), sa=DEV, sr=BLK)
    W, R = Access(0, WRITE, c(0), **kw), Access(0, READ, c(0), **kw)
    r = run([W, R], [(0, 1), (0, 0)], G, B, w)
    assert r[0]["by_class"] == [G * (G - 1) * B * B, 0, 0]
    assert r[1]["by_class"] == [G * (G - 1) * B * B, 0, 0]
    # device-scoped release, block-scoped acquire: for inter-block conflicts
    # a write's syn is its release, so two such writes are ordered
    W2 = Access(0, WRITE, c(0), **lock(c(0), sa=BLK, sr=DEV))
    r = run([W2], [(0, 0)], G, B, w)
    assert r[0]["by_class"] == [0, 0, 0]


def test_locks_in_different_arrays_never_match():
    """lock(L1[0]) against lock(L2[0]): equal indices in two arrays are two
    locks."""
    G, B, w = 2, 8, 4
    arrays = ARRAYS + [Array(GLOBAL, 64)]
    m = Model(0, arrays, [Access(0, WRITE, c(0), **lock(c(0), arr=1)),
                          Access(0, WRITE, c(0), **lock(c(0), arr=3))],
              Launch((G, 1, 1), (B, 1, 1), w), [[]])
    r = both(Workload([m], [(0, 0, 1, 7), (0, 0, 0, 7)]))
    assert r[0]["by_class"] == full(G, B, w)
    assert r[1]["by_class"] == [0, 0, 0]


def test_sync_statuses():
    """A bad lock array is malformed; errors in a synchronisation address
    count like address errors (only where the guard holds)."""
    G, B, w = 1, 4, 2
    bad = Access(0, WRITE, c(0), acq=Sync(7, c(0), DEV))
    div0 = Access(0, WRITE, c(0), acq=Sync(1, tid() // (tid() - 1), DEV))
    guarded = Access(0, WRITE, c(0), guard=lor(eq(tid(), 0), eq(tid(), 2)),
                     acq=Sync(1, tid() // (tid() - 1), DEV))
    m = Model(0, ARRAYS, [bad, div0, guarded], Launch((G, 1, 1), (B, 1, 1), w), [[]])
    r = both(Workload([m], [(0, 0, 0, 7), (0, 1, 1, 7), (0, 2, 2, 7)]))
    assert r[0]["status"] == -1
    assert r[1]["status"] == -4
    assert r[2]["status"] == 0 and r[2]["by_class"] == [0, 2, 0]  # no release: no syn


def _strip(wl):
    w2 = copy.deepcopy(wl)
    for m in w2.models:
        for a in m.accesses:
            a.acq = a.rel = None
    return w2


@pytest.mark.parametrize("seed", range(24))
def test_methods_agree_random_sync(seed):
    """Oracle-A (the predicate per point pair) against Oracle-B (group sums
    with the synchronisation key), and synchronisation only removes pairs."""
    wl = rand_sync_workload(seed)
    ra = both(wl)
    rn = oracle.check_pairs(_strip(wl), "B", threads=4)[0]
    for x, y in zip(ra, rn):
        if x["status"] or y["status"]:
            continue
        assert all(a <= b for a, b in zip(x["by_class"], y["by_class"]))


def test_random_sync_models_exercise_exclusion():
    removed = 0
    for seed in range(24):
        wl = rand_sync_workload(seed)
        ra = oracle.check_pairs(wl, "B", threads=4)[0]
        rn = oracle.check_pairs(_strip(wl), "B", threads=4)[0]
        removed += sum(1 for x, y in zip(ra, rn)
                       if x["status"] == 0 and y["status"] == 0 and x["count"] < y["count"])
    assert removed >= 20
