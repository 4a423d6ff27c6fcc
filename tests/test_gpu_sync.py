"""Synchronisation-aware query on the GPU (section 6.5, Figure 9, Table 2;
appendix A, Figure 10) against the CPU oracle, field by field: the
hand-pinned lock and producer/consumer models, random models with random
acquires and releases, synchronised pairs batched with plain ones, and
launches large enough to span many fallback tiles and chunks.

Every case prints its name before it runs.  All inputs are seeded.
"""
import sys

import pytest

import oracle
from workloads import (c, tid, bid, loop, mod, eq, lt, Model, Workload, Access,
                       Sync, Array, Launch, Loop, GLOBAL, SHARED, READ, WRITE,
                       ATOMIC, SCOPE_BLOCK, SCOPE_DEVICE)
from workloads.random_models import rand_sync_workload, rand_workload

pytestmark = pytest.mark.gpu

DEV, BLK = SCOPE_DEVICE, SCOPE_BLOCK
ARRAYS = [Array(GLOBAL, 64), Array(GLOBAL, 64), Array(SHARED, 32), Array(GLOBAL, 32)]


@pytest.fixture(scope="module")
def hg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2604_02106_amd as hg
    hg.default_context()
    return hg


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def run_both(hg, wl, name, **kw):
    say(name, "pairs=%d" % len(wl.pairs), kw)
    got = hg.check_pairs(wl, **kw)
    want, _ = oracle.check_pairs(wl, "B", threads=8)
    assert len(got) == len(want)
    for k, (g, w) in enumerate(zip(got, want)):
        assert g == w, "%s pair %d:\n gpu    %r\n oracle %r" % (name, k, g, w)
    return got


def lock(addr, arr=1, sa=DEV, sr=DEV):
    return dict(acq=Sync(arr, addr, sa), rel=Sync(arr, addr, sr))


def pin_models(G, B, w):
    """The closed-form models of the oracle's synchronisation pins."""
    accs = [
        Access(0, WRITE, c(0)),                                          # 0
        Access(0, WRITE, c(0), **lock(c(0))),                            # 1
        Access(0, WRITE, c(0), **lock(c(0), sa=BLK, sr=BLK)),            # 2
        Access(0, WRITE, c(0), **lock(bid())),                           # 3
        Access(0, WRITE, c(0), **lock(c(0), arr=2)),                     # 4
        Access(0, WRITE, c(0), **lock(mod(tid(), 2))),                   # 5
        Access(0, WRITE, bid(), guard=eq(tid(), 0), rel=Sync(1, bid(), DEV)),  # 6
        Access(0, READ, bid(), acq=Sync(1, bid(), DEV)),                 # 7
        Access(0, READ, bid(), acq=Sync(1, c(0), DEV)),                  # 8
        Access(0, WRITE, c(0), **lock(c(0), sa=DEV, sr=BLK)),            # 9
        Access(0, READ, c(0), **lock(c(0), sa=DEV, sr=BLK)),             # 10
        Access(0, ATOMIC, c(0), acq=Sync(1, c(0), DEV), rel=Sync(1, c(1), DEV)),  # 11
        Access(0, WRITE, c(0), **lock(c(0), sa=BLK, sr=DEV)),            # 12
        Access(0, WRITE, c(0), **lock(c(0), arr=3)),                     # 13
    ]
    m = Model(0, ARRAYS, accs, Launch((G, 1, 1), (B, 1, 1), w), [[]])
    pairs = [(0, 0), (1, 1), (2, 2), (3, 3), (4, 4), (5, 5), (6, 7), (6, 8),
             (9, 10), (9, 9), (1, 11), (12, 12), (1, 13)]
    return Workload([m], [(0, a, b, 7) for (a, b) in pairs])


@pytest.fixture(params=["lds", "fallback"])
def sync_path(request, monkeypatch):
    """Synchronised units through the LDS joins (those that qualify) or
    all through the HBM aggregation path."""
    if request.param == "fallback":
        monkeypatch.setenv("HGRD_SYNC_FALLBACK", "1")
    return request.param


@pytest.mark.parametrize("G,B,w", [(4, 16, 4), (3, 8, 2), (2, 32, 8), (40, 256, 32)])
def test_sync_pins(hg, G, B, w, sync_path):
    got = run_both(hg, pin_models(G, B, w), "sync pins G=%d B=%d w=%d %s" % (G, B, w, sync_path))
    full = [G * (G - 1) * B * B, G * B * (B - w), G * B * (w - 1)]
    assert got[0]["by_class"] == full
    assert got[1]["by_class"] == [0, 0, 0]
    assert got[2]["by_class"] == [full[0], 0, 0]
    assert got[5]["by_class"] == [full[0] // 2, G * B * (B - w) // 2, G * B * w // 2]
    assert got[7]["by_class"] == [0, (G - 1) * (B - w), (G - 1) * (w - 1)]
    assert got[7]["witness"] == (0, 1, 0, 0, 1, 1, 0)
    st = hg.default_context().stats()
    say("sync records", st["sync_records"], "hbm items", st["hbm_items"])
    if sync_path == "fallback":
        assert st["sync_records"] > 0
    else:
        assert st["sync_records"] == 0 and st["hbm_items"] > 0


def test_sync_every_level_and_pass(hg, sync_path):
    """Every level of the LDS join computed (barrier and warp-barrier
    interval ids that change with the iteration, so no level repeats the
    previous one), all three classes asked, and device- and block-scope
    acquires and releases on the records, so a synchronisation pass follows
    each level: the join uses its most table generations; every field
    equals the oracle's."""
    loops = [Loop(0, "lt", 3)]
    iv = dict(loops=[0], bint=loop(0), wint=loop(0) * 2 + 1)
    accs = [
        Access(0, WRITE, tid() % 16, **iv, **lock(mod(tid(), 2))),                  # 0
        Access(0, READ, tid() % 16, **iv, **lock(c(0), sa=BLK, sr=BLK)),            # 1
        Access(0, WRITE, (tid() + 1) % 16, **iv, **lock(mod(tid(), 2), sa=DEV, sr=BLK)),  # 2
    ]
    m = Model(0, ARRAYS, accs, Launch((6, 1, 1), (64, 1, 1), 16), [[]], loops=loops)
    wl = Workload([m], [(0, 0, 0, 7), (0, 0, 1, 7), (0, 1, 2, 7), (0, 0, 2, 7), (0, 2, 2, 7)])
    got = run_both(hg, wl, "sync every level %s" % sync_path)
    # threads 16 apart share an address and a parity lock: no race in (0, 0)
    assert got[0]["verdict"] == 0 and all(r["verdict"] for r in got[1:])
    st = hg.default_context().stats()
    say("sync records", st["sync_records"], "hbm items", st["hbm_items"])
    if sync_path == "lds":
        assert st["sync_records"] == 0 and st["hbm_items"] > 0


@pytest.mark.parametrize("seed", range(30))
def test_sync_random(hg, seed, sync_path):
    run_both(hg, rand_sync_workload(seed), "sync rand seed=%d %s" % (seed, sync_path))


def test_sync_batched_with_plain_pairs(hg, sync_path):
    """Synchronised and plain pairs in one call: each goes its own way and
    the results are the oracle's."""
    models, pairs = [], []
    for seed in range(200, 216):
        wl = rand_sync_workload(seed) if seed % 2 else rand_workload(seed)
        base = len(models)
        models += wl.models
        pairs += [(m + base, a, b, k) for (m, a, b, k) in wl.pairs]
    run_both(hg, Workload(models, pairs), "sync batch")


def test_sync_large(hg, sync_path):
    """Launches of tens of thousands of points per side, with loops and
    barrier-interval ids: lock by thread parity inside a loop, a lock per
    iteration, producer/consumer with the consumer on the wrong flag in
    every eighth block, and a shared-memory array with block-scoped locks."""
    loops = [Loop(0, "lt", 4), Loop(0, "lt", 3)]
    arrays = ARRAYS + [Array(SHARED, 64)]
    accs = [
        Access(0, WRITE, tid() % 64, loops=[0], bint=loop(0) % 2,
               **lock(mod(tid(), 2))),                                      # 0
        Access(0, WRITE, c(7), loops=[1], wint=loop(1), **lock(loop(1))),    # 1
        Access(0, WRITE, bid(), guard=lt(tid(), 2), rel=Sync(1, bid(), DEV)),  # 2
        Access(0, READ, bid(), acq=Sync(1, bid() + eq(mod(bid(), 8), 3) * 1000,
                                        DEV)),                              # 3
        Access(4, WRITE, tid() // 4, **lock(tid() // 8, arr=2, sa=BLK, sr=BLK)),  # 4
        Access(4, READ, tid() // 4 + 1, acq=Sync(2, tid() // 8, BLK)),        # 5
    ]
    m = Model(0, arrays, accs, Launch((96, 1, 1), (256, 1, 1), 32), [[]], loops=loops)
    wl = Workload([m], [(0, 0, 0, 7), (0, 1, 1, 7), (0, 2, 3, 7), (0, 4, 4, 7),
                        (0, 4, 5, 7), (0, 0, 1, 7)])
    got = run_both(hg, wl, "sync large %s" % sync_path)
    assert all(r["status"] == 0 for r in got)
    assert sum(r["verdict"] for r in got) >= 3


def test_sync_verdict_mode_is_exact(hg):
    """VERDICT mode leaves synchronised pairs (all but the first) to the
    exact path."""
    wl = pin_models(8, 64, 32)
    say("sync verdict", "pairs=%d" % len(wl.pairs))
    want = hg.check_pairs(wl)
    got = hg.check_pairs(wl, mode=hg.MODE_VERDICT, order=hg.ORDER_INTERVAL)
    assert got[1:] == want[1:]


def test_sync_statuses(hg):
    """Errors in synchronisation addresses reach the pair's status: a zero
    divisor where the guard holds, a 32-bit lock array overflowed, and a
    lock array index out of range."""
    accs = [
        Access(0, WRITE, c(0), acq=Sync(1, tid() // (tid() - 1), DEV)),
        Access(0, WRITE, c(0), **lock(tid() * (1 << 40), arr=3)),
        Access(0, WRITE, c(0), acq=Sync(9, c(0), DEV)),
        Access(0, WRITE, c(0), guard=eq(tid(), 0),
               acq=Sync(1, tid() // (tid() - 1), DEV)),
    ]
    m = Model(0, ARRAYS, accs, Launch((2, 1, 1), (8, 1, 1), 4), [[]])
    got = run_both(hg, Workload([m], [(0, k, k, 7) for k in range(4)]), "sync statuses")
    assert [r["status"] for r in got] == [-4, -3, -1, 0]


def test_sync_units_decided_without_a_join(hg):
    """Synchronised units whose accesses share no address (ranges apart) or
    use one thread-injective address are decided before any join when every
    expression is proven error-free; a lock address that may divide by zero
    keeps its unit on the join path (its error must be found)."""
    B = 64
    gid = tid() + bid() * B
    accs = [
        Access(0, WRITE, gid, **lock(c(0))),                        # 0
        Access(0, READ, gid + 100000, **lock(c(0))),                # 1: apart from 0
        Access(0, WRITE, gid, **lock(tid() // (tid() - 3))),        # 2: may fail
        Access(0, WRITE, gid * 2, **lock(mod(tid(), 2))),           # 3: injective
    ]
    m = Model(0, ARRAYS, accs, Launch((16, 1, 1), (B, 1, 1), 32), [[]])
    wl = Workload([m], [(0, 0, 1, 7), (0, 3, 3, 7), (0, 2, 2, 7), (0, 0, 0, 7)])
    got = run_both(hg, wl, "sync decided")
    assert [r["status"] for r in got] == [0, 0, -4, 0]
    st = hg.default_context().stats()
    say("sync decided", st["sync_decided"], "sync records", st["sync_records"])
    assert st["sync_decided"] >= 3
