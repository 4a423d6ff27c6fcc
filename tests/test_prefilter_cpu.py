"""The exact pre-filter (rd_options.prefilter) on the host, against the
oracle: every (pair, tuple) unit it decides must be race-free for every
class (the unit's accesses share no address), checked by running the oracle
on that unit alone with all classes enabled.  Also: the stress near misses
are all decided, and a one-element shift that makes them racy decides
none.  Host only (rd_prefilter_selftest touches no device)."""
import pytest

import oracle
import paper_2604_02106_amd as hg
from workloads import configs, c, tid, bid, bdim, loop, div
from workloads.model import (Workload, Model, Access, Array, Launch, Loop, ALL_CLASSES,
                             GLOBAL, WRITE, READ)
from workloads.random_models import rand_workload


def unit(wl, p, s):
    """Pair p of wl restricted to tuple s, all classes enabled."""
    m = wl.models[p[0]]
    m1 = Model(m.n_params, m.arrays, m.accesses, m.launch, [m.param_sets[s]],
               loops=m.loops, name=m.name)
    return Workload([m1], [(0, p[1], p[2], ALL_CLASSES)])


def decided_units(wl, which=1):
    """Units decided by the tests in bit mask `which` (1: address sets
    apart; 2: one thread-injective expression on both sides)."""
    pk = hg.Packed(wl)
    out = []
    for p in wl.pairs:
        if p[1] == p[2] and which == 1:
            continue
        for s in range(len(wl.models[p[0]].param_sets)):
            st, d = hg.prefilter_selftest(wl, p[0], p[1], p[2], s, packed=pk)
            assert st in (0, 2)
            if st == 0 and (d & which):
                out.append((p, s))
    return out


def test_decided_units_are_race_free():
    total = 0
    cases = [("rand %d" % k, rand_workload(k)) for k in range(24)]
    cases += [("batched", configs.batched(seed=96, n_models=24, scale=0.05, max_iters=8)),
              ("mixed", configs.mixed(seed=97, n_queries=128, log2_max=14))]
    for name, wl in cases:
        for p, s in decided_units(wl):
            want, _ = oracle.check_pairs(unit(wl, p, s), "A" if total < 40 else "B")
            r = want[0]
            assert r["status"] == 0 and r["verdict"] == 0 and r["count"] == 0, (name, p, s, r)
            total += 1
    assert total >= 20, total


def test_stress_near_misses_all_decided():
    wl = configs.stress(n_pairs=8, grid=1 << 8)
    got = decided_units(wl)
    assert len(got) == len(wl.pairs)
    for p, s in got[:2]:
        want, _ = oracle.check_pairs(unit(wl, p, s), "B")
        assert want[0]["verdict"] == 0


def test_shifted_near_misses_not_decided():
    wl = configs.stress(n_pairs=8, grid=1 << 7)
    m = wl.models[0]
    accs = list(m.accesses)
    for k in range(1, len(accs), 2):
        a = accs[k]
        d = 1 if (k // 2) % 2 == 0 else -1
        accs[k] = Access(a.array, a.kind, a.addr + c(d), a.guard, a.loops,
                         a.bint, a.wint, a.scope, a.name)
    m2 = Model(m.n_params, m.arrays, accs, m.launch, m.param_sets, loops=m.loops)
    wl2 = Workload([m2], wl.pairs)
    assert decided_units(wl2) == []


def test_injective_units_are_race_free():
    """Units decided because both accesses use one address expression that
    sends different threads to different addresses (self pairs included):
    the oracle finds each race-free with all classes on."""
    total = 0
    cases = [("rand %d" % k, rand_workload(k)) for k in range(24)]
    cases += [("batched", configs.batched(seed=98, n_models=24, scale=0.05, max_iters=8)),
              ("mixed", configs.mixed(seed=99, n_queries=160, log2_max=14))]
    for name, wl in cases:
        for p, s in decided_units(wl, 2):
            want, _ = oracle.check_pairs(unit(wl, p, s), "A" if total < 40 else "B")
            r = want[0]
            assert r["status"] == 0 and r["verdict"] == 0 and r["count"] == 0, (name, p, s, r)
            total += 1
    assert total >= 20, total


def _one(addr, block, grid=(4, 1, 1), iters=1):
    loops = [Loop(0, "lt", iters)] if iters > 1 else []
    m = Model(0, [Array(GLOBAL, 32)],
              [Access(0, WRITE, addr, None, [0] if iters > 1 else []),
               Access(0, READ, addr, None, [0] if iters > 1 else [])],
              Launch(grid, block, 32), [[]], loops=loops)
    return Workload([m], [(0, 0, 0, ALL_CLASSES), (0, 0, 1, ALL_CLASSES)])


@pytest.mark.parametrize("name,addr,block,grid,iters,decided", [
    ("tid", tid(), (64, 1, 1), (1, 1, 1), 1, True),
    ("tid/2", div(tid(), c(2)), (64, 1, 1), (1, 1, 1), 1, False),
    ("tid+32 bid, B=32", tid() + bid() * 32, (32, 1, 1), (4, 1, 1), 1, True),
    ("tid+32 bid, B=64", tid() + bid() * 32, (64, 1, 1), (4, 1, 1), 1, False),
    ("2-D row-major", tid(0) + tid(1) * 16 + bid() * 256, (16, 16, 1), (3, 1, 1), 1, True),
    ("2-D too narrow", tid(0) + tid(1) * 8, (16, 4, 1), (1, 1, 1), 1, False),
    ("same address every iteration", tid() + loop(0) * 0, (64, 1, 1), (2, 1, 1), 4, False),
    ("grid stride", tid() + bid() * 64 + loop(0) * 256, (64, 1, 1), (4, 1, 1), 4, True),
    ("iteration below thread", tid() * 4 + loop(0), (64, 1, 1), (1, 1, 1), 4, True),
    ("iteration overlaps threads", tid() + loop(0) * 16, (64, 1, 1), (1, 1, 1), 4, False),
])
def test_injectivity_cases(name, addr, block, grid, iters, decided):
    """Hand-made address maps: the dependence test decides exactly the
    thread-injective ones; the oracle confirms the decided ones race-free
    and finds the others racy."""
    wl = _one(addr, block, grid, iters)
    got = decided_units(wl, 2)
    want, _ = oracle.check_pairs(wl, "A")
    assert (len(got) == 2) == decided, (name, got)
    if decided:
        assert all(r["count"] == 0 for r in want), name
    elif name != "same address every iteration":
        assert all(r["verdict"] == 1 for r in want), (name, want)
