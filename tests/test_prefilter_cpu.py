"""The exact pre-filter (rd_options.prefilter) on the host, against the
oracle: every (pair, tuple) unit it decides must be race-free for every
class (the unit's accesses share no address), checked by running the oracle
on that unit alone with all classes enabled.  Also: the stress near misses
are all decided, and a one-element shift that makes them racy decides
none.  Host only (rd_prefilter_selftest touches no device)."""
import pytest

import oracle
import paper_2604_02106_amd as hg
from workloads import configs, c
from workloads.model import Workload, Model, Access, ALL_CLASSES
from workloads.random_models import rand_workload


def unit(wl, p, s):
    """Pair p of wl restricted to tuple s, all classes enabled."""
    m = wl.models[p[0]]
    m1 = Model(m.n_params, m.arrays, m.accesses, m.launch, [m.param_sets[s]],
               loops=m.loops, name=m.name)
    return Workload([m1], [(0, p[1], p[2], ALL_CLASSES)])


def decided_units(wl):
    pk = hg.Packed(wl)
    out = []
    for p in wl.pairs:
        if p[1] == p[2]:
            continue
        for s in range(len(wl.models[p[0]].param_sets)):
            st, d = hg.prefilter_selftest(wl, p[0], p[1], p[2], s, packed=pk)
            assert st in (0, 2)
            if st == 0 and d:
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
