"""Race-free throughput stress (128 pairs, 2^30 points per access, int64
addresses, strided and blocked near-miss patterns): at full size the exact
answer is known by construction (every count 0, every status OK, evals
2^31 per pair); a reduced grid of the same generator is compared with the
oracle field by field, and a one-element shift that makes pairs racy is
checked against the oracle too."""
import sys

import pytest

import oracle
from workloads import configs, c
from workloads.model import Workload, Model, Access

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hg():
    import torch
    assert torch.cuda.is_available()
    import paper_2604_02106_amd as hg
    hg.default_context()
    return hg


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def test_stress_reduced_grid_matches_oracle(hg):
    wl = configs.stress(n_pairs=16, grid=1 << 8)
    say("stress reduced", len(wl.pairs))
    got = hg.check_pairs(wl)
    want, _ = oracle.check_pairs(wl, "B", threads=8)
    assert got == want
    assert all(r["verdict"] == 0 for r in got)


def test_stress_near_miss_shifted_is_racy(hg):
    """Shift side b of every pair by one element onto side a: strided pairs
    (2f + 1 -> 2f + 2, the next thread's element) forward, blocked pairs
    (the range after side a's) back.  The near misses become conflicts;
    counts and witnesses equal the oracle's."""
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
    say("stress shifted")
    got = hg.check_pairs(wl2)
    want, _ = oracle.check_pairs(wl2, "B", threads=8)
    assert got == want
    assert all(r["verdict"] == 1 for r in got)


def test_stress_full_size(hg):
    """All 128 pairs at 2^30 points per access (2.75e11 evals)."""
    wl = configs.stress()
    say("stress full", len(wl.pairs), wl.meta["points_per_access"])
    got = hg.check_pairs(wl)
    for r in got:
        assert r["status"] == 0 and r["verdict"] == 0 and r["count"] == 0, r
        assert r["witness"] == (-1,) * 7
        assert r["evals"] == 2 * (1 << 30)


def test_stress_prefilter_decides_near_misses(hg):
    """Exact pre-filters: strided near misses (2f against 2f + 1) share no
    residue modulo 2; blocked ones interleave block by block over one
    address range, and their per-block intervals miss each other.  With
    the pre-filter on every (pair, tuple) unit is decided without
    enumeration, and every field stays equal to the oracle's.  The shifted
    (racy) variant keeps every unit (residues and intervals then meet) and
    equals the oracle's too."""
    wl = configs.stress(n_pairs=16, grid=1 << 8)
    units = sum(len(wl.models[p[0]].param_sets) for p in wl.pairs)
    say("stress pre-filtered", len(wl.pairs), "units", units)
    got = hg.check_pairs(wl, prefilter=1)
    want, _ = oracle.check_pairs(wl, "B", threads=8)
    assert got == want
    assert hg.default_context().stats()["prefiltered"] == units
    m = wl.models[0]
    accs = list(m.accesses)
    for k in range(1, len(accs), 2):
        a = accs[k]
        d = 1 if (k // 2) % 2 == 0 else -1
        accs[k] = Access(a.array, a.kind, a.addr + c(d), a.guard, a.loops,
                         a.bint, a.wint, a.scope, a.name)
    m2 = Model(m.n_params, m.arrays, accs, m.launch, m.param_sets, loops=m.loops)
    wl2 = Workload([m2], wl.pairs)
    say("stress shifted pre-filtered")
    got = hg.check_pairs(wl2, prefilter=1)
    want, _ = oracle.check_pairs(wl2, "B", threads=8)
    assert got == want
    assert hg.default_context().stats()["prefiltered"] == 0
