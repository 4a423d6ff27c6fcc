"""Term-table lowering, checked on the host: for every access and tuple of
the seeded workloads, tables built as the device builds them must give the
interpreter's guard, address and interval ids at every point of the launch
box (sampled for the largest boxes)."""
import pytest

import paper_2604_02106_amd as hg
from workloads import configs, families as F
from workloads.random_models import rand_workload


def sweep(wl, max_points=0):
    pk = hg.Packed(wl)
    stats = {0: 0, 1: 0, 2: 0}
    for mi, m in enumerate(wl.models):
        for a in range(len(m.accesses)):
            for s in range(len(m.param_sets)):
                st, n = hg.table_selftest(wl, mi, a, s, max_points, packed=pk)
                assert st in (0, 1, 2), (wl.name, mi, a, s, st)
                stats[st] += 1
    return stats


@pytest.mark.parametrize("seed", range(0, 60))
def test_random_models(seed):
    sweep(rand_workload(seed))


def test_tiny_and_families():
    st = sweep(configs.tiny())
    assert st[0] == sum(st.values())  # affine: every access qualifies
    for m in (F.f1_neighbour(40, 128, 32), F.f2_tree_reduction(256),
              F.f3_stride_mod(1024, (16, 3)), F.f4_guard_halves(64, extra=1)):
        sweep(F.single(m, 0, 0))


def test_paper_examples():
    for m in (F.k1_copy_upp_low([[16, 16], [32, 1]]), F.k2_reduce_final([[1], [7]]),
              F.k3_tone_mapping([[16, 1, 2], [32, 2, 2]]),
              F.k4_lud_internal([[64, 0], [64, -47]]), F.k5_shift([[512], [0], [3]])):
        sweep(F.single(m, 0, 0))


def test_batched_models_mostly_tabulated():
    wl = configs.batched(seed=2002, n_models=24, scale=0.05, max_iters=8)
    st = sweep(wl)
    assert st[0] >= 0.8 * (st[0] + st[1]), st


def test_stress_and_sparse_sampled():
    st = sweep(configs.stress(n_pairs=4, grid=1 << 16), max_points=1 << 16)
    assert st[1] == 0 and st[0] == 8
    st = sweep(configs.sparse(seed=5, n_queries=16, G=256, B=256,
                              queries_per_model=16), max_points=1 << 15)
    assert st[1] == 0


def test_mixed_models():
    st = sweep(configs.mixed(seed=5005, n_queries=96, log2_max=16), max_points=1 << 14)
    assert st[0] >= 0.8 * (st[0] + st[1]), st


def test_division_splits():
    """Truncating divisions and remainders of sums that mix groups: every
    form below must qualify for tables (status 0) and agree with the
    interpreter at every box point."""
    from workloads import (Access, Array, Launch, Loop, Model, Workload, GLOBAL,
                           WRITE, tid, bid, loop, c, param)
    gid8 = bid(0) * 8 + tid(0)          # block of 8: 8 * bid is a multiple of 8
    gid96 = (bid(0) + bid(1) * 3) * 96 + tid(0)
    exprs = [gid8 // 32, gid8 % 32, gid8 // 4, gid8 % 8,       # small-rest rule
             gid96 // 32, gid96 % 32,                            # divisor rule
             (bid(0) * 64 + tid(0) * 8 + loop(0)) // 8,          # two groups, rest
             (loop(0) * 16 + tid(0)) // 16 + param(0),
             (bid(0) * 64 + tid(0) * 2 + loop(0)) // 8]          # rest of two groups
    accs = [Access(0, WRITE, e, None, [0]) for e in exprs]
    m = Model(1, [Array(GLOBAL, 32)], accs, Launch((6, 2, 1), (8, 1, 1), 32),
              [[3], [7]], loops=[Loop(0, "lt", 4)])
    wl = Workload([m], [(0, k, k, 7) for k in range(len(accs))])
    pk = hg.Packed(wl)
    for a in range(len(accs)):
        for s in range(2):
            st, n = hg.table_selftest(wl, 0, a, s, packed=pk)
            if a == len(accs) - 1:
                assert st == 1  # no split: the interpreter keeps it
                continue
            assert st == 0 and n == 6 * 2 * 8 * 4, (a, s, st, n)
