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
