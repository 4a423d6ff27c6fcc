"""GPU path against the CPU oracle, field by field (EXACT mode is bit-exact:
statuses, verdicts, per-class u64 counts, lexicographically smallest witness,
witness class and address, evals).

Every case prints its name before it runs so a failing device step names its
case.  All inputs are seeded.
"""
import sys

import pytest

import oracle
from workloads import (Access, Array, Launch, Loop, Model, Workload, c, param, emin,
                       tid, bid, bdim, loop, div, lt, GLOBAL, SHARED, WRITE,
                       READ, ATOMIC, SCOPE_BLOCK)
from workloads import families as F, configs
from workloads.random_models import rand_workload

pytestmark = pytest.mark.gpu

I64MAX = (1 << 63) - 1


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


def compare(got, want, name=""):
    assert len(got) == len(want)
    for k, (g, w) in enumerate(zip(got, want)):
        assert g == w, "%s pair %d:\n gpu    %r\n oracle %r" % (name, k, g, w)


def run_both(hg, wl, name, **kw):
    say(name, "pairs=%d" % len(wl.pairs), kw)
    got = hg.check_pairs(wl, **kw)
    want, _ = oracle.check_pairs(wl, "B", threads=8)
    compare(got, want, name)
    return got


def test_tiny_config(hg):
    wl = configs.tiny()
    got = run_both(hg, wl, "tiny")
    assert sum(r["verdict"] for r in got) == 16


@pytest.mark.parametrize("cfg", [1024, 1536, 3072])
def test_tiny_every_tile_shape(hg, cfg):
    run_both(hg, configs.tiny(), "tiny lds_cap=%d" % cfg, lds_cap=cfg)


def test_families(hg):
    cases = [
        ("F1", F.single(F.f1_neighbour(4, 64, 32), 0, 1)),
        ("F1 big", F.single(F.f1_neighbour(300, 256, 32), 0, 1)),
        ("F1 self", F.single(F.f1_neighbour(40, 128, 32), 0, 0)),
        ("F2", F.single(F.f2_tree_reduction(64), 0, 1)),
        ("F2 1024", F.single(F.f2_tree_reduction(1024), 0, 1)),
        ("F2 barrier", F.single(F.f2_tree_reduction(256, barrier=True), 0, 1)),
        ("F3", F.single(F.f3_stride_mod(64, (16, 48, 64, 100)), 0, 0)),
        ("F3 shared", F.single(F.f3_stride_mod(1024, (16, 3), space=SHARED), 0, 0)),
        ("F4", F.single(F.f4_guard_halves(64), 0, 0)),
        ("F4+1", F.single(F.f4_guard_halves(64, extra=1), 0, 0)),
        ("F4 none", F.single(F.f4_guard_halves(1024, guarded=False), 0, 0)),
    ]
    for name, wl in cases:
        run_both(hg, wl, name)


def test_paper_examples(hg):
    cases = [
        ("K1 square", F.k1_copy_upp_low([[16, 16], [32, 32], [48, 48]]), (1, 1)),
        ("K1 32x1", F.k1_copy_upp_low([[32, 1]]), (1, 1)),
        ("K1 rw", F.k1_copy_upp_low([[32, 32], [32, 1]]), (1, 0)),
        ("K2", F.k2_reduce_final([[1], [2], [7]]), (0, 0)),
        ("K3", F.k3_tone_mapping([[16, 1, 2], [32, 2, 2], [16, 2, 2]]), (0, 0)),
        ("K4", F.k4_lud_internal([[64, 0], [64, 16], [64, -47]]), (0, 0)),
        ("K5", F.k5_shift([[512], [0], [3]]), (0, 0)),
    ]
    for name, m, (a, b) in cases:
        run_both(hg, F.single(m, a, b), name)


@pytest.mark.parametrize("seed", range(0, 60))
def test_random_models(hg, seed):
    run_both(hg, rand_workload(seed), "rand seed=%d" % seed)


def test_random_models_batched(hg):
    # many random models in one call: LDS items, HBM items and masks together
    models, pairs = [], []
    for seed in range(100, 140):
        wl = rand_workload(seed)
        base = len(models)
        models += wl.models
        pairs += [(m + base, a, b, k) for (m, a, b, k) in wl.pairs]
    run_both(hg, Workload(models, pairs), "rand batch")


def test_heavy_hitter_fallback(hg):
    """Every thread of a big grid writes one address: buckets overflow and
    the query goes through the HBM hash aggregation."""
    m = Model(0, [Array(GLOBAL, 32), Array(SHARED, 32)],
              [Access(0, WRITE, c(5)), Access(0, READ, c(5) + tid() % 2),
               Access(1, WRITE, tid() // 64), Access(0, WRITE, tid() // 4 + bid() * 2)],
              Launch((64, 1, 1), (256, 1, 1), 32), [[]])
    wl = Workload([m], [(0, 0, 0, 7), (0, 0, 1, 7), (0, 2, 2, 7), (0, 3, 3, 7),
                        (0, 3, 1, 7), (0, 0, 3, 5)])
    run_both(hg, wl, "heavy")


def test_skew_paths(hg):
    """Hot addresses at three scales: groups that fit after re-bucketing,
    groups that only fit once split by (address, block) with level 0
    counted per address, and (address, block) groups too big for any tile
    (HBM aggregation)."""
    m = Model(1, [Array(GLOBAL, 32), Array(SHARED, 32)],
              [Access(0, WRITE, tid() % 8, loops=[0]),                 # split
               Access(0, READ, tid() % 8 + loop(0) * 0, loops=[0]),
               Access(0, WRITE, tid() // 32 + bid() * 0, loops=[0]),    # split
               Access(0, WRITE, c(0) + loop(0) * 0, loops=[0]),          # fallback
               Access(0, WRITE, tid() + bid() * 64 + loop(0), loops=[0]),  # retry
               Access(1, WRITE, tid() % 2 + loop(0), loops=[0])],       # shared
              Launch((param(0), 1, 1), (256, 1, 1), 32), [[96], [40]],
              loops=[Loop(0, "lt", 12)])
    pairs = [(0, 0, 0, 7), (0, 0, 1, 7), (0, 2, 2, 7), (0, 3, 3, 7), (0, 3, 0, 7),
             (0, 4, 4, 7), (0, 4, 0, 7), (0, 5, 5, 7), (0, 0, 1, 1), (0, 2, 2, 6)]
    run_both(hg, Workload([m], pairs), "skew")
    import paper_2604_02106_amd as H
    st = H.default_context().stats()
    say("skew stats", {k: st[k] for k in ("retry_items", "split_items", "overflow_items",
                                          "fallback_records", "fallback_groups")})
    assert st["split_items"] > 0 and st["overflow_items"] > 0
    # every lane of a warp writes address 0 in access 3, so the lanes of one
    # warp share one fallback record there
    assert 0 < st["fallback_groups"] * 2 <= st["fallback_records"]
    assert st["presplit_items"] > 0  # tid % 8 over 96 blocks: routed at once


def test_overflow_then_split(hg):
    """Addresses that average far below a bucket of points but hold hot
    spots (every thread from 8 on shares one address per block, 4
    iterations): the item is partitioned first, overflows, and is split by
    (address, block); counts and witnesses equal the oracle's."""
    m = Model(0, [Array(GLOBAL, 32)],
              [Access(0, WRITE, emin(tid(), c(8)) + bid() * 16, loops=[0]),
               Access(0, READ, emin(tid(), c(8)) + bid() * 16 + loop(0) * 0, loops=[0])],
              Launch((64, 1, 1), (256, 1, 1), 32), [[]],
              loops=[Loop(0, "lt", 4)])
    wl = Workload([m], [(0, 0, 0, 7), (0, 0, 1, 7), (0, 1, 0, 6)])
    run_both(hg, wl, "overflow then split")
    st = hg.default_context().stats()
    say("overflow stats", {k: st[k] for k in ("presplit_items", "split_items",
                                               "retry_items", "overflow_items")})
    assert st["presplit_items"] == 0 and st["split_items"] > 0


def test_statuses(hg):
    ms = []

    def one(accs, launch=None, sets=([3],), loops=(), arrays=None):
        arrays = arrays or [Array(GLOBAL, 64), Array(SHARED, 32)]
        ms.append(Model(1, arrays, accs, launch or Launch((2, 1, 1), (8, 1, 1), 4),
                        [list(s) for s in sets], loops=loops))
        return len(ms) - 1

    pairs = []
    pairs.append((one([Access(0, WRITE, tid(), div(tid(), param(0) - 3))]), 0, 0, 7))
    pairs.append((one([Access(0, WRITE, div(c(1), tid() - 7), lt(tid(), 7))]), 0, 0, 7))
    pairs.append((one([Access(0, WRITE, c(I64MAX) + tid())]), 0, 0, 7))
    pairs.append((one([Access(0, WRITE, div(c(I64MAX) + param(0), param(0) - 3))],
                      sets=([1], [3])), 0, 0, 7))
    pairs.append((one([Access(1, WRITE, c(1 << 31) + tid())]), 0, 0, 7))
    pairs.append((one([Access(0, WRITE, tid())], launch=Launch((1, 1, 1), (2048, 1, 1))), 0, 0, 7))
    pairs.append((one([Access(0, WRITE, tid(), bint=c(-1))]), 0, 0, 7))
    pairs.append((one([Access(0, WRITE, tid()), Access(1, WRITE, tid())]), 0, 1, 7))
    pairs.append((one([Access(0, WRITE, loop(0), loops=[0])], loops=[Loop(0, "lt", 1 << 20)]), 0, 0, 7))
    pairs.append((one([Access(0, WRITE, c(0))], launch=Launch((param(0) - 3, 1, 1), (8, 1, 1))), 0, 0, 7))
    pairs.append((one([Access(0, READ, c(0)), Access(0, READ, c(0))]), 0, 1, 7))
    pairs.append((one([Access(0, ATOMIC, c(0), scope=SCOPE_BLOCK), Access(0, ATOMIC, c(0))]), 0, 1, 7))
    # a loop whose update overflows on one side only: the other side's
    # points are still scanned for a stronger error
    pairs.append((one([Access(0, WRITE, loop(0), loops=[0]),
                       Access(0, WRITE, tid(), bint=c(70000))],
                      loops=[Loop(1, "lt", I64MAX, "mul", 3)]), 0, 1, 7))
    run_both(hg, Workload(ms, pairs), "statuses")


def test_batched_config_subset(hg):
    """Batched uneven config at reduced grid scale, all pairs."""
    wl = configs.batched(seed=2002, n_models=48, scale=0.05, max_iters=16)
    got = run_both(hg, wl, "batched small")
    assert any(r["verdict"] for r in got) and not all(r["verdict"] for r in got)


def test_invariance_tile_shapes(hg):
    wl = configs.batched(seed=77, n_models=16, scale=0.1, max_iters=8)
    say("invariance")
    base = hg.check_pairs(wl)
    for cap in (1024, 3072):
        compare(hg.check_pairs(wl, lds_cap=cap), base, "lds_cap=%d" % cap)
    # a tiny device budget forces many HBM waves
    compare(hg.check_pairs(wl, max_device_bytes=1 << 22), base, "waves")


def test_graph_replay_matches_eager(hg):
    """The first phase is captured once and replayed: every replay, with
    eager work and synchronisations between replays, equals the eager run
    (log_level 2 runs the first phase eagerly) and the oracle."""
    ctx = hg.default_context()
    wl = configs.batched(seed=91, n_models=12, scale=0.05, max_iters=8)
    say("graph replay")
    want, _ = oracle.check_pairs(wl, "B", threads=8)
    eager = hg.Plan(ctx, wl, log_level=2)
    graph = hg.Plan(ctx, wl)
    base = eager.execute()
    compare(base, want, "eager")
    for rep in range(4):
        compare(graph.execute(), base, "replay %d" % rep)
        compare(eager.execute(), base, "eager %d" % rep)
        compare(hg.check_pairs(configs.tiny()), oracle.check_pairs(configs.tiny(), "B")[0],
                "tiny between replays")
    eager.close()
    graph.close()


def test_autotune_picks_a_shape_and_keeps_results(hg):
    ctx = hg.Context(0)
    wl = configs.batched(seed=92, n_models=8, scale=0.05, max_iters=8)
    say("autotune")
    cap, wave, ms = hg.rd_autotune(ctx, wl, reps=1)
    say("autotune picked", cap, wave, ms)
    assert cap in (1024, 1536, 3072) and wave in (768 << 20, 3072 << 20, 12288 << 20)
    assert ms > 0
    want, _ = oracle.check_pairs(wl, "B", threads=8)
    compare(hg.rd_check_pairs(ctx, wl), want, "after autotune")


@pytest.mark.parametrize("seed", range(0, 60, 6))
def test_random_models_interpreter_only(hg, seed, monkeypatch):
    """Term tables switched off (HGRD_INTERP): every point goes through the
    expression interpreter; results stay identical to the oracle."""
    monkeypatch.setenv("HGRD_INTERP", "1")
    run_both(hg, rand_workload(seed), "rand interp seed=%d" % seed)
    run_both(hg, configs.batched(seed=93, n_models=6, scale=0.05, max_iters=8),
             "batched interp")


def test_mixed_config_small(hg):
    """Mixed domain sizes (2^8..2^16 per query), 2-D/3-D launches, up to 64
    tuples, shared and global: every field equal to the oracle's."""
    wl = configs.mixed(seed=5005, n_queries=160, log2_max=16)
    got = run_both(hg, wl, "mixed small")
    assert any(r["verdict"] for r in got)


def test_pipelined_batches_match_one_plan(hg, monkeypatch):
    """rd_check_pairs with more pairs than one batch prepares batch k + 1 on
    a second context while batch k executes: every field equals the
    oracle's and the one-plan results at several batch sizes, and the
    stats are the sums over the batches."""
    wl = configs.mixed(seed=97, n_queries=240, log2_max=17)
    want, _ = oracle.check_pairs(wl, "B", threads=8)
    monkeypatch.setenv("HGRD_BATCH_PAIRS", "0")
    say("one plan", len(wl.pairs))
    compare(hg.check_pairs(wl), want, "one plan")
    one = hg.default_context().stats()
    for b in ("37", "100", "239"):
        monkeypatch.setenv("HGRD_BATCH_PAIRS", b)
        say("batches of", b)
        compare(hg.check_pairs(wl), want, "batches of " + b)
        st = hg.default_context().stats()
        for k in ("evals", "small_items", "hbm_items", "units_apart", "block_symmetric"):
            assert st[k] == one[k], (b, k, st[k], one[k])
        assert st["total_ms"] > 0


def test_prefilter_is_exact(hg):
    """The interval pre-filter decides (pair, tuple) units whose address
    ranges cannot meet; every field stays equal to the oracle's."""
    for name, wl in (("batched pre", configs.batched(seed=94, n_models=16, scale=0.05,
                                                      max_iters=8)),
                     ("mixed pre", configs.mixed(seed=95, n_queries=96, log2_max=15)),
                     ("rand pre", rand_workload(7))):
        run_both(hg, wl, name, prefilter=1)
    st = hg.default_context().stats()
    say("prefiltered", st["prefiltered"])


def test_unit_filter_is_exact(hg, monkeypatch):
    """The unit filter of rd_execute (two accesses proven never to share an
    address are neither partitioned nor joined) decides the mixed
    workload's near-miss and interleaved pairs; every field equals the
    oracle's with it and without it (HGRD_NO_UNIT_FILTER)."""
    wl = configs.mixed(seed=96, n_queries=160, log2_max=19)
    want, _ = oracle.check_pairs(wl, "B", threads=8)
    say("unit filter on", len(wl.pairs))
    compare(hg.check_pairs(wl), want, "unit filter on")
    st = hg.default_context().stats()
    say("units apart", st["units_apart"], "hbm items", st["hbm_items"])
    assert st["units_apart"] > 0
    monkeypatch.setenv("HGRD_NO_UNIT_FILTER", "1")
    say("unit filter off")
    compare(hg.check_pairs(wl), want, "unit filter off")
    assert hg.default_context().stats()["units_apart"] == 0


def test_block_symmetry_is_exact(hg, monkeypatch):
    """Shared-array units whose address and guard do not depend on the
    block are joined on block 0 and counted once per block; a unit whose
    address does depend on the block is joined block by block.  Every
    field equals the oracle's, with and without the shortcut."""
    t = tid()
    m = Model(2, [Array(SHARED, 32)],
              [Access(0, WRITE, t // 32 + loop(0) * 8, lt(t, param(0)), [0]),
               Access(0, READ, t % param(1) + loop(0), None, [0]),
               Access(0, WRITE, t * 2 + loop(0), None, [0]),
               Access(0, WRITE, t % 4 + bid() % 2, None, [0])],
              Launch((37, 3, 1), (64, 2, 1), 32), [[100, 24], [128, 7]],
              loops=[Loop(0, "lt", 3)])
    wl = Workload([m], [(0, 0, 1, 7), (0, 0, 0, 7), (0, 1, 2, 7), (0, 2, 2, 7),
                        (0, 3, 3, 7), (0, 3, 1, 7)])
    want, _ = oracle.check_pairs(wl, "B", threads=8)
    say("symmetry on")
    compare(hg.check_pairs(wl), want, "symmetry on")
    st = hg.default_context().stats()
    say("block symmetric units", st["block_symmetric"])
    assert st["block_symmetric"] >= 2 * 2  # at least the self pairs 0 and 3 of both tuples
    assert sum(r["verdict"] for r in want) >= 3
    monkeypatch.setenv("HGRD_NO_SYMMETRY", "1")
    say("symmetry off")
    compare(hg.check_pairs(wl), want, "symmetry off")
    assert hg.default_context().stats()["block_symmetric"] == 0


def test_global_block_symmetry_is_exact(hg, monkeypatch):
    """Global-array units whose address and guard do not depend on the
    block are joined on block 0: its address groups stand for G identical
    groups (inter-block pairs G^2 S_0 - G S_1, the other classes G times
    block 0's).  Covers an access whose points are alone in block 0 (every
    point still races with its copies in the other blocks), masks without
    the inter-block class, a one-block tuple, and a unit with a block term.
    Every field equals the oracle's, with and without the shortcut."""
    t = tid()
    m = Model(2, [Array(GLOBAL, 32)],
              [Access(0, WRITE, t // 32 + loop(0) * 8, lt(t, param(0)), [0]),
               Access(0, READ, t % param(1) + loop(0), None, [0]),
               Access(0, WRITE, t * 2 + loop(0) * 1000, None, [0]),
               Access(0, WRITE, t % 4 + bid() % 2, None, [0])],
              Launch((param(1), 1, 1), (64, 2, 1), 32), [[100, 24], [128, 7], [50, 1]],
              loops=[Loop(0, "lt", 3)])
    wl = Workload([m], [(0, 0, 1, 7), (0, 0, 0, 7), (0, 1, 2, 7), (0, 2, 2, 7),
                        (0, 3, 3, 7), (0, 3, 1, 7), (0, 0, 1, 6), (0, 2, 2, 1),
                        (0, 1, 2, 4)])
    want, _ = oracle.check_pairs(wl, "B", threads=8)
    say("global symmetry on")
    compare(hg.check_pairs(wl), want, "global symmetry on")
    st = hg.default_context().stats()
    say("block symmetric units", st["block_symmetric"])
    assert st["block_symmetric"] >= 6
    assert want[3]["by_class"][0] > 0  # lone points in block 0 race with their copies
    monkeypatch.setenv("HGRD_NO_SYMMETRY", "1")
    say("global symmetry off")
    compare(hg.check_pairs(wl), want, "global symmetry off")
    assert hg.default_context().stats()["block_symmetric"] == 0


def test_global_block_symmetry_large_blocks(hg, monkeypatch):
    """The same symmetry for blocks larger than one LDS tile: block 0's
    points alone are partitioned through HBM and joined with the scaled
    address level; a block-0 address held by more points than a bucket
    overflows to the fallback, which scales the same way."""
    t = tid(0) + tid(1) * 256
    m = Model(1, [Array(GLOBAL, 32)],
              [Access(0, WRITE, t + loop(0) * 16, None, [0]),
               Access(0, READ, t // 4 + loop(0), lt(t, param(0)), [0]),
               Access(0, WRITE, c(5) + loop(0) * 0, None, [0]),
               Access(0, WRITE, t * 16 + loop(0), None, [0])],
              Launch((3, 1, 1), (256, 4, 1), 32), [[700], [1024]],
              loops=[Loop(0, "lt", 16)])
    wl = Workload([m], [(0, 0, 0, 7), (0, 0, 1, 7), (0, 2, 2, 7), (0, 2, 0, 7),
                        (0, 3, 3, 7), (0, 3, 0, 5), (0, 0, 1, 6)])
    want, _ = oracle.check_pairs(wl, "B", threads=8)
    say("global symmetry, large blocks")
    compare(hg.check_pairs(wl), want, "global symmetry large")
    st = hg.default_context().stats()
    say("symmetric", st["block_symmetric"], "overflow", st["overflow_items"],
        "hbm", st["hbm_items"])
    assert st["block_symmetric"] >= 10 and st["overflow_items"] > 0
    assert sum(r["verdict"] for r in want) >= 4
    monkeypatch.setenv("HGRD_NO_SYMMETRY", "1")
    say("global symmetry, large blocks, off")
    compare(hg.check_pairs(wl), want, "global symmetry large off")


def test_bucket_filter_drops_own_thread_buckets(hg, monkeypatch):
    """Accesses that meet only in their own thread (one injective map,
    written as two different expressions so that the unit filter does not
    decide the unit first) hold equal addresses in every bucket, yet no
    conflict: the bucket filter compares threads and passes no bucket to
    the join.  A map that sends two threads to one address keeps its
    buckets.  (The dense-item bypass, which would skip the filter for these
    four-points-per-address items, is off here; the results are the same
    either way.)"""
    monkeypatch.setenv("HGRD_DENSE", "0")
    g = tid() + bid() * 256
    m = Model(0, [Array(GLOBAL, 32), Array(GLOBAL, 64)],
              [Access(0, WRITE, g, loops=[0]), Access(0, READ, (g + c(1)) - c(1), loops=[0]),
               Access(1, WRITE, c(1 << 40) + g * 4 + loop(0), loops=[0]),
               Access(1, READ, c(1 << 40) + (g * 4 + loop(0)), loops=[0]),
               Access(0, WRITE, g // 2, loops=[0]), Access(0, READ, g // 2, loops=[0])],
              Launch((256, 1, 1), (256, 1, 1), 32), [[]], loops=[Loop(0, "lt", 4)])
    own = Workload([m], [(0, 0, 1, 7), (0, 2, 3, 7)])
    got = run_both(hg, own, "own thread")
    assert not any(r["verdict"] for r in got)
    st = hg.default_context().stats()
    say("own thread stats", {k: st[k] for k in ("hbm_items", "join_tab_bytes",
                                                "filter_tab_bytes")})
    assert st["hbm_items"] > 0 and st["filter_tab_bytes"] > 0 and st["join_tab_bytes"] == 0
    two = Workload([m], [(0, 4, 5, 7)])
    got = run_both(hg, two, "two threads")
    assert got[0]["verdict"] == 1
    assert hg.default_context().stats()["join_tab_bytes"] > 0


def test_batched_full_size_sampled(hg):
    """The headline workload at full size (256 models x 16 pairs, seed 2002)
    in the configuration bench.py times; a seeded random sample of pairs
    whose domains the oracle enumerates in seconds (40 of at most 2^22
    evaluations, 8 of 2^22..2^25, which take the HBM path) is compared with
    the oracle field by field, and every status is OK."""
    import numpy as np
    wl = configs.batched(seed=2002)
    say("batched full", len(wl.pairs))
    got = hg.check_pairs(wl)
    assert all(r["status"] == 0 for r in got)
    rng = np.random.Generator(np.random.PCG64(11))
    order = [int(k) for k in rng.permutation(len(wl.pairs))]
    small = [k for k in order if got[k]["evals"] <= (1 << 22)][:40]
    large = [k for k in order if (1 << 22) < got[k]["evals"] <= (1 << 25)][:8]
    assert len(small) == 40 and len(large) == 8
    idx = small + large
    want, _ = oracle.check_pairs(wl.subset(idx), "B", threads=8)
    compare([got[k] for k in idx], want, "batched full sample")
    assert any(got[k]["verdict"] for k in idx)
