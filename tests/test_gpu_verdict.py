"""VERDICT mode with LEX and learned (MLP) tile orders, the network's GPU
forward/backward against the float64 reference, tile labels against a brute
force, training, and the gain of the learned order over LEX.

VERDICT-mode bar: verdicts and statuses equal the oracle's; every racy
witness is a conflicting pair by the oracle's predicate; counts are lower
bounds; pairs not stopped by the tile search are identical to EXACT.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import mlp as ref
from workloads import Workload, GLOBAL, SHARED, ATOMIC
from workloads import configs, families as F
from workloads.random_models import rand_workload
from tests import npeval

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


def _mask(m, a, b, k):
    x, y = m.accesses[a], m.accesses[b]
    mask = k & 7
    if x.kind == "read" and y.kind == "read":
        return 0
    if x.kind == ATOMIC and y.kind == ATOMIC:
        if x.scope == "device" and y.scope == "device":
            return 0
        mask &= 1
    if m.arrays[x.array].space == SHARED:
        mask &= ~1
    return mask


def check_verdict(hg, wl, got, tiles, name):
    want, _ = oracle.check_pairs(wl, "B", threads=8)
    for k, (g, w, t) in enumerate(zip(got, want, tiles)):
        assert g["status"] == w["status"], (name, k, g, w)
        assert g["verdict"] == w["verdict"], (name, k, g, w)
        if not (g["flags"] & 2):
            assert t == 0
            assert g == w, (name, k, g, w)
            continue
        assert t >= 1 and w["verdict"] == 1
        assert 1 <= g["count"] <= w["count"]
        for c in range(3):
            assert g["by_class"][c] <= w["by_class"][c]
        # the witness is a conflicting pair by the oracle's predicate
        mi, a, b, kk = wl.pairs[k]
        m = wl.models[mi]
        s, b1, t1, i1, b2, t2, i2 = g["witness"]
        pi, pj = npeval.points(m, a, s), npeval.points(m, b, s)

        def pick(P, bl, tl, il):
            sel = (P[1] == bl) & (P[2] == tl) & (P[3] == il)
            assert sel.sum() == 1
            return [int(P[n][sel][0]) for n in (0, 1, 2, 4, 5)]
        p, q = pick(pi, b1, t1, i1), pick(pj, b2, t2, i2)
        cls = oracle.conflict_class(p, q, m.launch.warp, _mask(m, a, b, kk))
        assert cls and cls == g["witness_class"], (name, k, g)
        assert g["w_addr"] == p[0]
    return want


@pytest.mark.parametrize("order", [0, 1])
def test_verdict_mode_tiny_and_random(hg, order):
    ctx = hg.default_context()
    w = None
    if order == 1:
        from paper_2604_02106_amd import tile_mlp
        w = tile_mlp.init_weights(3)
    for name, wl in [("tiny", configs.tiny()),
                     ("rand", rand_workload(77)), ("rand2", rand_workload(78)),
                     ("sparse", configs.sparse(seed=11, n_queries=64, G=16, B=32,
                                               queries_per_model=16))]:
        say(name, "order", order)
        plan = hg.Plan(ctx, wl, mode=hg.MODE_VERDICT, order=order, mlp=w,
                       tile_budget=64)
        got = plan.execute()
        check_verdict(hg, wl, got, plan.tiles(), name)
        # replay gives the same results
        assert plan.execute() == got


def test_mlp_forward_and_gradient_match_float64(hg):
    ctx = hg.default_context()
    rng = np.random.Generator(np.random.PCG64(5))
    X = rng.normal(size=(300, 32)).astype(np.float32)
    Y = (rng.random(300) < 0.4).astype(np.float32)
    p = ref.init(9)
    w = ref.flatten(p).astype(np.float32)
    p32 = ref.unflatten(w.astype(np.float64))
    z_gpu = hg.rd_mlp_forward(ctx, w, X)
    z_ref, _ = ref.forward(p32, X.astype(np.float64))
    assert np.allclose(z_gpu, z_ref, rtol=1e-4, atol=1e-5)
    g_gpu, loss_gpu = hg.rd_mlp_grad(ctx, w, X, Y)
    g_ref = ref.flatten(ref.grad(p32, X.astype(np.float64), Y.astype(np.float64)))
    scale = np.abs(g_ref).max()
    assert abs(loss_gpu - ref.loss(p32, X, Y)) < 1e-4 * max(1.0, abs(loss_gpu))
    assert np.allclose(g_gpu, g_ref, rtol=1e-4, atol=1e-5 * scale)


def test_adam_steps_match_closed_form(hg):
    """Two full-batch steps of rd_mlp_train (Adam, beta1 0.9, beta2 0.999,
    eps 1e-8, bias-corrected) against the same two steps in float64 with
    the reference network's gradients."""
    ctx = hg.default_context()
    rng = np.random.Generator(np.random.PCG64(6))
    X = rng.normal(size=(256, 32)).astype(np.float32)
    Y = (rng.random(256) < 0.4).astype(np.float32)
    w0 = ref.flatten(ref.init(11)).astype(np.float32)
    lr = 1e-3
    w_gpu, _ = hg.rd_mlp_train(ctx, w0, X, Y, epochs=2, batch=256, lr=lr, seed=3)
    b1, b2, eps = 0.9, 0.999, 1e-8
    w = w0.astype(np.float64)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    for t in (1, 2):
        g = ref.flatten(ref.grad(ref.unflatten(w), X.astype(np.float64), Y.astype(np.float64)))
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        w = w - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    moved = np.abs(w - w0) > 0.5 * lr
    assert moved.mean() > 0.5  # most weights take about lr per step
    assert np.allclose(w_gpu, w, rtol=0, atol=2e-2 * lr)


def test_tile_labels_match_brute_force(hg):
    ctx = hg.default_context()
    wl = configs.sparse(seed=12, n_queries=8, G=8, B=16, queries_per_model=8)
    X, Y, ids = hg.rd_tile_data(ctx, wl)
    assert X.shape == (8 * 64, 32) and set(np.unique(Y)) <= {0.0, 1.0}
    for row in range(len(Y)):
        k, s, b1, b2 = [int(v) for v in ids[row]]
        mi, a, b, _ = wl.pairs[k]
        m = wl.models[mi]
        pi, pj = npeval.points(m, a, s), npeval.points(m, b, s)
        ai = pi[0][pi[1] == b1]
        aj = pj[0][pj[1] == b2]
        ti = pi[2][pi[1] == b1]
        tj = pj[2][pj[1] == b2]
        hit = False
        for x, tx in zip(ai, ti):
            same = (aj == x) & ~((b1 == b2) & (tj == tx))
            if same.any():
                hit = True
                break
        assert bool(Y[row]) == hit, (row, k, b1, b2)


def test_training_lowers_loss_and_mlp_order_gains(hg):
    """Train on tile labels of training workloads (seed 4005), then on
    held-out queries whose tiles all overlap but one conflicts (seed 4004)
    compare the tiles examined before the first witness: the trained
    network against plain index order (LEX), index order after the tiles
    proven disjoint (interval order), and the same network untrained."""
    ctx = hg.default_context()
    from paper_2604_02106_amd import tile_mlp
    say("train")
    w, losses, info = tile_mlp.train(ctx, epochs=12, seed=1)
    assert losses[-1] < 0.5 * losses[0], losses
    G = 64
    wl = configs.sparse_overlap(seed=4004, n_queries=256, G=G, B=64, queries_per_model=32)
    arms = {"lex": (hg.ORDER_LEX, None), "interval": (hg.ORDER_INTERVAL, None),
            "trained": (hg.ORDER_MLP, w)}
    # the same network untrained: 8 random initialisations (one of them may
    # happen to rank the lone off-diagonal overlapping tile first)
    for s in range(8):
        arms["untrained %d" % s] = (hg.ORDER_MLP, tile_mlp.init_weights(100 + s))
    want, _ = oracle.check_pairs(wl, "B", threads=8)
    racy = [k for k, r in enumerate(want) if r["verdict"]]
    assert len(racy) > 50
    med = {}
    for name, (order, wt) in arms.items():
        say("gain arm", name)
        plan = hg.Plan(ctx, wl, mode=hg.MODE_VERDICT, order=order, mlp=wt,
                       tile_budget=G * G)
        got = plan.execute()
        tiles = plan.tiles()
        assert [g["verdict"] for g in got] == [r["verdict"] for r in want], name
        t = np.array([tiles[k] or G * G + 1 for k in racy])
        med[name] = float(np.median(t))
    untrained = float(np.mean([med["untrained %d" % s] for s in range(8)]))
    say("median tiles to the witness", med, "untrained mean", untrained)
    assert med["trained"] <= 4
    assert med["interval"] > 8 and med["lex"] > 100
    assert untrained >= 4 * max(1.0, med["trained"])
