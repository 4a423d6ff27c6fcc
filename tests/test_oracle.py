"""Pins of the CPU oracle to facts that do not come from the oracle itself.

* closed forms F1-F4, derived by hand (docstrings below);
* the verdicts the paper states for its worked examples (tests/golden);
* planted labels of the tiny config, which hold by construction;
* C integer semantics on specific values (C99 6.5.5, 6.5.7);
* the equi-join identity computed with numpy.unique;
* Oracle-A (the definition) against Oracle-B (sort + prefix groups);
* invariants: swapping the pair, additivity over tuples and masks,
  translation of addresses, shared vs global with intra-block classes.
"""
import json
import os

import numpy as np
import pytest

import oracle
from workloads import (E, c, param, tid, bid, bdim, loop, div, mod, shl, shr,
                       neg, lt, Model, Workload, Access, Array, Launch, Loop,
                       GLOBAL, SHARED, READ, WRITE, ATOMIC, SCOPE_BLOCK,
                       SCOPE_DEVICE, INTER, INTRA_BLOCK, INTRA_WARP)
from workloads import families as F, configs
from workloads.random_models import rand_workload
from tests import npeval

HERE = os.path.dirname(os.path.abspath(__file__))


def run(wl, method="B"):
    return oracle.check_pairs(wl, method, threads=4)[0]


def both(wl):
    ra, rb = run(wl, "A"), run(wl, "B")
    assert ra == rb
    return ra


# ---------------------------------------------------------------------------
# closed forms

@pytest.mark.parametrize("G,B,w", [(4, 64, 32), (3, 32, 8), (1, 16, 4), (5, 8, 2)])
def test_f1_neighbour(G, B, w):
    """W A[g] vs W A[g+1]: thread g conflicts with thread g-1 only.
    count = GB - 1; inter = G - 1 (first thread of each block but the first);
    same-warp pairs: t % w != 0, t >= 1 -> B - B/w per block;
    other intra-block: t % w == 0, t >= 1 -> B/w - 1 per block.
    Witness: p = (b0, t1), q = (b0, t0), address 1, intra-warp (w >= 2)."""
    r = both(F.single(F.f1_neighbour(G, B, w), 0, 1))[0]
    assert r["status"] == 0 and r["verdict"] == 1
    assert r["count"] == G * B - 1
    assert r["by_class"] == [G - 1, G * (B // w - 1), G * (B - B // w)]
    assert r["witness"] == (0, 0, 1, 0, 0, 0, 0)
    assert r["w_addr"] == 1 and r["witness_class"] == INTRA_WARP
    # the self-pair A[g] vs A[g] is injective: race-free
    r = both(F.single(F.f1_neighbour(G, B, w), 0, 0))[0]
    assert r["verdict"] == 0 and r["count"] == 0
    assert r["witness"] == (-1,) * 7


@pytest.mark.parametrize("B", [8, 16, 64, 128])
def test_f2_tree_reduction(B):
    """Without a barrier, W sd[t] at iteration k meets R sd[t'+s_k'] at
    iteration k' iff k < k' (then t = t' + s_k' < 2 s_k' <= s_k): count =
    sum_k k * s_k with s_k = B >> (k+1) (57 for B = 64).  Smallest p with a
    partner: t = 1 (t = t'+s needs s = 1, i.e. the last iteration, t' = 0)
    at iteration 0.  With a barrier per iteration (bint = k) nothing races."""
    L = B.bit_length() - 1
    expect = sum(k * (B >> (k + 1)) for k in range(L))
    r = both(F.single(F.f2_tree_reduction(B), 0, 1))[0]
    assert r["count"] == expect
    if B == 64:
        assert expect == 57
    assert r["witness"] == (0, 0, 1, 0, 0, 0, L - 1)
    assert r["w_addr"] == 1
    rb = both(F.single(F.f2_tree_reduction(B, barrier=True), 0, 1))[0]
    assert rb["verdict"] == 0
    for pair in [(0, 0), (0, 2), (2, 0)]:
        for bar in (False, True):
            r0 = both(F.single(F.f2_tree_reduction(B, barrier=bar), *pair))[0]
            assert r0["count"] == 0, pair


def _f3_count(B, W):
    n = [len(range(r, B, W)) for r in range(min(W, B))]
    return sum(x * (x - 1) for x in n)


@pytest.mark.parametrize("B,Ws", [(64, (16,)), (64, (48,)), (64, (64,)),
                                  (64, (16, 48, 100)), (32, (3, 5))])
def test_f3_stride_mod(B, Ws):
    """Self-pair A[tid % W]: count = sum_r n_r (n_r - 1), n_r = #{t < B: t = r
    mod W}; 192 for (64, 16), 32 for (64, 48), 0 for W >= B; additive over
    tuples.  Witness (t0 ; tW) in the first tuple with W < B."""
    r = both(F.single(F.f3_stride_mod(B, Ws), 0, 0))[0]
    assert r["count"] == sum(_f3_count(B, W) for W in Ws)
    if (B, Ws) == (64, (16,)):
        assert r["count"] == 192
    if (B, Ws) == (64, (48,)):
        assert r["count"] == 32
    first = next((s for s, W in enumerate(Ws) if W < B), None)
    if first is None:
        assert r["verdict"] == 0
    else:
        assert r["witness"] == (first, 0, 0, 0, 0, Ws[first], 0)
        assert r["witness_class"] == (INTRA_WARP if Ws[first] < 32 else INTRA_BLOCK)


def test_f4_guard_halves():
    """Self-pair A[tid % H], H = B/2: guard tid < H is injective -> 0; guard
    tid < H + 1 adds thread H, which meets thread 0 -> 2 ordered pairs,
    witness (t0 ; tH); no guard -> every t < H meets t + H -> B pairs."""
    B = 64
    assert both(F.single(F.f4_guard_halves(B), 0, 0))[0]["count"] == 0
    r = both(F.single(F.f4_guard_halves(B, extra=1), 0, 0))[0]
    assert r["count"] == 2 and r["witness"] == (0, 0, 0, 0, 0, B // 2, 0)
    assert both(F.single(F.f4_guard_halves(B, guarded=False), 0, 0))[0]["count"] == B


# ---------------------------------------------------------------------------
# the paper's worked examples

def _paper_cases():
    with open(os.path.join(HERE, "golden", "paper_examples.json")) as f:
        return json.load(f)["cases"]


_MODELS = {"k1": F.k1_copy_upp_low, "k2": F.k2_reduce_final, "k3": F.k3_tone_mapping,
           "k4": F.k4_lud_internal, "k5": F.k5_shift}


@pytest.mark.parametrize("case", _paper_cases(), ids=lambda c: c["id"])
def test_paper_examples(case):
    m = _MODELS[case["model"]](case["sets"])
    r = both(F.single(m, *case["pair"]))[0]
    ex = case["expect"]
    assert r["status"] == 0
    assert r["verdict"] == ex["verdict"], case["cite"]
    if "classes" in ex:
        assert r["classes"] == ex["classes"]
    if "classes_include" in ex:
        assert r["classes"] & ex["classes_include"]


def test_k5_small_pitch_reading():
    """rowSize in {1, 2, 3} is positive but rowSize/4 = 0, so exact semantics
    still race (the reading taken for Figure 5)."""
    for rs in (1, 2, 3):
        assert both(F.single(F.k5_shift([[rs]]), 0, 0))[0]["verdict"] == 1


# ---------------------------------------------------------------------------
# planted labels

def test_tiny_planted_labels():
    wl = configs.tiny()
    assert len(wl.pairs) == 64
    r = both(wl)
    assert [bool(x["verdict"]) for x in r] == wl.meta["planted_racy"]
    assert sum(x["verdict"] for x in r) == 16
    assert all(x["status"] == 0 for x in r)
    assert sum(x["evals"] for x in r) == 64 * 2 * 4 * 64 * 8


# ---------------------------------------------------------------------------
# C integer semantics (C99 6.5.5 and 6.5.7)

I64MIN, I64MAX = -(1 << 63), (1 << 63) - 1


@pytest.mark.parametrize("expr,value,err", [
    (div(c(-7), c(2)), -3, 0), (mod(c(-7), c(2)), -1, 0),
    (div(c(7), c(-2)), -3, 0), (mod(c(7), c(-2)), 1, 0),
    (mod(c(-8), c(4)), 0, 0), (div(c(5), c(0)), 0, 1), (mod(c(5), c(0)), 0, 1),
    (div(c(I64MIN), c(-1)), 0, 2), (mod(c(I64MIN), c(-1)), 0, 2),
    (shr(c(-7), c(1)), -4, 0), (shr(c(-1), c(63)), -1, 0), (shr(c(7), c(1)), 3, 0),
    (shl(c(3), c(4)), 48, 0), (shl(c(-1), c(63)), I64MIN, 0), (shl(c(1), c(63)), 0, 2),
    (shl(c(1), c(64)), 0, 2), (shl(c(1), c(-1)), 0, 2), (shr(c(1), c(64)), 0, 2),
    (c(I64MAX) + 1, 0, 2), (c(I64MIN) - 1, 0, 2), (c(1 << 62) * 2, 0, 2),
    (neg(c(I64MIN)), 0, 2), (neg(c(5)), -5, 0),
    (lt(c(-1), c(0)), 1, 0),
    # errors continue with 0: (5/0) + (MAX + 1) has both bits
    (div(c(5), c(0)) + (c(I64MAX) + 1), 0, 3),
    (param(0) * param(1), 12, 0),
])
def test_integer_semantics(expr, value, err):
    v, e = oracle.eval_uniform(expr, [3, 4])
    assert (v, e) == (value, err)


# ---------------------------------------------------------------------------
# Oracle-A == Oracle-B on random tiny models

@pytest.mark.parametrize("seed", range(40))
def test_methods_agree_random(seed):
    wl = rand_workload(seed)
    ra, rb = run(wl, "A"), run(wl, "B")
    assert ra == rb


# ---------------------------------------------------------------------------
# equi-join identity via numpy.unique

def _join(keys_i, keys_j):
    """sum over keys of n_i(key) * n_j(key), with numpy.unique counting."""
    if len(keys_i) == 0 or len(keys_j) == 0:
        return 0
    ui, ci = np.unique(keys_i, axis=0, return_counts=True)
    uj, cj = np.unique(keys_j, axis=0, return_counts=True)
    di = {tuple(k): n for k, n in zip(ui.tolist(), ci.tolist())}
    return sum(n * di.get(tuple(k), 0) for k, n in zip(uj.tolist(), cj.tolist()))


@pytest.mark.parametrize("seed", range(12))
def test_equi_join_identity(seed):
    """All-class mask, constant intervals: count = J(addr) - J(addr, b, t)."""
    wl = rand_workload(1000 + seed)
    for (mi, a, b, _), r in zip(wl.pairs, run(Workload(wl.models, [
            (p[0], p[1], p[2], 7) for p in wl.pairs]))):
        m = wl.models[mi]
        acc_a, acc_b = m.accesses[a], m.accesses[b]
        if acc_a.bint or acc_a.wint or acc_b.bint or acc_b.wint:
            continue
        if m.arrays[acc_a.array].space != GLOBAL:
            continue
        kinds = {acc_a.kind, acc_b.kind}
        if kinds == {READ} or kinds == {ATOMIC}:
            continue
        total = 0
        for s in range(len(m.param_sets)):
            pi, pj = npeval.points(m, a, s), npeval.points(m, b, s)
            if pi is None:
                continue
            ki = np.stack([pi[0]], 1)
            kj = np.stack([pj[0]], 1)
            ki3 = np.stack([pi[0], pi[1], pi[2]], 1)
            kj3 = np.stack([pj[0], pj[1], pj[2]], 1)
            total += _join(ki, kj) - _join(ki3, kj3)
        assert r["count"] == total


# ---------------------------------------------------------------------------
# invariants

@pytest.mark.parametrize("seed", range(10))
def test_invariants(seed):
    wl = rand_workload(2000 + seed)
    base = run(wl)
    # count = sum of classes; verdict iff count > 0
    for r in base:
        assert r["count"] == sum(r["by_class"])
        assert r["verdict"] == (r["count"] > 0)
        assert (r["witness"][0] >= 0) == bool(r["verdict"])
    # swapping the pair keeps counts per class
    sw = run(Workload(wl.models, [(m, b, a, k) for (m, a, b, k) in wl.pairs]))
    for r, q in zip(base, sw):
        assert (r["count"], r["by_class"], r["status"]) == (q["count"], q["by_class"], q["status"])
    # single-class masks add up
    per = [run(Workload(wl.models, [(m, a, b, k & cl) for (m, a, b, k) in wl.pairs]))
           for cl in (1, 2, 4)]
    for i, r in enumerate(base):
        if r["flags"] & 1:
            continue
        assert r["count"] == sum(p[i]["count"] for p in per)


@pytest.mark.parametrize("seed", range(6))
def test_tuples_add_up(seed):
    wl = rand_workload(3000 + seed)
    base = run(wl)
    for idx, ((mi, a, b, k), r) in enumerate(zip(wl.pairs, base)):
        m = wl.models[mi]
        tot = 0
        for s in m.param_sets:
            ms = Model(m.n_params, m.arrays, m.accesses, m.launch, [s], m.loops)
            tot += run(Workload([ms], [(0, a, b, k)]))[0]["count"]
        assert r["count"] == tot


def test_translation_and_witness_predicate():
    """Adding a constant to both addresses changes only w_addr; every witness
    satisfies the conflict predicate."""
    for seed in range(8):
        wl = rand_workload(4000 + seed)
        base = run(wl)
        for (mi, a, b, k), r in zip(wl.pairs, base):
            if not r["verdict"]:
                continue
            m = wl.models[mi]
            sh = [Access(x.array, x.kind, x.addr + 1000, x.guard, x.loops, x.bint,
                         x.wint, x.scope) for x in m.accesses]
            ms = Model(m.n_params, m.arrays, sh, m.launch, m.param_sets, m.loops)
            q = run(Workload([ms], [(0, a, b, k)]))[0]
            assert q["count"] == r["count"] and q["witness"] == r["witness"]
            assert q["w_addr"] == r["w_addr"] + 1000
            s, b1, t1, i1, b2, t2, i2 = r["witness"]
            pi, pj = npeval.points(m, a, s), npeval.points(m, b, s)

            def pick(P, bl, tl, il):
                sel = (P[1] == bl) & (P[2] == tl) & (P[3] == il)
                assert sel.sum() == 1
                return [int(P[n][sel][0]) for n in (0, 1, 2, 4, 5)]
            p = pick(pi, b1, t1, i1)
            qq = pick(pj, b2, t2, i2)
            mask = k
            acc = m.accesses[a]
            if m.arrays[acc.array].space == SHARED:
                mask &= ~INTER
            if acc.kind == ATOMIC and m.accesses[b].kind == ATOMIC:
                mask &= INTER
            assert oracle.conflict_class(p, qq, m.launch.warp, mask) == r["witness_class"]


def test_shared_equals_global_intra():
    for seed in range(6):
        wl = rand_workload(5000 + seed)
        sh, gl = [], []
        for m in wl.models:
            sh.append(Model(m.n_params, [Array(SHARED, 64)] * 2,
                            [Access(0, x.kind, x.addr, x.guard, x.loops, x.bint, x.wint, x.scope)
                             for x in m.accesses], m.launch, m.param_sets, m.loops))
            gl.append(Model(m.n_params, [Array(GLOBAL, 64)] * 2,
                            [Access(0, x.kind, x.addr, x.guard, x.loops, x.bint, x.wint, x.scope)
                             for x in m.accesses], m.launch, m.param_sets, m.loops))
        rs = run(Workload(sh, [(mi, a, b, 7) for (mi, a, b, _) in wl.pairs]))
        rg = run(Workload(gl, [(mi, a, b, 6) for (mi, a, b, _) in wl.pairs]))
        for x, y in zip(rs, rg):
            assert (x["count"], x["by_class"], x["witness"]) == (y["count"], y["by_class"], y["witness"])


# ---------------------------------------------------------------------------
# masks and statuses

def _one(acc_list, pair, launch=None, sets=([3],), loops=(), arrays=None, mask=7):
    arrays = arrays or [Array(GLOBAL, 64), Array(SHARED, 32)]
    m = Model(1, arrays, acc_list, launch or Launch((2, 1, 1), (8, 1, 1), 4),
              [list(s) for s in sets], loops=loops)
    return run(Workload([m], [(0, pair[0], pair[1], mask)]))[0]


def test_trivial_masks():
    """Section 6.1 / appendix A.2: read/read and device-scoped atomic pairs
    are trivially race-free; atomics with a block-scoped side only race
    across blocks."""
    r = _one([Access(0, READ, c(0)), Access(0, READ, c(0))], (0, 1))
    assert r["flags"] & 1 and r["verdict"] == 0
    r = _one([Access(0, ATOMIC, c(0)), Access(0, ATOMIC, c(0))], (0, 1))
    assert r["flags"] & 1
    r = _one([Access(0, ATOMIC, c(0), scope=SCOPE_BLOCK), Access(0, ATOMIC, c(0))], (0, 1))
    assert r["flags"] == 0 and r["classes"] == INTER
    assert r["count"] == 2 * 8 * 8          # ordered pairs across the two blocks
    r = _one([Access(0, READ, c(0)), Access(0, ATOMIC, c(0))], (0, 1))
    assert r["classes"] == 7                 # read vs atomic is checked
    r = _one([Access(1, WRITE, c(0)), Access(1, WRITE, c(0))], (0, 1))
    assert r["by_class"][0] == 0 and r["count"] == 2 * 8 * 7   # shared: no inter-block
    r = _one([Access(0, WRITE, c(0)), Access(0, WRITE, c(0))], (0, 1), mask=0)
    assert r["flags"] & 1


def test_statuses():
    # divide by zero in the guard (evaluated everywhere)
    r = _one([Access(0, WRITE, tid(), div(tid(), param(0) - 3))], (0, 0))
    assert r["status"] == -4 and r["count"] == 0 and r["verdict"] == 0
    # divide by zero in the address only where the guard is false: fine
    r = _one([Access(0, WRITE, div(c(1), tid() - 7), lt(tid(), 7))], (0, 0))
    assert r["status"] == 0
    # overflow in the address
    r = _one([Access(0, WRITE, c(I64MAX) + tid())], (0, 0))
    assert r["status"] == -3
    # divide-by-zero outranks overflow, even in another tuple
    r = _one([Access(0, WRITE, div(c(I64MAX) + param(0), param(0) - 3))], (0, 0),
             sets=([1], [3]))
    assert r["status"] == -4
    # 32-bit array, address outside int32
    r = _one([Access(1, WRITE, c(1 << 31) + tid())], (0, 0))
    assert r["status"] == -3
    # block of more than 1024 threads
    r = _one([Access(0, WRITE, tid())], (0, 0), launch=Launch((1, 1, 1), (2048, 1, 1)))
    assert r["status"] == -2
    # interval id outside [0, 65536)
    r = _one([Access(0, WRITE, tid(), bint=c(-1))], (0, 0))
    assert r["status"] == -2
    # malformed expression, unknown parameter, pair across arrays
    bad = Access(0, WRITE, E([("const", 1), ("add",)]))
    assert _one([bad], (0, 0))["status"] == -1
    assert _one([Access(0, WRITE, param(5))], (0, 0))["status"] == -1
    assert _one([Access(0, WRITE, tid()), Access(1, WRITE, tid())], (0, 1))["status"] == -1
    # loop variable outside the access's loops; tid in a loop bound
    assert _one([Access(0, WRITE, loop(0))], (0, 0),
                loops=[Loop(0, "lt", 3)])["status"] == -1
    assert _one([Access(0, WRITE, loop(0), loops=[0])], (0, 0),
                loops=[Loop(0, "lt", tid())])["status"] == -1
    # too many iterations
    assert _one([Access(0, WRITE, loop(0), loops=[0])], (0, 0),
                loops=[Loop(0, "lt", 1 << 20)])["status"] == -2
    # an empty launch (a zero extent) has no points
    r = _one([Access(0, WRITE, c(0))], (0, 0), launch=Launch((param(0) - 3, 1, 1), (8, 1, 1)))
    assert r["status"] == 0 and r["verdict"] == 0


@pytest.mark.parametrize("G,B,w", [(4, 64, 32), (3, 32, 8), (2, 16, 4)])
def test_f1_in_loop_interval_ids(G, B, w):
    """F1 inside a two-iteration loop i in {0, 1} whose addresses do not
    depend on i; each conflicting thread pair of F1 then meets in 2 x 2
    iteration pairs.  Derived by hand:
      * wint = i, bint constant: inter-block ignores barriers (4 (G - 1));
        intra-block needs equal bint only (4 G (B/w - 1)); intra-warp also
        needs equal wint, so only i_p = i_q (2 G (B - B/w)).  Witness: p =
        (b0, t1, i0) with q = (b0, t0, i0), same warp, equal wint.
      * bint = i (a block barrier in the loop body): intra-block and
        intra-warp both need i_p = i_q: [4 (G - 1), 2 G (B/w - 1),
        2 G (B - B/w)]."""
    g = bid(0) * bdim(0) + tid(0)
    lp = [Loop(0, "lt", 2)]
    for kw, want in (({"wint": loop(0)},
                      [4 * (G - 1), 4 * G * (B // w - 1), 2 * G * (B - B // w)]),
                     ({"bint": loop(0)},
                      [4 * (G - 1), 2 * G * (B // w - 1), 2 * G * (B - B // w)])):
        m = Model(0, [Array(GLOBAL, 32)],
                  [Access(0, WRITE, g, None, [0], **kw),
                   Access(0, WRITE, g + 1, None, [0], **kw)],
                  Launch((G, 1, 1), (B, 1, 1), w), [[]], loops=lp)
        r = both(Workload([m], [(0, 0, 1, 7)]))[0]
        assert r["status"] == 0
        assert r["by_class"] == want, (kw, r)
        assert r["count"] == sum(want)
        assert r["witness"] == (0, 0, 1, 0, 0, 0, 0)
        assert r["witness_class"] == INTRA_WARP and r["w_addr"] == 1


def test_error_precedence_five_loops():
    """Status precedence (EINVAL > EUNSUPPORTED > EDIVZERO > ERANGE over the
    errors of a pair), with one reading for an access that lists more loops
    than the interface's four slots: that access is EUNSUPPORTED as a whole
    (its loop list cannot be described, so its expressions, which may name
    those loops, are not examined); the other access and the pair itself are
    still examined, and an EINVAL there wins."""
    loops = [Loop(0, "lt", 2)] * 5
    five = Access(0, WRITE, E([("const", 1), ("add",)]), loops=[0, 1, 2, 3, 4])
    ok = Access(0, WRITE, tid())
    bad = Access(0, WRITE, E([("const", 1), ("add",)]))
    assert _one([five], (0, 0), loops=loops)["status"] == -2
    assert _one([five, ok], (0, 1), loops=loops)["status"] == -2
    assert _one([five, bad], (0, 1), loops=loops)["status"] == -1
    # a pair across arrays is EINVAL whatever the accesses hold
    other = Access(1, WRITE, tid())
    assert _one([five, other], (0, 1), loops=loops)["status"] == -1
