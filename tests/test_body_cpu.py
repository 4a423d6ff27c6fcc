"""Kernel-body front end (section 6.1 "Avoiding race checks"; section 6.5,
Figures 9 and 10): the library's derivation (rd_derive_body, closed forms
over a structured body) against the oracle's (running the body for barrier
counts; dominator chains of an explicit control-flow graph for acquire and
release), on hand-written bodies and on random ones; plus the paper's
barrier example (the tree reduction of Figure 2's kind with a barrier in
the loop) reproduced from its body.
"""
import numpy as np
import pytest

import oracle
from oracle import body as ob
from tests import npeval
from workloads import (c, tid, bid, param, loop, lt, Model, Workload, Access, Array,
                       Launch, Loop, GLOBAL, SHARED, READ, WRITE)
from workloads import families as F


def derive(model, body):
    import paper_2604_02106_amd as hg
    return hg.derive_body(model, body)


def check(model, body):
    """Every access's derived interval ids equal the counts of running the
    body, at every loop-value tuple of every parameter tuple; acquire and
    release equal the dominator-chain search."""
    d = derive(model, body)
    ops = ob.sync_ops(body)
    for k, a in enumerate(d.accesses):
        if k not in ops:
            continue
        acq, rel = ops[k]
        for got, want in ((a.acq, acq), (a.rel, rel)):
            if want is None:
                assert got is None, (k, got)
            else:
                assert got is not None and (got.array, got.addr.code, got.scope) == \
                    (want[0], want[1].code, want[2]), (k, got, want)
    for params in model.param_sets:
        counts = ob.barrier_counts(model, body, params)
        for k, occ in counts.items():
            a = d.accesses[k]
            for vals, (nb, nw) in occ.items():
                assert len(vals) == len(a.loops)
                env = {("param", i): v for i, v in enumerate(params)}
                env.update({("loop", l): v for l, v in zip(a.loops, vals)})
                bi = int(npeval.ev(a.bint, env, (), 0))
                wi = int(npeval.ev(a.wint, env, (), 0))
                assert (bi, wi) == (nb, nw), (k, params, vals, (bi, wi), (nb, nw))
    return d


def model_of(n_acc, loops, sets=([3],), arrays=2):
    accs = [Access(0, WRITE if k % 2 == 0 else READ, tid() + k) for k in range(n_acc)]
    return Model(1, [Array(GLOBAL, 64)] * arrays, accs, Launch((2, 1, 1), (8, 1, 1), 4),
                 [list(s) for s in sets], loops=loops)


LOOPS = [Loop(0, "lt", param(0)), Loop(1, "ge", 0, "sub", 2), Loop(0, "le", 5, "add", 2),
         Loop(1, "lt", 9, "mul", 3)]


def test_tree_reduction_body_gives_the_family_intervals():
    """The tree reduction with a barrier at the end of the loop body: the
    derived bint of all three accesses is the iteration index (the
    hand-written family uses the loop value, 0, 1, ...), and the race query
    gives the same results for both models."""
    m = F.f2_tree_reduction(64, barrier=False)
    body = [("loop", 0), ("access", 2), ("access", 1), ("access", 0), ("barrier",), ("end",)]
    d = check(m, body)
    want = F.f2_tree_reduction(64, barrier=True)
    pairs = [(0, 0, 1, 7), (0, 0, 2, 7), (0, 0, 0, 7)]
    ra = oracle.check_pairs(Workload([d], pairs), "B", threads=4)[0]
    rb = oracle.check_pairs(Workload([want], pairs), "B", threads=4)[0]
    assert ra == rb
    assert all(r["verdict"] == 0 for r in ra)  # the barrier removes every race
    # without the barrier the first pair races (section 4's example)
    nob = check(m, body[:4] + body[5:])
    assert oracle.check_pairs(Workload([nob], pairs), "B")[0][0]["verdict"] == 1


def test_nested_loops_branches_and_locks():
    m = model_of(4, LOOPS[:2], sets=([3], [0], [5]))
    body = [("barrier",), ("cas", 1, bid(), "device"), ("fence", "device"),
            ("loop", 0), ("access", 0), ("warp_barrier",),
            ("loop", 1), ("barrier",), ("access", 1), ("end",),
            ("if",), ("barrier",), ("access", 2), ("else",), ("warp_barrier",), ("end",),
            ("barrier",), ("end",),
            ("access", 3),
            ("fence", "block"), ("exch", 1, bid(), "device")]
    d = check(m, body)
    assert d.accesses[0].acq.scope == "device" and d.accesses[0].rel.scope == "block"
    assert d.accesses[1].loops == [0, 1]


def test_loops_without_closed_forms_count_no_barrier():
    m = model_of(3, [LOOPS[2], LOOPS[3]])
    body = [("loop", 1), ("barrier",), ("access", 0), ("end",),
            ("loop", 0), ("barrier",), ("access", 1), ("loop", 1), ("warp_barrier",),
            ("end",), ("access", 2), ("end",)]
    d = check(m, body)
    assert d.accesses[0].bint is None  # a MUL loop: its barrier counts for nothing


def test_acquire_release_search():
    """Figure 10: fence first, then a CAS before it (acquire); fence first,
    then an Exch after it (release); operations inside a branch or a loop
    that does not contain the access do not dominate it; the nearest pair
    is taken."""
    m = model_of(6, LOOPS[:1])
    body = [("cas", 0, c(1), "device"), ("fence", "device"),
            ("cas", 1, tid() % 2, "block"),          # no fence after it: not an acquire
            ("access", 0),                            # acq: cas(0, 1)
            ("if",), ("fence", "device"), ("cas", 1, c(5), "device"), ("end",),
            ("access", 1),                            # the branch dominates nothing
            ("loop", 0), ("cas", 1, loop(0), "device"), ("fence", "block"),
            ("access", 2),                            # acq: cas(1, i) at block scope
            ("fence", "device"), ("exch", 1, loop(0), "device"), ("end",),
            ("access", 3),                            # rel: after the loop
            ("fence", "device"),
            ("access", 4), ("exch", 0, c(2), "device"),
            ("if",), ("access", 5), ("fence", "device"), ("exch", 1, c(7), "device"),
            ("else",), ("end",)]
    d = check(m, body)
    a = d.accesses
    assert (a[0].acq.array, a[0].acq.addr.code) == (0, c(1).code)
    assert (a[2].acq.array, a[2].acq.scope) == (1, "block")
    assert a[2].rel is not None and a[2].rel.addr.code == loop(0).code
    assert a[5].rel is not None and a[5].rel.addr.code == c(7).code


def _random_body(rng, n_acc, n_loops):
    """A random well-formed body naming each access once."""
    out, accs = [], list(range(n_acc))
    rng.shuffle(accs)
    depth = []

    def stmt():
        r = rng.random()
        if r < 0.25:
            return ("barrier",)
        if r < 0.35:
            return ("warp_barrier",)
        if r < 0.5:
            return ("fence", ["block", "device"][int(rng.integers(0, 2))])
        open_loops = [x for x in depth if isinstance(x, int)]
        e = [c(int(rng.integers(0, 3))), tid() % 2, bid()] + [loop(l) for l in open_loops]
        ex = e[int(rng.integers(0, len(e)))]
        return (["cas", "exch"][int(rng.integers(0, 2))], int(rng.integers(0, 2)), ex,
                ["block", "device"][int(rng.integers(0, 2))])

    while accs or depth:
        r = rng.random()
        if accs and r < 0.3:
            out.append(("access", accs.pop()))
        elif r < 0.45 and len(depth) < 3:
            free = [l for l in range(n_loops) if l not in depth]
            if free and rng.random() < 0.6:
                l = free[int(rng.integers(0, len(free)))]
                out.append(("loop", l))
                depth.append(l)
            else:
                out.append(("if",))
                depth.append("if")
        elif r < 0.55 and depth:
            if depth[-1] == "if" and rng.random() < 0.5:
                out.append(("else",))
                depth[-1] = "else"
            else:
                out.append(("end",))
                depth.pop()
        elif not accs and depth:
            out.append(("end",))
            depth.pop()
        else:
            out.append(stmt())
    return out


@pytest.mark.parametrize("seed", range(40))
def test_random_bodies(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    m = model_of(5, LOOPS, sets=([2], [4]))
    body = _random_body(rng, 5, 4)
    check(m, body)


def test_malformed_bodies():
    m = model_of(2, LOOPS[:1])
    bad = [[("end",)], [("if",), ("access", 0)], [("else",)], [("loop", 0), ("else",), ("end",)],
           [("access", 0), ("access", 0)], [("loop", 7), ("end",)], [("access", 9)],
           [("loop", 0), ("loop", 0), ("end",), ("end",)],
           [("cas", 5, c(0), "device")], [("cas", 1, loop(0), "device")]]
    for b in bad:
        with pytest.raises(RuntimeError, match="invalid"):
            derive(m, b)
