"""Aliased array views and vector accesses on the GPU against the CPU
oracle, field by field: the hand-pinned cases of tests/test_alias_oracle.py
at several sizes and random models whose arrays are views of one memory.
Every case prints its name before it runs.
"""
import sys

import numpy as np
import pytest

import oracle
from workloads import (c, tid, bid, loop, Model, Workload, Access, Sync, Array, Launch,
                       Loop, GLOBAL, SHARED, READ, WRITE)
from workloads.random_models import rand_model

pytestmark = pytest.mark.gpu


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


def run_both(hg, wl, name):
    say(name, "pairs=%d" % len(wl.pairs))
    got = hg.check_pairs(wl)
    want, _ = oracle.check_pairs(wl, "B", threads=8)
    for k, (g, w) in enumerate(zip(got, want)):
        assert g == w, "%s pair %d:\n gpu    %r\n oracle %r" % (name, k, g, w)
    return got


@pytest.mark.parametrize("G,N,w", [(1, 64, 32), (3, 256, 32), (40, 512, 64)])
def test_alias_cases(hg, G, N, w):
    arrays = [Array(GLOBAL, 64, alias=1, base=0), Array(GLOBAL, 64, alias=1, base=10),
              Array(GLOBAL, 64, alias=2, base=0), Array(GLOBAL, 64, alias=2, base=3),
              Array(GLOBAL, 32, alias=4, base=(1 << 31) - 100), Array(SHARED, 64, alias=1)]
    lk = lambda arr, e: dict(acq=Sync(arr, e), rel=Sync(arr, e))
    gid = tid() + bid() * N
    accs = [Access(0, WRITE, gid), Access(1, WRITE, gid), Access(1, READ, tid()),
            Access(0, WRITE, c(0), **lk(2, c(5))), Access(0, WRITE, c(0), **lk(3, c(2))),
            Access(4, WRITE, tid()), Access(0, WRITE, tid() * 4 + loop(0), loops=[0]),
            Access(1, READ, tid() + bid()), Access(5, WRITE, tid())]
    m = Model(0, arrays, accs, Launch((G, 1, 1), (N, 1, 1), w), [[]],
              loops=[Loop(0, "lt", 4)])
    pairs = [(0, 1), (1, 0), (0, 2), (3, 4), (5, 5), (6, 2), (6, 7), (0, 8), (7, 6)]
    got = run_both(hg, Workload([m], [(0, a, b, 7) for (a, b) in pairs]),
                   "alias G=%d N=%d" % (G, N))
    assert got[7]["status"] == -1  # a global and a shared view: two memories
    assert sum(r["verdict"] for r in got) >= 4


@pytest.mark.parametrize("seed", range(16))
def test_alias_random(hg, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    models, pairs = [], []
    for mi in range(3):
        m = rand_model(rng)
        space = m.arrays[0].space
        m.arrays = [Array(space, 64, alias=1, base=int(rng.integers(-3, 4))),
                    Array(space, 64, alias=1, base=int(rng.integers(-3, 4)))]
        models.append(m)
        for _ in range(6):
            pairs.append((mi, int(rng.integers(0, 4)), int(rng.integers(0, 4)), 7))
    run_both(hg, Workload(models, pairs), "alias random seed=%d" % seed)
