"""Models derived from kernel bodies (rd_derive_body: barrier-interval ids,
acquire and release from a structured body) on the GPU against the CPU
oracle, field by field.  Every case prints its name before it runs.
"""
import sys

import numpy as np
import pytest

import oracle
from tests.test_body_cpu import _random_body, LOOPS
from workloads import (c, tid, bid, Model, Workload, Access, Array, Launch, GLOBAL,
                       READ, WRITE, ATOMIC)

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


ADDRS = [c(0), tid() % 3, tid() // 2, bid(), tid() % 2 + bid()]


def derived_workload(hg, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    kinds = [WRITE, READ, WRITE, ATOMIC, READ]
    accs = [Access(0, kinds[k], ADDRS[int(rng.integers(0, len(ADDRS)))]) for k in range(5)]
    m = Model(1, [Array(GLOBAL, 64), Array(GLOBAL, 64)], accs,
              Launch((3, 1, 1), (16, 1, 1), 4), [[2], [3]], loops=LOOPS)
    d = hg.derive_body(m, _random_body(rng, 5, 4))
    pairs = [(0, a, b, 7) for a in range(5) for b in range(a, 5)]
    return Workload([d], pairs)


@pytest.mark.parametrize("seed", range(20))
def test_derived_models(hg, seed):
    wl = derived_workload(hg, seed)
    say("derived body seed=%d" % seed, "pairs=%d" % len(wl.pairs))
    got = hg.check_pairs(wl)
    want, _ = oracle.check_pairs(wl, "B", threads=8)
    for k, (g, w) in enumerate(zip(got, want)):
        assert g == w, "seed %d pair %d:\n gpu    %r\n oracle %r" % (seed, k, g, w)
