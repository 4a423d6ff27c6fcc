"""rd_check_pairs_noalloc (every device buffer in the library's fixed
scratch area) against rd_check_pairs on the same inputs, field by field:
two calls in a row, the second smaller, then a batch too large for the
area (RD_ECAPACITY, decided on the host before any kernel runs), then the
small batch again."""
import sys

import pytest

from workloads import (Access, Array, Launch, Loop, Model, Workload, c, param,
                       tid, bid, loop, GLOBAL, SHARED, WRITE, READ)
from workloads import configs

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2604_02106_amd as hg
    return hg


def skew_workload():
    """Hot addresses at three scales (re-bucketing, split by (address,
    block), HBM aggregation), a shared array and a plain HBM item."""
    m = Model(1, [Array(GLOBAL, 32), Array(SHARED, 32)],
              [Access(0, WRITE, tid() % 8, loops=[0]),
               Access(0, READ, tid() % 8 + loop(0) * 0, loops=[0]),
               Access(0, WRITE, tid() // 32 + bid() * 0, loops=[0]),
               Access(0, WRITE, c(0) + loop(0) * 0, loops=[0]),
               Access(0, WRITE, tid() + bid() * 64 + loop(0), loops=[0]),
               Access(1, WRITE, tid() % 2 + loop(0), loops=[0])],
              Launch((param(0), 1, 1), (256, 1, 1), 32), [[24], [10]],
              loops=[Loop(0, "lt", 12)])
    pairs = [(0, 0, 0, 7), (0, 0, 1, 7), (0, 2, 2, 7), (0, 3, 3, 7), (0, 3, 0, 7),
             (0, 4, 4, 7), (0, 4, 0, 7), (0, 5, 5, 7), (0, 0, 1, 1), (0, 2, 2, 6)]
    return Workload([m], pairs)


def too_big_workload():
    """One pair whose records alone (2 x 2^25 points, 8 B each) exceed the
    scratch area."""
    m = Model(0, [Array(GLOBAL, 32)],
              [Access(0, WRITE, tid() + bid() * 256), Access(0, READ, tid() + bid() * 256 + 1)],
              Launch((1 << 17, 1, 1), (256, 1, 1), 32), [[]])
    return Workload([m], [(0, 0, 1, 7)])


def test_noalloc_matches_check_pairs(hg):
    ctx = hg.Context(0)
    big, small = skew_workload(), configs.tiny()
    assert len(small.pairs) > 0
    for name, wl in (("skew (10 pairs, 24 x 256 x 12 points)", big),
                     ("tiny (64 pairs, 4 x 64 x 8 points)", small)):
        say("noalloc", name)
        want = hg.rd_check_pairs(ctx, wl)
        st, got = hg.rd_check_pairs_noalloc(ctx, wl)
        assert st == hg.RD_OK, hg.rd_strerror(st)
        s = ctx.stats()
        say("stats", {k: s[k] for k in ("small_items", "hbm_items", "retry_items",
                                         "split_items", "overflow_items")})
        assert got == want, name
        if wl is big:
            assert s["hbm_items"] > 0 and s["split_items"] > 0 and s["overflow_items"] > 0
    say("noalloc too big")
    st, got = hg.rd_check_pairs_noalloc(ctx, too_big_workload())
    assert st == hg.RD_ECAPACITY and got is None
    say("noalloc tiny after the capacity error")
    st, got = hg.rd_check_pairs_noalloc(ctx, small)
    assert st == hg.RD_OK and got == hg.rd_check_pairs(ctx, small)
    ctx.close()
