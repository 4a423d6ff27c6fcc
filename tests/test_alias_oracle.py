"""Pins of aliased array views and vector accesses (the paper is silent on
both; the reading: views with one alias id share their elements, element k
of a view being element base + k of the memory; a vector access of w
elements is an access in an extra loop of w iterations).  Closed forms by
hand; both oracle methods.
"""
import numpy as np
import pytest

import oracle
from workloads import (c, tid, bid, loop, Model, Workload, Access, Sync, Array, Launch,
                       Loop, GLOBAL, SHARED, READ, WRITE, INTRA_BLOCK, INTRA_WARP)
from workloads.random_models import rand_model


def both(wl):
    ra = oracle.check_pairs(wl, "A", threads=4)[0]
    rb = oracle.check_pairs(wl, "B", threads=4)[0]
    assert ra == rb
    return ra


def one_block(arrays, accs, pairs, N=64, w=32, G=1, loops=()):
    m = Model(0, arrays, accs, Launch((G, 1, 1), (N, 1, 1), w), [[]], loops=loops)
    return both(Workload([m], [(0, a, b, 7) for (a, b) in pairs]))


def test_two_views_with_an_offset():
    """W A[t] against W B[t] where B starts 10 elements into A's memory:
    thread t of A meets thread t - 10 of B (t >= 10).  With 64 threads and
    warps of 32: t in [10, 32) and [42, 64) pair inside one warp (22 + 22),
    t in [32, 42) across warps (10)."""
    arrays = [Array(GLOBAL, 64, alias=1, base=0), Array(GLOBAL, 64, alias=1, base=10)]
    r = one_block(arrays, [Access(0, WRITE, tid()), Access(1, WRITE, tid())], [(0, 1), (1, 0)])
    assert r[0]["by_class"] == [0, 10, 44]
    assert r[1]["by_class"] == [0, 10, 44]
    # witness: smallest p of A with a partner: t = 10, partner thread 0 of B
    assert r[0]["witness"] == (0, 0, 10, 0, 0, 0, 0) and r[0]["w_addr"] == 10


def test_views_and_memories():
    """Different alias ids, or one id in two spaces, are different memories:
    a pair across them is malformed; without an alias an array is its own
    memory whatever its base."""
    arrays = [Array(GLOBAL, 64, alias=1), Array(GLOBAL, 64, alias=2),
              Array(SHARED, 64, alias=1), Array(GLOBAL, 64, alias=0, base=7),
              Array(GLOBAL, 64, alias=0)]
    accs = [Access(k, WRITE, tid()) for k in range(5)]
    r = one_block(arrays, accs, [(0, 1), (0, 2), (3, 4), (3, 3)])
    assert [x["status"] for x in r] == [-1, -1, -1, 0]
    assert r[3]["by_class"] == [0, 0, 0]


def test_lock_through_two_views():
    """A lock taken through two views of one memory at one element is one
    lock: lock(V1[5]) and lock(V2[2]) with V2 starting 3 elements in."""
    arrays = [Array(GLOBAL, 64), Array(GLOBAL, 64, alias=3, base=0),
              Array(GLOBAL, 64, alias=3, base=3)]
    lk = lambda arr, e: dict(acq=Sync(arr, e), rel=Sync(arr, e))
    accs = [Access(0, WRITE, c(0), **lk(1, c(5))), Access(0, WRITE, c(0), **lk(2, c(2))),
            Access(0, WRITE, c(0), **lk(2, c(3)))]
    r = one_block(arrays, accs, [(0, 1), (0, 2)], N=8, w=4, G=2)
    assert r[0]["by_class"] == [0, 0, 0]
    assert r[1]["by_class"] == [2 * 1 * 8 * 8, 2 * 8 * 4, 2 * 8 * 3]


def test_effective_address_errors():
    """base + address overflowing int64 is a range error; a 32-bit view
    must keep its effective address in int32."""
    big = (1 << 63) - 2
    arrays = [Array(GLOBAL, 64, alias=1, base=big), Array(GLOBAL, 32, alias=2, base=(1 << 31) - 4),
              Array(GLOBAL, 64, alias=1, base=0)]
    accs = [Access(0, WRITE, tid()), Access(1, WRITE, tid()), Access(2, WRITE, tid())]
    r = one_block(arrays, accs, [(0, 0), (1, 1), (2, 2)], N=8, w=4)
    assert [x["status"] for x in r] == [-3, -3, 0]


@pytest.mark.parametrize("N,w", [(64, 32), (32, 8)])
def test_vector_access_as_a_loop(N, w):
    """A float4 store V[t] (elements 4t .. 4t + 3, an extra loop j < 4 with
    address 4t + j) against a float load S[t] of the same memory: thread t's
    element t is inside thread t // 4's vector; the pair (p = (u, j), q = t)
    conflicts when 4u + j = t and u != t, so for every t >= 1 exactly one
    ordered pair; its class is that of threads t // 4 and t."""
    arrays = [Array(GLOBAL, 64)]
    accs = [Access(0, WRITE, tid() * 4 + loop(0), loops=[0]), Access(0, READ, tid())]
    r = one_block(arrays, accs, [(0, 1)], N=N, w=w, loops=[Loop(0, "lt", 4)])
    warp = sum(1 for t in range(1, N) if (t // 4) // w == t // w)
    assert r[0]["by_class"] == [0, N - 1 - warp, warp]


@pytest.mark.parametrize("seed", range(16))
def test_methods_agree_random_aliased(seed):
    """Random models whose two arrays are views of one memory (random bases,
    pairs across the views)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    models, pairs = [], []
    for mi in range(3):
        m = rand_model(rng)
        space = m.arrays[0].space
        m.arrays = [Array(space, 64, alias=1, base=int(rng.integers(-3, 4))),
                    Array(space, 64, alias=1, base=int(rng.integers(-3, 4)))]
        models.append(m)
        for _ in range(6):
            a, b = int(rng.integers(0, 4)), int(rng.integers(0, 4))
            pairs.append((mi, a, b, 7))
    both(Workload(models, pairs))
