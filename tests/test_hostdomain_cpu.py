"""rd_expand_host_domain (section 4 classes 1-5, section 6.3) through the C
ABI, host only: the tuples of the paper's Figures 1-5 host code written out
by hand, a brute-force enumeration of small random host domains, statuses,
and the tile-scoring network's weight file."""

import numpy as np
import pytest

from workloads import HostDomain, HostVar, c, param, eq, lt, gt, land
from workloads import families as F

from tests.npeval import ev


@pytest.fixture(scope="module")
def hg():
    import paper_2604_02106_amd as hg
    hg.lib()
    return hg


def test_k1_assert_keeps_square_matrices(hg):
    # Figure 1: assert(rows == cols) keeps only the equal pairs
    assert hg.expand_host_domain(F.k1_host()) == [[16, 16], [32, 32], [48, 48]]


def test_k2_one_block(hg):
    # Figure 2: reduceFinal<<<1, THREADS>>>: one tuple, gridDim.x = 1
    assert hg.expand_host_domain(F.k2_host()) == [[1]]


def test_k3_width_and_grid_from_one_variable(hg):
    # Figure 3: grid.x = hWidth / 16 and width = hWidth, joint
    assert hg.expand_host_domain(F.k3_host()) == [[16, 1, 2], [32, 2, 2], [48, 3, 2]]


def test_k4_offset_from_host_loop(hg):
    # Figure 4: offset iterates [0, hMatrixDim) in steps of 16
    assert hg.expand_host_domain(F.k4_host()) == [[64, 0], [64, 16], [64, 32], [64, 48]]
    assert hg.expand_host_domain(F.k4_host((32, 48))) == [[32, 0], [32, 16], [48, 0],
                                                         [48, 16], [48, 32]]


def test_k5_allocation_size_positive(hg):
    # Figure 5: the pitch sizes an allocation, so 0 is not a value it takes
    assert hg.expand_host_domain(F.k5_host()) == [[256], [512]]
    assert hg.expand_host_domain(F.k5_host((0, -4))) == []


def _brute(dom):
    """Reference enumeration written out with itertools and explicit loops
    (values small: no overflow)."""
    out = []

    def val(e, env):
        return int(ev(e, {("param", k): v for k, v in env.items()}, (), 0))

    def walk(k, env):
        if k == len(dom.vars):
            if any(val(a, env) == 0 for a in dom.asserts):
                return
            if any(val(a, env) <= 0 for a in dom.alloc_sizes):
                return
            row = [val(p, env) for p in dom.params]
            if row not in out:
                out.append(row)
            return
        v = dom.vars[k]
        if v.kind == "input":
            for x in v.values:
                walk(k + 1, {**env, k: x})
        elif v.kind == "expr":
            walk(k + 1, {**env, k: val(v.init, env)})
        else:
            it, bound, step = val(v.init, env), val(v.bound, env), val(v.step, env)
            cmp = {"lt": lambda a, b: a < b, "le": lambda a, b: a <= b,
                   "gt": lambda a, b: a > b, "ge": lambda a, b: a >= b,
                   "ne": lambda a, b: a != b}[v.cmp]
            while cmp(it, bound):
                walk(k + 1, {**env, k: it})
                it = {"add": it + step, "sub": it - step, "mul": it * step}[v.upd]

    walk(0, {})
    return out


@pytest.mark.parametrize("seed", range(12))
def test_random_domains_match_brute_force(hg, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    a = HostVar.input(sorted(set(int(x) for x in rng.integers(-3, 9, 4))))
    b = HostVar.input([int(x) for x in rng.integers(0, 6, 3)])
    lo = int(rng.integers(-2, 2))
    loop = HostVar.loop(lo, "lt", param(0) + 3, "add", int(rng.integers(1, 3)))
    der = HostVar.expr(param(1) * 2 + param(2))
    dom = HostDomain([a, b, loop, der],
                     params=[param(0), param(2) - param(1), param(3) // 3, c(7)],
                     asserts=[lt(param(1), param(0) + 4)] if seed % 2 else [],
                     alloc_sizes=[param(3) + 1] if seed % 3 else [])
    assert hg.expand_host_domain(dom) == _brute(dom)


def test_equal_tuples_kept_once(hg):
    dom = HostDomain([HostVar.input([1, 2, 3, 4])], params=[param(0) // 2])
    assert hg.expand_host_domain(dom) == [[0], [1], [2]]


def test_statuses(hg):
    import paper_2604_02106_amd as H
    # a thread coordinate is not a host value
    from workloads import tid
    with pytest.raises(RuntimeError, match=r"\(-1\)"):
        hg.expand_host_domain(HostDomain([], params=[tid(0)]))
    # a variable read before it is set
    with pytest.raises(RuntimeError, match=r"\(-1\)"):
        hg.expand_host_domain(HostDomain([HostVar.expr(param(0))], params=[param(0)]))
    # division by zero in one assignment
    with pytest.raises(RuntimeError, match=r"\(-4\)"):
        hg.expand_host_domain(HostDomain([HostVar.input([2, 0])], params=[c(8) // param(0)]))
    # overflow
    with pytest.raises(RuntimeError, match=r"\(-3\)"):
        hg.expand_host_domain(HostDomain([HostVar.input([1 << 62])], params=[param(0) * 4]))
    # a host loop of more than 65536 iterations
    with pytest.raises(RuntimeError, match=r"\(-2\)"):
        hg.expand_host_domain(HostDomain([HostVar.loop(0, "lt", 1 << 20)], params=[param(0)]))
    # a buffer too small for every tuple
    with pytest.raises(RuntimeError, match=r"\(-7\)"):
        hg.expand_host_domain(HostDomain([HostVar.input(range(10))], params=[param(0)]),
                              cap_values=4)
    assert H.RD_ECAPACITY == -7


def test_mlp_weight_file_roundtrip(hg, tmp_path):
    w = np.random.Generator(np.random.PCG64(3)).normal(0, 1, hg.N_MLP).astype(np.float32)
    p = str(tmp_path / "w.hgrdmlp")
    hg.mlp_save(w, p, 5)
    raw = open(p, "rb").read()
    assert raw[:8] == b"HGRDMLP1" and len(raw) == 32 + 4 * hg.N_MLP
    w2, fv = hg.mlp_load(p)
    assert fv == 5 and np.array_equal(w, w2)
    # a truncated file is refused
    open(p, "wb").write(raw[:100])
    with pytest.raises(RuntimeError):
        hg.mlp_load(p)
    with pytest.raises(RuntimeError):
        hg.mlp_load(str(tmp_path / "missing"))
