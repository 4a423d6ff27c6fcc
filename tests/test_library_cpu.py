"""Host-only checks of the GPU library: it loads, exports every entry point
that include/hgrd.h declares, its integer helpers pass their self-checks,
and the binding's structures have the header's sizes.  No compute runs."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "hgrd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rd_\w+)\s*\(", text)))


def test_exports_every_declared_symbol():
    import paper_2604_02106_amd as hg
    L = hg.lib()
    names = _declared()
    assert "rd_check_pairs" in names and "rd_context_create" in names
    for n in names:
        assert hasattr(L, n), n


def test_selftest_and_strerror():
    import paper_2604_02106_amd as hg
    L = hg.lib()
    L.rd_selftest.restype = C.c_int
    assert L.rd_selftest() == 0
    assert hg.rd_strerror(-4) == "division by zero"


def test_struct_sizes():
    import paper_2604_02106_amd as hg
    assert C.sizeof(hg.rd_pair_result) == 88
    assert C.sizeof(hg.rd_insn) == 16
    assert C.sizeof(hg.rd_access) == 96
    assert C.sizeof(hg.rd_array) == 24
    assert C.sizeof(hg.rd_sync) == 16
    assert C.sizeof(hg.rd_options) == 48
    assert C.sizeof(hg.rd_mlp) == 4 * 6337
    assert C.sizeof(hg.rd_stats) == 41 * 8


def test_packed_concat_keeps_every_model():
    """Packed.concat lays several images' models end to end: each model's
    descriptor and the instructions it points to are the part's."""
    import paper_2604_02106_amd as hg
    from workloads import configs
    wl = configs.mixed(seed=11, n_queries=40, log2_max=12)
    parts = [hg.Packed(wl.compact(range(0, 17))), hg.Packed(wl.compact(range(17, 40)))]
    pk = hg.Packed.concat(parts)
    assert pk.n_models == parts[0].n_models + parts[1].n_models
    k = 0
    for p in parts:
        for i in range(p.n_models):
            a, b = pk.models[k], p.models[i]
            assert (a.n_insns, a.n_arrays, a.n_loops, a.n_acc, a.n_params) == \
                   (b.n_insns, b.n_arrays, b.n_loops, b.n_acc, b.n_params)
            assert [(a.insns[j].op, a.insns[j].imm) for j in range(a.n_insns)] == \
                   [(b.insns[j].op, b.insns[j].imm) for j in range(b.n_insns)]
            assert pk.launch[k].warp_size == p.launch[i].warp_size
            assert pk.params[k].n_sets == p.params[i].n_sets
            k += 1


def test_no_device_fails_loudly():
    import paper_2604_02106_amd as hg
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    with pytest.raises(RuntimeError):
        hg.Context(0)
