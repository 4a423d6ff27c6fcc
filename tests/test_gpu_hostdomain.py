"""The race verdicts the paper states for Figures 1-5 (tests/golden/
paper_examples.json), reproduced from tuples that rd_expand_host_domain
builds out of the figures' host code (section 4 classes 1-5), on the GPU,
every field equal to the oracle's."""
import json
import os
import sys

import pytest

import oracle
from workloads import families as F

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def hg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2604_02106_amd as hg
    hg.default_context()
    return hg


def test_paper_examples_from_host_domains(hg):
    golden = {c["id"]: c for c in json.load(open(os.path.join(HERE, "golden",
                                                              "paper_examples.json")))["cases"]}
    cases = [  # (golden case, model builder, host domain)
        ("K1-square", F.k1_copy_upp_low, F.k1_host()),
        ("K1-square-rw", F.k1_copy_upp_low, F.k1_host()),
        ("K2-one-block", F.k2_reduce_final, F.k2_host()),
        ("K3-joint", F.k3_tone_mapping, F.k3_host()),
        ("K4-host-loop", F.k4_lud_internal, F.k4_host()),
        ("K5-pitch", F.k5_shift, F.k5_host((0, 512))),
    ]
    for cid, build, dom in cases:
        g = golden[cid]
        sets = hg.expand_host_domain(dom)
        assert sets, cid
        wl = F.single(build(sets), *g["pair"])
        print("[case]", cid, "tuples", sets, flush=True)
        sys.stdout.flush()
        got = hg.check_pairs(wl)
        want, _ = oracle.check_pairs(wl, "B")
        assert got == want, (cid, got, want)
        assert got[0]["status"] == 0 and got[0]["verdict"] == g["expect"]["verdict"], (cid, got)
