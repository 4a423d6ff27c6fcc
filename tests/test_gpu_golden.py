"""Full-size parity against stored oracle results (tests/golden/, written by
tests/golden/make_goldens.py, which calls only the CPU oracle):

* every one of the 4096 pairs of the batched uneven workload (256 models x
  16 pairs, seed 2002), in one plan as bench.py runs it;
* the stratified sample of the mixed workload (100 000 queries, seed 5005;
  60 queries per log2 domain band, the top band 2^24..2^28 points per
  access), both as one plan of the sampled queries and inside the
  5000-query batch of bench.py's step that holds the most of them.

Every field is compared: status, verdict, count, per-class counts, classes,
witness (lexicographically smallest), witness class and address, flags,
evals."""
import os
import sys

import pytest

from workloads import configs

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_goldens as G  # noqa: E402

STEP = 5000  # queries per bench.py step on the mixed workload


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


def _check(got, gold, idx, name):
    bad = []
    for k, i in enumerate(idx):
        g = {f: got[k][f] for f in G.FIELDS}
        g["by_class"] = list(g["by_class"])
        w = dict(gold[k])
        w["by_class"] = list(w["by_class"])
        if g != w:
            bad.append((i, g, w))
    assert not bad, "%s: %d of %d differ, first: pair %d\n gpu    %r\n oracle %r" % (
        name, len(bad), len(idx), bad[0][0], bad[0][1], bad[0][2])


def test_batched_every_pair(hg):
    gold = G.load("batched_2002.json.gz")
    wl = configs.batched(seed=2002)
    assert G.digest(wl) == gold["digest"], "generator changed since the goldens were written"
    say("batched golden", len(wl.pairs))
    got = hg.check_pairs(wl)
    _check(got, gold["results"], gold["indices"], "batched")
    assert sum(r["verdict"] for r in got) > 0


def test_mixed_sample(hg):
    path = os.path.join(HERE, "golden", "mixed_5005_sample.json.gz")
    if not os.path.exists(path):
        pytest.skip("mixed goldens not written yet")
    gold = G.load("mixed_5005_sample.json.gz")
    wl = configs.mixed(seed=5005)
    assert G.digest(wl) == gold["digest"], "generator changed since the goldens were written"
    idx = gold["indices"]
    say("mixed golden sample", len(idx))
    got = hg.check_pairs(wl.compact(idx))
    _check(got, gold["results"], idx, "mixed sample")
    # the bench step (5000 consecutive queries) holding the most sampled ones
    steps = {}
    for k, i in enumerate(idx):
        steps.setdefault(i // STEP, []).append(k)
    s = max(steps, key=lambda t: len(steps[t]))
    lo, hi = s * STEP, min(len(wl.pairs), (s + 1) * STEP)
    say("mixed golden step", s, "queries", lo, hi, "sampled", len(steps[s]))
    res = hg.check_pairs(wl.compact(range(lo, hi)))
    _check([res[idx[k] - lo] for k in steps[s]], [gold["results"][k] for k in steps[s]],
           [idx[k] for k in steps[s]], "mixed step %d" % s)


@pytest.mark.parametrize("path", ["lds", "fallback"])
def test_synced_every_pair(hg, monkeypatch, path):
    """All 4000 pairs of the synchronised workload against the oracle's
    stored results, through the LDS joins (where they qualify) and all
    through the HBM aggregation path."""
    gold = G.load("synced_6006.json.gz")
    wl = configs.synced(seed=6006)
    assert G.digest(wl) == gold["digest"], "generator changed since the goldens were written"
    if path == "fallback":
        monkeypatch.setenv("HGRD_SYNC_FALLBACK", "1")
    say("synced golden", len(wl.pairs), path)
    got = hg.check_pairs(wl)
    _check(got, gold["results"], gold["indices"], "synced " + path)
    assert sum(r["verdict"] for r in got) > 100
