"""Writes the oracle's expected results for the benchmark workloads.

Calls only the CPU oracle (method B, sort + prefix groups; pinned to the
definition by tests/test_oracle.py) on the seeded workloads of ``workloads``;
nothing here touches the GPU library.  Output (gzip JSON, one file per
workload, next to this script):

  batched_2002.json.gz   every one of the 4096 pairs of the batched
                         uneven workload (256 models x 16 pairs, seed 2002)
  mixed_5005_sample.json.gz
                         a stratified sample of the mixed workload (100 000
                         queries, seed 5005): per log2 domain band
                         [8,12) [12,16) [16,20) [20,24) [24,28.2] a fixed
                         number of queries drawn with seed 55, at least 50 in
                         the top band (2^24..2^28 points per access)
  synced_6006.json.gz    every one of the 4000 pairs of the synchronised
                         workload (mixed queries of 2^8..2^22 points under
                         lock and producer/consumer patterns, seed 6006)

Each file holds the workload's digest (sha256 of its JSON), the pair
indices, and per pair: status, verdict, count, by_class[3], classes,
witness_class, flags, witness[7], w_addr, evals.

    python tests/golden/make_goldens.py [batched] [mixed] [synced] [--threads N]
"""
import gzip
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from workloads import configs  # noqa: E402

FIELDS = ("status", "verdict", "count", "by_class", "classes",
          "witness_class", "flags", "witness", "w_addr", "evals")
MIXED_BANDS = ((8, 12, 60), (12, 16, 60), (16, 20, 60), (20, 24, 60),
               (24, 29, 60))


def digest(wl):
    return hashlib.sha256(wl.dumps().encode()).hexdigest()


def encode(r):
    return [r[k] if not isinstance(r[k], tuple) else list(r[k]) for k in FIELDS]


def decode(row):
    d = dict(zip(FIELDS, row))
    d["witness"] = tuple(d["witness"])
    return d


def load(name):
    with gzip.open(os.path.join(HERE, name), "rt") as f:
        g = json.load(f)
    g["results"] = [decode(r) for r in g["results"]]
    return g


def mixed_sample(wl, seed=55):
    """Pair indices of the stratified sample (deterministic)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dom = np.log2(np.array(wl.meta["evals"], dtype=float) / 2)
    out = []
    for lo, hi, n in MIXED_BANDS:
        idx = np.flatnonzero((dom >= lo) & (dom < hi))
        take = rng.choice(idx, size=min(n, len(idx)), replace=False)
        out += sorted(int(i) for i in take)
    return out


def per_set_points(wl, k):
    m = wl.models[wl.pairs[k][0]]
    return wl.meta["evals"][k] // max(1, len(m.param_sets))


def run(wl, idx, threads, mem_gib=40):
    """Oracle B over the pairs idx, in groups whose peak sort memory (about
    48 bytes per point of one tuple, both sides) fits mem_gib."""
    res = {}
    t0 = time.time()
    order = sorted(idx, key=lambda k: wl.meta.get("evals", [0] * len(wl.pairs))[k])
    pos = 0
    while pos < len(order):
        k = order[pos]
        need = 48 * per_set_points(wl, k) if "evals" in wl.meta else 0
        th = max(1, min(threads, int(mem_gib * (1 << 30) // max(1, need))))
        group = order[pos:pos + max(th, 64 if th >= threads else th)]
        sub = wl.subset(group)
        got, _ = oracle.check_pairs(sub, "B", threads=th)
        for kk, r in zip(group, got):
            res[kk] = r
        pos += len(group)
        print("  %d/%d pairs, %.0f s (threads %d)" % (pos, len(order), time.time() - t0, th),
              flush=True)
    return [res[k] for k in idx], time.time() - t0


def write(name, wl, idx, results, secs, threads, extra):
    g = {"workload": wl.name, "digest": digest(wl), "n_pairs": len(wl.pairs),
         "indices": idx, "fields": FIELDS,
         "results": [encode(r) for r in results], "oracle": "B",
         "threads": threads, "seconds": round(secs, 1)}
    g.update(extra)
    with gzip.open(os.path.join(HERE, name), "wt") as f:
        json.dump(g, f)
    print("wrote", name, flush=True)


def main():
    args = sys.argv[1:]
    threads = os.cpu_count() or 1
    if "--threads" in args:
        threads = int(args[args.index("--threads") + 1])
    what = [a for a in args if a in ("batched", "mixed", "synced")] or [
        "batched", "mixed", "synced"]
    if "batched" in what:
        wl = configs.batched(seed=2002)
        idx = list(range(len(wl.pairs)))
        res, secs = run(wl, idx, threads)
        write("batched_2002.json.gz", wl, idx, res, secs, threads,
              {"generator": "configs.batched(seed=2002)"})
    if "mixed" in what:
        wl = configs.mixed(seed=5005)
        idx = mixed_sample(wl)
        res, secs = run(wl, idx, threads)
        write("mixed_5005_sample.json.gz", wl, idx, res, secs, threads,
              {"generator": "configs.mixed(seed=5005)", "sample_seed": 55,
               "bands": MIXED_BANDS})
    if "synced" in what:
        wl = configs.synced(seed=6006)
        idx = list(range(len(wl.pairs)))
        res, secs = run(wl, idx, threads)
        write("synced_6006.json.gz", wl, idx, res, secs, threads,
              {"generator": "configs.synced(seed=6006)"})


if __name__ == "__main__":
    main()
