"""Benchmark: exact race queries per second on one MI355X.

Default workload: the mixed batched workload at full size (100 000 queries
over 6250 kernel models, per-query domain log-uniform in 2^8..2^28 points,
1-64 parameter tuples per model, 2-D/3-D launches, global and shared arrays,
10% racy; seed 5005; about 3.98e12 thread-access evaluations).  It runs as
20 fixed batches of 5000 consecutive queries, each prepared once beforehand
(descriptors and term tables resident in HBM); one step = one rd_execute of
one batch: every generate / partition / filter / join kernel, the
re-partition rounds, witness pass 2 and the results copied back.  The 20
timed steps cover the workload exactly once.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--config ...]
"""
import argparse
import ctypes
import json
import os
import sys
import time
import types

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM counter summary of the mixed workload's dominant kernel (the
# table-path bucket join)
MIXED_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_counters_mixed.md")
MIXED_STEP = 5000  # queries per step of the mixed workload (20 steps cover it)
# rd_stats fields of the table-path kernels timed per launch with HIP events
# (the context's default LDS tile: 1024 records, 2048 table slots)
KERNELS = (
    ("k_scatter<true>", "scatter_launches", "scatter_tab_ms", "scatter_tab_bytes",
     "generates every point and writes its record (8 B for int32 addresses, 16 B "
     "for int64) into an HBM bucket"),
    ("k_bucket_filter<1024>", "filter_tab_launches", "filter_tab_ms", "filter_tab_bytes",
     "reads every record back and keeps the buckets holding an address of both "
     "accesses (per-wavefront LDS hash table)"),
    ("k_bucket_join<1024, 2048, true, false>", "join_tab_launches", "join_tab_ms",
     "join_tab_bytes", "reads the records of the buckets the filter kept and "
     "joins them in LDS level by level"),
)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2604_02106_amd", "csrc", f)
                  for f in ("hgrd_kernels.hip", "hgrd_device.h", "hgrd_internal.h")]


LIMITER = {
    "k_bucket_join<1024, 2048, true, false>":
        "LDS hash joins level by level with workgroup barriers between levels "
        "(latency- and barrier-bound, not HBM: waves wait about half their "
        "cycles, scalar instructions outnumber vector ones)",
    "k_scatter<true>": "vector ALU issue (decode, table lookups, bucket map, run claims)",
    "k_bucket_filter<1024>": "LDS hash probes per record",
}


def kernel_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(path, field="traffic bytes per launch"):
    """HBM bytes per launch of a kernel from its committed counter summary
    (or another figure of it), if it was taken on the current kernel
    sources (else None)."""
    try:
        text = open(path).read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("source digest") != kernel_digest():
        return None
    try:
        return float(fields[field])
    except (KeyError, ValueError):
        return None


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(wl, gpu_res, budget_s=20.0, seed=7, max_pair_evals=4e6):
    """The oracle (sort + prefix groups) on a bounded random sample of pairs,
    on every host core.  When the workload knows each pair's evals, the
    sample is drawn among pairs of at most max_pair_evals (so that one
    round of pairs stays within the budget) and the rate is scaled to
    queries/s of the whole workload through evals/s: value = (sample evals
    per second) / (mean evals per query of the workload).  The sampled
    pairs are also compared with the GPU results field by field."""
    import numpy as np
    import oracle
    rng = np.random.Generator(np.random.PCG64(seed))
    order = rng.permutation(len(wl.pairs))
    ev_all = wl.meta.get("evals")
    if ev_all and len(ev_all) == len(wl.pairs):
        order = [int(i) for i in order if ev_all[int(i)] <= max_pair_evals]
    else:
        ev_all = None
    threads = os.cpu_count() or 1
    done, t_used, used = 0, 0.0, 1
    step = max(threads, 16)
    evals = 0
    agree = 0
    while done < len(order) and t_used < budget_s:
        idx = [int(i) for i in order[done:done + step]]
        sub = wl.subset(idx)
        t0 = time.perf_counter()
        res, used = oracle.check_pairs(sub, "B", threads=threads)
        t_used += time.perf_counter() - t0
        evals += sum(r["evals"] for r in res)
        agree += sum(1 for i, r in zip(idx, res) if gpu_res[i] == r)
        done += len(idx)
    out = {"value": done / t_used, "unit": "queries/s", "cores": used,
           "kind": "oracle",
           "sample": "%d of %d pairs drawn at random (seed %d), %.1f s, %.3g evals"
                     % (done, len(wl.pairs), seed, t_used, evals),
           "evals_per_s": evals / t_used,
           "agreement": "%d/%d sampled pairs identical to the GPU" % (agree, done)}
    if ev_all:
        mean = float(sum(ev_all)) / len(ev_all)
        out["sample_queries_per_s"] = out["value"]
        out["value"] = evals / t_used / mean
        out["sample"] = ("%d of %d pairs drawn at random among those of at most %.0e evals "
                         "(seed %d), %.1f s, %.3g evals; value = evals/s over the "
                         "workload's mean of %.3g evals per query"
                         % (done, len(wl.pairs), max_pair_evals, seed, t_used, evals, mean))
    return out


def run_learned(args):
    """Learned tile order on sparse witnesses among overlapping tiles
    (16384 queries, G = 256 blocks of 256 threads per side; in a racy query
    one block pair of 2^16 conflicts, and every tile's address ranges
    overlap its diagonal neighbours', so interval pruning leaves about G + 1
    candidates): EXACT, then VERDICT with index order (LEX), interval order
    (tiles proven disjoint last), the untrained network and the trained
    network, each timed over the same steps; tiles examined before the
    first witness."""
    import numpy as np
    import torch
    import paper_2604_02106_amd as hg
    from paper_2604_02106_amd import tile_mlp
    from workloads import configs
    wl = configs.sparse_overlap(seed=4004, n_queries=int(16384 * args.scale))
    try:
        w, meta = tile_mlp.load()
        wsrc = "committed weights (%s)" % os.path.relpath(tile_mlp.DEFAULT, ROOT)
    except (OSError, AssertionError):
        log("no committed weights for these features: training")
        w, _, _ = tile_mlp.train(hg.Context(0))
        wsrc = "trained in this run"
    ctx = hg.Context(0)
    n = len(wl.pairs)
    out = {}
    arms = (("exact", hg.MODE_EXACT, hg.ORDER_LEX, None),
            ("verdict_lex", hg.MODE_VERDICT, hg.ORDER_LEX, None),
            ("verdict_interval", hg.MODE_VERDICT, hg.ORDER_INTERVAL, None),
            ("verdict_mlp", hg.MODE_VERDICT, hg.ORDER_MLP, w))
    # the same network untrained, 4 random initialisations
    arms += tuple(("verdict_untrained%d" % s, hg.MODE_VERDICT, hg.ORDER_MLP,
                   tile_mlp.init_weights(100 + s)) for s in range(4))
    for name, mode, order, wt in arms:
        plan = hg.Plan(ctx, wl, mode=mode, order=order, mlp=wt)
        for _ in range(max(1, args.warmup)):
            res = plan.execute()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.execute(raw=True)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        out[name] = (res, plan.tiles(), dt)
        log("%s: %.3f s per step" % (name, dt))
        plan.close()
    verdicts = [r["verdict"] for r in out["exact"][0]]
    agree = all([r["verdict"] for r in out[k][0]] == verdicts for k in out)
    racy = [k for k, v in enumerate(verdicts) if v]

    def tile_stats(tiles):
        t = np.array([tiles[k] if tiles[k] else 10 ** 9 for k in racy], dtype=float)
        found = t < 10 ** 9
        return {"median": float(np.median(t[found])) if found.any() else None,
                "p90": float(np.percentile(t[found], 90)) if found.any() else None,
                "stopped": int(found.sum()), "racy": len(racy)}
    line = {
        "metric": "race queries/sec, VERDICT mode with learned tile order",
        "value": n / out["verdict_mlp"][2], "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": out["verdict_mlp"][2] * 1000, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "sparse witnesses among overlapping tiles: %d queries, "
                               "256 blocks x 256 threads per side, one conflicting "
                               "block pair in 2^16 for the racy half, seed 4004" % n,
                   "weights": wsrc},
        "time_to_verdict_ms": {k: v[2] * 1000 for k, v in out.items()},
        "queries_per_s": {k: n / v[2] for k, v in out.items()},
        "tiles_to_witness": {k[8:]: tile_stats(out[k][1]) for k in out if k != "exact"},
        "verdicts_agree": agree,
    }
    print(json.dumps(line), flush=True)


def kernel_rooflines(stats, traffic_files=None):
    """Per table-path kernel: algorithmic record bytes per launch over the
    mean launch duration, both from the timed steps (HIP events on the
    library's stream around every launch), against the HBM peak."""
    out = {}
    for name, lk, mk, bk, what in KERNELS:
        launches = sum(s[lk] for s in stats)
        ms = sum(s[mk] for s in stats)
        nbytes = sum(s[bk] for s in stats)
        if not launches or ms <= 0:
            continue
        avg_ms = ms / launches
        per_launch = nbytes / launches
        achieved = per_launch / (avg_ms / 1e3) / 1e9
        tfile = (traffic_files or {}).get(name)
        # priced against HBM: records are the kernel's only HBM traffic; what
        # holds it below that bound is stated in "limiter"
        traffic = measured_traffic(tfile) if tfile else None
        alg = measured_traffic(tfile, "algorithmic bytes per launch (same steps)") \
            if tfile else None
        limiter = LIMITER.get(name)
        if traffic and alg and limiter:
            limiter += "; counters: HBM traffic %.2fx the record bytes" % (traffic / alg)
        out[name] = {"bound": "hbm", "kernel": name, "achieved": achieved,
                     "limiter": limiter,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "bytes_per_launch": per_launch, "avg_launch_ms": avg_ms,
                     "launches_per_step": launches / len(stats),
                     "ms_per_step": ms / len(stats), "work": what}
    return out


def golden_agreement(wl, results, name):
    """Stored oracle results (tests/golden/, written by a script that calls
    only the oracle) against the GPU results, field by field."""
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    try:
        import make_goldens as G
        gold = G.load(name)
    except (OSError, ImportError):
        return None
    if G.digest(wl) != gold["digest"]:
        return "generator differs from the goldens' workload"
    agree = 0
    for i, w in zip(gold["indices"], gold["results"]):
        g = {f: results[i][f] for f in G.FIELDS}
        agree += g == w
    return "%d/%d stored oracle results identical to the GPU (%s)" % (
        agree, len(gold["indices"]), name)


def run_mixed(args):
    """The headline: the mixed workload in fixed batches of MIXED_STEP
    consecutive queries, one batch per step."""
    import numpy as np
    import torch
    import paper_2604_02106_amd as hg
    from workloads import configs
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    wl = configs.mixed(seed=5005, n_queries=int(100000 * args.scale))
    n = len(wl.pairs)
    nb = (n + MIXED_STEP - 1) // MIXED_STEP
    batches = [wl.compact(range(i * MIXED_STEP, min(n, (i + 1) * MIXED_STEP)))
               for i in range(nb)]
    log("workload: %d models, %d queries, %d batches (%.1f s to generate)"
        % (len(wl.models), n, nb, time.perf_counter() - t0))
    ctx = hg.Context(0)
    used = sorted(set([i % nb for i in range(args.warmup)] +
                      [i % nb for i in range(args.steps)]))
    plans = {}
    t0 = time.perf_counter()
    for i in used:
        plans[i] = hg.Plan(ctx, batches[i], max_device_bytes=args.wave_mib << 20)
        log("batch %d prepared" % i)
    prep_s = time.perf_counter() - t0
    for i in range(args.warmup):
        plans[i % nb].execute(raw=True)
        log("warmup %d (batch %d) done" % (i, i % nb))
    # Timed steps: the first phase runs eagerly with HIP events around every
    # partition, filter and join launch (the roofline figures come from
    # these steps); each batch's results stay in its plan's buffer.
    os.environ["HGRD_TIMING"] = "1"
    stats, step_s = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        plans[i % nb].execute(raw=True)
        step_s.append(time.perf_counter() - ts)
        stats.append(ctx.stats())
        log("step %d (batch %d) done in %.3f s" % (i, i % nb, step_s[-1]))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    del os.environ["HGRD_TIMING"]
    queries = sum(len(batches[i % nb].pairs) for i in range(args.steps))
    evals = sum(s["evals"] for s in stats)
    results = {}
    for i in used:
        out = plans[i].out
        results[i] = [hg.result_dict(out[k]) for k in range(len(batches[i].pairs))]
    covered = [i for i in range(nb) if i in results]
    flat = None
    if len(covered) == nb:
        flat = [r for i in range(nb) for r in results[i]]
    racy = sum(r["verdict"] for i in covered for r in results[i])
    line = {
        "metric": "race queries/sec and thread-access evals/sec (G/s) at 100% oracle agreement",
        "value": queries / dt,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1000 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "mixed batched: %d queries over %d kernel models, "
                               "per-query domain log-uniform 2^8..2^28 points, 1-64 "
                               "parameter tuples per model, 2-D/3-D launches, global "
                               "(a quarter 64-bit) and shared arrays, 10%% racy, seed "
                               "5005; %d batches of %d queries, one per step"
                               % (n, len(wl.models), nb, MIXED_STEP),
                   "queries_timed": queries, "evals_timed": evals, "racy": racy,
                   "scale": args.scale, "wave_mib": args.wave_mib or 3072},
        "evals_per_s_G": evals / dt / 1e9,
        "prepare_s": prep_s,
        "step_s": {"min": min(step_s), "max": max(step_s)},
        "kernel_ms_steps": {k: sum(s[k] for s in stats) / len(stats) for k in (
            "scatter_ms", "bucket_ms", "small_ms", "retry_ms", "fallback_ms",
            "witness_ms", "verdict_ms", "split_ms", "waves_ms", "device_ms",
            "total_ms")},
        "items_per_step": {k: sum(s[k] for s in stats) / len(stats) for k in (
            "small_items", "hbm_items", "retry_items", "split_items",
            "overflow_items", "fallback_records", "buckets", "records")},
        # exact shortcuts inside the timed steps: HBM (pair, tuple) units the
        # unit filter proved free of conflicts (nothing partitioned), and
        # shared-array units joined on block 0 only (block symmetry)
        "exact_shortcuts_per_step": {k: sum(s[k] for s in stats) / len(stats) for k in (
            "units_apart", "block_symmetric")},
    }
    kr = kernel_rooflines(stats, {"k_bucket_join<1024, 2048, true, false>": MIXED_TRAFFIC_FILE})
    if kr:
        dom = max(kr, key=lambda k: kr[k]["ms_per_step"])
        line["roofline"] = kr[dom]
        line["roofline_other_kernels"] = {k: v for k, v in kr.items() if k != dom}
    if flat is not None:
        line["golden_agreement"] = golden_agreement(wl, flat, "mixed_5005_sample.json.gz")
    if not args.no_extras:
        # the same batches replaying their captured graphs (the first
        # execute of a plan above ran eagerly, so this captures, then the
        # timed loop replays)
        k = min(args.steps, 4)
        for i in range(k):
            plans[i % nb].execute(raw=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(k):
            plans[i % nb].execute(raw=True)
        torch.cuda.synchronize()
        tg = time.perf_counter() - t0
        q = sum(len(batches[i % nb].pairs) for i in range(k))
        line["graph_replay"] = {"queries_per_s": q / tg,
                                "eager_queries_per_s": q / sum(step_s[:k]),
                                "batches": k}
        # VERDICT mode with the trained tile order on the first two batches
        # against EXACT on the same batches (from the timed steps)
        try:
            from paper_2604_02106_amd import tile_mlp
            w, _ = tile_mlp.load()
            k = min(2, len(step_s))
            vt, vres = 0.0, []
            for i in range(k):
                vp = hg.Plan(ctx, batches[i], mode=hg.MODE_VERDICT, order=hg.ORDER_MLP, mlp=w)
                vp.execute(raw=True)
                torch.cuda.synchronize()
                ts = time.perf_counter()
                r = vp.execute()
                vt += time.perf_counter() - ts
                vres.append(r)
                vp.close()
            q = sum(len(batches[i].pairs) for i in range(k))
            same = all(a["verdict"] == b["verdict"] and a["status"] == b["status"]
                       for i in range(k) for a, b in zip(vres[i], results[i]))
            line["verdict_mlp"] = {"queries_per_s": q / vt,
                                   "exact_queries_per_s": q / sum(step_s[:k]),
                                   "batches": k, "verdicts_equal_exact": same}
        except (OSError, RuntimeError, AssertionError) as e:
            line["verdict_mlp"] = "not run: %s" % e
        # the plain checker: one query per call, on a random sample
        rng = np.random.Generator(np.random.PCG64(17))
        pick = [int(x) for x in rng.choice(len(batches[0].pairs), 64, replace=False)]
        one = [batches[0].compact([p]) for p in pick]
        hg.rd_check_pairs(ctx, one[0])
        torch.cuda.synchronize()
        ts = time.perf_counter()
        same = True
        for p, w1 in zip(pick, one):
            same &= hg.rd_check_pairs(ctx, w1)[0] == results[0][p]
        line["plain_checker"] = {"queries_per_s": len(pick) / (time.perf_counter() - ts),
                                 "sample": "%d queries of batch 0, one rd_check_pairs "
                                           "call each" % len(pick),
                                 "results_equal_batched": bool(same)}
        # end to end: a fresh plan of batch 0 through the C ABI (lowering,
        # upload, execute, results), its Python marshalling timed apart
        ts = time.perf_counter()
        pk0 = hg.Packed(batches[0])
        line["python_marshal_s"] = time.perf_counter() - ts
        ts = time.perf_counter()
        e2e = hg.rd_check_pairs(ctx, batches[0], packed=pk0)
        line["end_to_end_queries_per_s"] = len(batches[0].pairs) / (time.perf_counter() - ts)
        line["end_to_end_equal"] = e2e == results[0]
        # end to end over the whole workload: one rd_check_pairs call on every
        # query (the library splits it into batches and lowers batch k + 1 on
        # a host thread while batch k runs on the GPU), against the execute
        # time of the timed steps, which cover each batch once
        if flat is not None and args.steps >= nb:
            pk_all = hg.Packed.concat([plans[i].packed for i in range(nb)])
            allp, base = [], 0
            for i in range(nb):
                allp += [(m + base, a, b, k) for (m, a, b, k) in batches[i].pairs]
                base += plans[i].packed.n_models
            cp = hg._pairs(types.SimpleNamespace(pairs=allp))
            out = (hg.rd_pair_result * len(allp))()
            opt, _ = hg._options(hg.MODE_EXACT, hg.ORDER_LEX, 0, args.wave_mib << 20, 0, None)
            ts = time.perf_counter()
            st = hg.lib().rd_check_pairs(ctx.h, pk_all.models, pk_all.n_models, cp, len(allp),
                                         pk_all.launch, pk_all.params, ctypes.byref(opt), out)
            te = time.perf_counter() - ts
            ex = sum(step_s[:nb])
            line["end_to_end_whole"] = {
                "queries_per_s": len(allp) / te, "s": te, "execute_s": ex,
                "ratio_to_execute": te / ex, "status": st,
                "equal": st == 0 and all(hg.result_dict(out[k]) == flat[k]
                                         for k in range(len(allp))),
                "note": "one call on all queries: lowering, upload, execute and results "
                        "(batches of 4096 pairs, the next lowered during the current "
                        "one's GPU work); execute_s = the timed steps"}
            log("end to end (whole workload): %.2f s, %.2fx the timed steps"
                % (te, te / ex))
        # the same two batches with the exact shortcuts off (unit filter and
        # block symmetry): every unit enumerated
        k = min(2, len(step_s))
        os.environ["HGRD_NO_SYMMETRY"] = "1"
        os.environ["HGRD_NO_UNIT_FILTER"] = "1"
        try:
            tp, same = 0.0, True
            for i in range(k):
                pp = hg.Plan(ctx, batches[i], max_device_bytes=args.wave_mib << 20)
                torch.cuda.synchronize()
                ts = time.perf_counter()
                r = pp.execute()
                tp += time.perf_counter() - ts
                same &= r == results[i]
                pp.close()
        finally:
            del os.environ["HGRD_NO_SYMMETRY"]
            del os.environ["HGRD_NO_UNIT_FILTER"]
        q = sum(len(batches[i].pairs) for i in range(k))
        line["without_exact_shortcuts"] = {"queries_per_s": q / tp,
                                           "with_queries_per_s": q / sum(step_s[:k]),
                                           "batches": k, "results_equal": bool(same)}
    if not args.no_cpu_baseline and 0 in results:
        line["cpu_baseline"] = cpu_baseline(batches[0], results[0])
        line["cpu_baseline"]["sample"] += " (batch 0 of the mixed workload)"
    print(json.dumps(line), flush=True)


def run_synced(args):
    """Synchronisation-aware queries: the synced workload (mixed queries of
    2^8..2^22 points per access with lock and producer/consumer patterns
    around the accesses) in fixed batches, against the same batches with the
    acquires and releases removed (the plain path)."""
    import copy
    import torch
    import paper_2604_02106_amd as hg
    from workloads import configs
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    step_q = 1000
    wl = configs.synced(seed=6006, n_queries=int(4000 * args.scale))
    plain = copy.deepcopy(wl)
    for m in plain.models:
        for a in m.accesses:
            a.acq = a.rel = None
    n = len(wl.pairs)
    nb = (n + step_q - 1) // step_q
    ctx = hg.Context(0)
    out = {}
    for name, w in (("synced", wl), ("synced_fallback", wl), ("plain", plain)):
        batches = [w.compact(range(i * step_q, min(n, (i + 1) * step_q))) for i in range(nb)]
        # synced_fallback: every synchronised unit through the HBM
        # aggregation path instead of the LDS joins
        if name == "synced_fallback":
            os.environ["HGRD_SYNC_FALLBACK"] = "1"
        try:
            plans = [hg.Plan(ctx, b) for b in batches]
        finally:
            os.environ.pop("HGRD_SYNC_FALLBACK", None)
        for i in range(args.warmup):
            plans[i % nb].execute(raw=True)
        torch.cuda.synchronize()
        stats, res = [], []
        t0 = time.perf_counter()
        for i in range(args.steps):
            res.append(plans[i % nb].execute())
            stats.append(ctx.stats())
            log("%s step %d done" % (name, i))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        q = sum(len(batches[i % nb].pairs) for i in range(args.steps))
        out[name] = {"queries_per_s": q / dt, "ms_per_step": dt * 1000 / args.steps,
                     "evals_per_s_G": sum(s["evals"] for s in stats) / dt / 1e9,
                     "fallback_ms_per_step": sum(s["fallback_ms"] for s in stats) / len(stats),
                     "sync_records_per_step": sum(s["sync_records"] for s in stats) / len(stats),
                     "hbm_items_per_step": sum(s["hbm_items"] for s in stats) / len(stats),
                     "racy": sum(r["verdict"] for rr in res for r in rr)}
        if name == "synced":
            sres, sb = res[0], batches[0]
        for p in plans:
            p.close()
    line = {"metric": "synchronisation-aware race queries/sec", "value":
            out["synced"]["queries_per_s"], "unit": "queries/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "dtype": "int64",
            "data": "synthetic",
            "config": {"workload": "synced: %d mixed queries of 2^8..2^22 points per "
                                   "access with lock / producer-consumer patterns, "
                                   "seed 6006; batches of %d" % (n, step_q)},
            "synced": out["synced"], "synced_all_fallback": out["synced_fallback"],
            "plain_same_queries": out["plain"]}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(sb, sres)
        line["cpu_baseline"]["sample"] += " (batch 0 of the synced workload)"
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 20 for the mixed workload, "
                         "one pass over it; 5 otherwise)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps first (default 1 mixed, 2 otherwise)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the figures reported beside the headline "
                         "(graph replay, VERDICT mode, the plain checker, the "
                         "end-to-end calls, the exact shortcuts switched off; "
                         "they run after the timed steps)")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--config", default="mixed",
                    choices=("batched", "stress", "mixed", "learned", "synced"),
                    help="workload: mixed batched queries (the headline), "
                         "batched uneven queries, race-free stress (128 "
                         "pairs, 2^30 points per access), the learned tile "
                         "order on sparse witnesses, or queries under "
                         "acquire/release synchronisation")
    ap.add_argument("--wave-mib", type=int, default=0,
                    help="partition wave size in MiB (0: the library default)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 8 GiB three times "
                         "(the reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only; --gpus %d is not supported "
              "(queries shard across GPUs without exchange, see the design "
              "notes)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.steps is None:
        args.steps = 20 if args.config == "mixed" else 5
    if args.warmup is None:
        args.warmup = 1 if args.config == "mixed" else 2
    if args.config == "learned":
        return run_learned(args)
    if args.config == "synced":
        return run_synced(args)
    if args.config == "mixed" and not args.calibrate_copy:
        return run_mixed(args)
    import torch
    if args.calibrate_copy:
        # 8 GiB: far beyond the 256 MiB last-level cache, so the counters see
        # HBM traffic of the copy itself
        src = torch.empty(1 << 31, dtype=torch.int32, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied 3 x %d bytes" % (src.numel() * 4))
        return
    import paper_2604_02106_amd as hg
    from workloads import configs
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    if args.config == "stress":
        wl = configs.stress()
        desc = ("race-free stress: 128 access pairs, 2^30 points per access "
                "(grid 65536 x block 256 x 64 iterations), int64 addresses, "
                "strided and blocked near misses, seed 3003")
    else:
        wl = configs.batched(seed=2002, scale=args.scale)
        desc = ("batched uneven queries: 256 kernel models x 16 access pairs, "
                "seed 2002, grids up to 1024 blocks x 256 threads, loops up to "
                "64 iterations, 1-16 parameter tuples")
    log("workload: %d models, %d pairs" % (len(wl.models), len(wl.pairs)))
    ctx = hg.Context(0)
    t0 = time.perf_counter()
    e2e = hg.rd_check_pairs(ctx, wl, max_device_bytes=args.wave_mib << 20)
    e2e_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    plan = hg.Plan(ctx, wl, max_device_bytes=args.wave_mib << 20)
    prep_s = time.perf_counter() - t0
    log("prepared in %.3f s (end-to-end call %.3f s)" % (prep_s, e2e_s))
    for i in range(max(1, args.warmup)):
        res = plan.execute()
        log("warmup %d done" % i)
    assert res == e2e
    # Timed steps run the first phase eagerly with HIP events around every
    # partition kernel (the roofline figures come from these same steps).
    os.environ["HGRD_TIMING"] = "1"
    plan.execute(raw=True)  # untimed: first eager pass
    torch.cuda.synchronize()
    log("eager pass done")
    stats = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        plan.execute(raw=True)
        stats.append(ctx.stats())
        log("step %d done" % i)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    del os.environ["HGRD_TIMING"]
    res = [hg.result_dict(plan.out[k]) for k in range(len(wl.pairs))]
    assert res == e2e
    tstat = stats[-1]
    dt_pre = dt_graph = pre_units = None
    if not args.no_extras:
        # with the exact interval pre-filter (beside the headline)
        pplan = hg.Plan(ctx, wl, max_device_bytes=args.wave_mib << 20, prefilter=1)
        pres = pplan.execute()
        assert pres == res
        torch.cuda.synchronize()
        log("pre-filtered plan checked")
        t0 = time.perf_counter()
        for i in range(args.steps):
            pplan.execute(raw=True)
            log("pre-filtered step %d done" % i)
        torch.cuda.synchronize()
        dt_pre = time.perf_counter() - t0
        pre_units = ctx.stats()["prefiltered"]
        pplan.close()
        # the same plan replaying its captured graph (beside the headline)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            plan.execute(raw=True)
            log("graph step %d done" % i)
        torch.cuda.synchronize()
        dt_graph = time.perf_counter() - t0
    log("timed %d steps in %.3f s" % (args.steps, dt))
    n = len(wl.pairs)
    evals = stats[-1]["evals"]
    racy = sum(r["verdict"] for r in res)
    line = {
        "metric": "race queries/sec and thread-access evals/sec (G/s) at 100% oracle agreement",
        "value": n * args.steps / dt,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1000 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": desc,
                   "queries": n, "evals_per_step": evals, "racy": racy,
                   "scale": args.scale, "wave_mib": args.wave_mib or 3072},
        "evals_per_s_G": evals * args.steps / dt / 1e9,
        "end_to_end_queries_per_s": n / e2e_s,
        "graph_replay_queries_per_s": n * args.steps / dt_graph if dt_graph else None,
        "prefilter_queries_per_s": n * args.steps / dt_pre if dt_pre else None,
        "prefilter_units": pre_units,
        "prepare_s": prep_s,
        "kernel_ms": {k: sum(s[k] for s in stats) / len(stats)
                      for k in ("device_ms", "total_ms")},
        "kernel_ms_steps": {k: sum(s[k] for s in stats) / len(stats) for k in (
            "scatter_ms", "bucket_ms", "small_ms", "retry_ms", "fallback_ms",
            "witness_ms", "verdict_ms", "split_ms", "waves_ms")},
        "items": {k: stats[-1][k] for k in ("small_items", "hbm_items",
                                            "retry_items", "split_items",
                                            "overflow_items", "fallback_records",
                                            "buckets", "records", "scatter_bytes")},
    }
    kr = kernel_rooflines(stats)
    if kr:
        dom = max(kr, key=lambda k: kr[k]["ms_per_step"])
        line["roofline"] = kr[dom]
        line["roofline_other_kernels"] = {k: v for k, v in kr.items() if k != dom}
    if args.config == "batched" and args.scale == 1.0:
        line["golden_agreement"] = golden_agreement(wl, res, "batched_2002.json.gz")
    if not args.no_cpu_baseline and args.config == "batched":
        line["cpu_baseline"] = cpu_baseline(wl, res)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
