#!/usr/bin/env python3
"""Benchmark: batched worst-case response-time analyses per second on one GPU.

Workload (the paper's Sec. IV-F analysis over synthetic chain sets): 1,000,000
chain sets of 4-64 chains x 2-12 callbacks, 4 executors (pairs share a core),
one accelerator, periods log-uniform over 10-1000 ms, segment share per set
U(10, 60) % of the callbacks with 5-80 % of the callback WCET; drawn at total
utilisation 1 and analysed at the 18 utilisation levels 0.10, 0.15, ..., 0.95.
One step = the whole sweep: 18 launches of the analysis (one per level, every
chain's end-to-end bound, cap = deadline), captured once as a HIP graph and
replayed.  Inputs are resident in HBM before the timed region.

Printed JSON line: value = analyses per second (18 M per step); roofline of
the analysis kernel (ALU-bound: interference terms per second against the
fp64 issue rate); cpu_baseline = the CPU oracle, single-threaded, on a sample
of the same sweep, whose outputs are also compared bit-exactly with the GPU's.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Peak interference-term rate: a term is one fp64 add, mul, floor and fma on a
# lane; 256 CUs x 64 lanes x 2.4 GHz issue 39.3 T fp64 lane-ops/s (the
# published 78.6 TFLOP/s fp64 vector rate counts an fma as 2).
FP64_LANE_OPS = 256 * 64 * 2.4e9
OPS_PER_TERM = 4
PEAK_TERMS = FP64_LANE_OPS / OPS_PER_TERM


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


# HBM bytes per full-mode launch of the analysis kernel on the default
# workload (mean over the launches of a sweep, one per size class and level),
# from two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE) scaled by the
# counters' reading for the 1 GiB calibration copy.  Valid only for the kernel
# source with this SHA-256 at the same waves per CU; null otherwise.
TRAFFIC = {"sha256": "94161b1f2453528e5ca1baf49a5ac98bcecad7047e3371d4b8d5daf3bb6f1e9d",
           "bytes_per_launch": 16.11e9, "sets": 1_000_000, "waves_per_cu": 20}
KERNEL_SRC = os.path.join(ROOT, "paper_2404_06452_amd", "csrc", "paam_kernels.hip")

COPY_BYTES = 1 << 30


def measured_traffic(n_sets, waves_per_cu):
    import hashlib
    with open(KERNEL_SRC, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if sha != TRAFFIC["sha256"] or n_sets != TRAFFIC["sets"]:
        return None
    return TRAFFIC["bytes_per_launch"]


def copy_calibration(torch, stream):
    """A plain device-to-device copy of COPY_BYTES: its measured rate is the
    attainable HBM bandwidth, and in a counter profile of this script its
    FETCH_SIZE / WRITE_SIZE per dispatch (COPY_BYTES each way) give the
    counters' scale."""
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        dst.copy_(src)
        torch.cuda.synchronize()
        a.record(stream)
        for _ in range(5):
            dst.copy_(src)
        b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / 5
    del src, dst
    return 2 * COPY_BYTES / (ms * 1e-3) / 1e9


def search_section(args, torch, log):
    """Priority-order search over 256 candidate orders per set, plain and
    guided by the ranking network (trained here by the library's kernels),
    at the workload's utilisation and at a scale near the feasibility
    boundary.  Times are HIP events on the launch stream."""
    from paper_2404_06452_amd import _paam, chaingen, surrogate

    n_cand, top_k, seed = 256, 16, 2404
    stream = torch.cuda.Stream()

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) * 1e-3

    t0 = time.perf_counter()
    cs = chaingen.generate("search", args.search_sets)
    dev = _paam.Chainset(cs, device="cuda:0")
    n = cs.n_sets
    out = _paam.SearchOut(dev)
    scores = torch.empty(n * n_cand, dtype=torch.float32, device="cuda:0")

    def run_search(util, guided, fallback=True):
        o = _paam.search_opts(n_cand, seed, guided=guided, top_k=top_k, fallback=fallback,
                              scores=scores if guided else None, util_permille=util)
        ws = _paam.workspace(_paam.paam_search_bytes(dev, o))
        dt = timed(lambda: _paam.paam_priority_search(dev, o, out, ws, stream))
        return dt, out.found.cpu().numpy(), out.n_exact.cpu().numpy()

    def run_score(net, util):
        o = _paam.search_opts(n_cand, seed, util_permille=util)
        ws = _paam.workspace(_paam.paam_score_bytes(dev, o))
        return timed(lambda: _paam.paam_score_candidates(dev, o, net.params, net.packed, scores,
                                                         ws, stream))

    # the ranking network, trained on the sweep generator's sets
    t1 = time.perf_counter()
    tcs = chaingen.generate("sweep", args.train_sets)
    tdev = _paam.Chainset(tcs, device="cuda:0")
    net = _paam.Network(chaingen.mlp_init(seed), device="cuda:0")
    tr = surrogate.Trainer(tdev, net, seed, batch=4096)
    pairs = torch.from_numpy(surrogate.recipe_pairs(tcs.n_sets, args.train_samples, seed)).cuda()
    t_targets = timed(lambda: setattr(tr, "_tg", tr.targets(pairs)))
    target = tr._tg.ratio[:args.train_samples]
    t2 = time.perf_counter()
    losses = tr.fit(pairs, target, epochs=args.train_epochs, lr=2e-3, lr_final=1e-4,
                    order_seed=seed, log=log)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t2
    hcs = chaingen.generate("sweep", 20000, set_begin=args.train_sets)
    hdev = _paam.Chainset(hcs, device="cuda:0")
    htr = surrogate.Trainer(hdev, net, seed, batch=4096)
    hp = torch.from_numpy(surrogate.recipe_pairs(hcs.n_sets, 200000, seed + 1)).cuda()
    hy = htr.targets(hp).ratio[:200000].cpu().numpy()
    hpred = htr.predict(hp).cpu().numpy()
    sur = {
        "train_sets": tcs.n_sets, "train_samples": args.train_samples,
        "epochs": args.train_epochs, "target_s": t_targets, "train_s": t_fit,
        "epoch_losses": losses, "holdout_samples": len(hy),
        "holdout_mae": float(np.mean(np.abs(hpred - hy))),
        "holdout_spearman": surrogate.spearman(hpred, hy),
        "recipe": "sweep-generator sets at utilisation 0.2-10 % (log-uniform) of their U=1 "
                  "draw, k uniform in 0..255, target min(max R/D, 2)",
    }
    log("surrogate: trained in %.1f s (targets %.2f s), holdout MAE %.3f, Spearman %.3f" % (
        time.perf_counter() - t1, t_targets, sur["holdout_mae"], sur["holdout_spearman"]))
    untrained = _paam.Network(chaingen.mlp_init(seed + 7), device="cuda:0")

    res = {"workload": "%d chain sets of 16 chains x 2-8 callbacks, 4 executors, 1 accelerator, "
                       "U ~ U(0.5, 0.9); %d candidate orders per set (uploaded rate-monotonic "
                       "order + seeded swap walk); guided: top %d by predicted max R/D" % (
                           n, n_cand, top_k),
           "surrogate": sur}
    for name, util in (("workload_utilisation", 1000), ("near_boundary_5pct", 50)):
        t_plain, f_plain, e_plain = run_search(util, False)
        found_plain = f_plain >= 0
        t_score = run_score(net, util)
        t_fb, f_fb, e_fb = run_search(util, True, True)
        t_top, f_top, e_top = run_search(util, True, False)
        rel = (lambda f: float((f >= 0).sum() / max(found_plain.sum(), 1)))
        entry = {
            "util_scale": util / 1000,
            "plain": {"sets_per_s": n / t_plain, "ms": t_plain * 1e3,
                      "found_frac": float(found_plain.mean()),
                      "mean_exact_evals": float(e_plain.mean())},
            "guided_with_fallback": {"sets_per_s": n / (t_score + t_fb), "score_ms": t_score * 1e3,
                                     "search_ms": t_fb * 1e3, "found_frac": float((f_fb >= 0).mean()),
                                     "found_vs_plain": rel(f_fb),
                                     "mean_exact_evals": float(e_fb.mean())},
            "guided_top_k_only": {"sets_per_s": n / (t_score + t_top), "score_ms": t_score * 1e3,
                                  "search_ms": t_top * 1e3, "found_frac": float((f_top >= 0).mean()),
                                  "found_vs_plain": rel(f_top),
                                  "mean_exact_evals": float(e_top.mean())},
        }
        if util != 1000:
            run_score(untrained, util)
            _, f_un, e_un = run_search(util, True, False)
            entry["untrained_network_top_k_only"] = {"found_frac": float((f_un >= 0).mean()),
                                                     "found_vs_plain": rel(f_un),
                                                     "mean_exact_evals": float(e_un.mean())}
            # the same budget without a ranking: the first top_k candidates of
            # the walk, which starts at the uploaded rate-monotonic order
            o_ix = _paam.search_opts(top_k, seed, util_permille=util)
            ws_ix = _paam.workspace(_paam.paam_search_bytes(dev, o_ix))
            t_ix = timed(lambda: _paam.paam_priority_search(dev, o_ix, out, ws_ix, stream))
            f_ix, e_ix = out.found.cpu().numpy(), out.n_exact.cpu().numpy()
            entry["first_k_in_index_order"] = {"sets_per_s": n / t_ix,
                                               "found_frac": float((f_ix >= 0).mean()),
                                               "found_vs_plain": rel(f_ix),
                                               "mean_exact_evals": float(e_ix.mean())}
        res[name] = entry
        log("search %s: plain %.3g sets/s found %.3f evals %.1f | guided+fb %.3g sets/s found %.3f "
            "evals %.1f | top-%d %.3g sets/s found %.3f" % (
                name, entry["plain"]["sets_per_s"], entry["plain"]["found_frac"],
                entry["plain"]["mean_exact_evals"], entry["guided_with_fallback"]["sets_per_s"],
                entry["guided_with_fallback"]["found_frac"],
                entry["guided_with_fallback"]["mean_exact_evals"], top_k,
                entry["guided_top_k_only"]["sets_per_s"], entry["guided_top_k_only"]["found_frac"]))
    res["setup_s"] = time.perf_counter() - t0
    return res, net


def large_section(args, torch, log, net):
    """Sets of 256 chains x 2-32 callbacks, 8 executors, one accelerator, U ~
    U(0.3, 0.95), half the callbacks with a segment: the exact analysis of the
    uploaded rate-monotonic order, network scores of 1,024 candidate orders
    per set, and the exact confirmation of the top 32, captured together in one
    HIP graph; plain search over the same 1,024 candidates on a subset for
    comparison.  Times are HIP events on the launch stream."""
    from paper_2404_06452_amd import _paam, chaingen

    n_cand, top_k, seed = 1024, 32, 2404
    stream = torch.cuda.Stream()

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) * 1e-3

    t0 = time.perf_counter()
    cs = chaingen.generate("large", args.large_sets)
    dev = _paam.Chainset(cs, device="cuda:0")
    n = cs.n_sets
    m = min(args.large_plain_sets, n)
    sub = _paam.Chainset(cs.subset(range(m)), device="cuda:0")
    log("large sets: %d sets (%d chains, %d callbacks, %d segments) ready in %.1f s" % (
        n, cs.n_chains, cs.n_callbacks, cs.n_segments, time.perf_counter() - t0))
    res = {"workload": "%d chain sets of 256 chains x 2-32 callbacks, 8 executors, 1 accelerator, "
                       "U ~ U(0.3, 0.95), 50 %% of callbacks with a segment; %d candidate orders "
                       "per set, top %d confirmed exactly; plain search on the first %d sets" % (
                           n, n_cand, top_k, m),
           "sets": n, "chains": cs.n_chains, "callbacks": cs.n_callbacks,
           "segments": cs.n_segments}
    wout = _paam.WcrtOut(dev, False)
    sout = _paam.SearchOut(dev)
    pout = _paam.SearchOut(sub)
    scores = torch.empty(n * n_cand, dtype=torch.float32, device="cuda:0")
    levels = [("workload_utilisation", 1000)]
    if args.large_util:
        levels.append(("scaled_%g_permille" % args.large_util, args.large_util))
    for name, util in levels:
        wo = _paam.wcrt_opts(full=False, util_permille=util)
        so = _paam.search_opts(n_cand, seed, util_permille=util)
        go = _paam.search_opts(n_cand, seed, guided=True, top_k=top_k, fallback=False,
                               scores=scores, util_permille=util)
        po = _paam.search_opts(n_cand, seed, util_permille=util)
        wws = _paam.workspace(_paam.paam_wcrt_bytes(dev, wo))
        sws = _paam.workspace(_paam.paam_score_bytes(dev, so))
        gws = _paam.workspace(_paam.paam_search_bytes(dev, go))
        pws = _paam.workspace(_paam.paam_search_bytes(sub, po))

        def analyse(s):
            _paam.paam_wcrt_batch(dev, wo, wout, wws, s)

        def score(s):
            _paam.paam_score_candidates(dev, so, net.params, net.packed, scores, sws, s)

        def confirm(s):
            _paam.paam_priority_search(dev, go, sout, gws, s)

        t_an = timed(lambda: analyse(stream))
        t_sc = timed(lambda: score(stream))
        t_gd = timed(lambda: confirm(stream))
        ref = (wout.set_sched.clone(), sout.found.clone(), sout.n_exact.clone())
        # the three steps as one captured graph, replayed; every replay must
        # reproduce the eager outputs
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            s = torch.cuda.current_stream()
            analyse(s)
            score(s)
            confirm(s)
        torch.cuda.synchronize()
        t_graph = []
        for _ in range(2):
            t_graph.append(timed(graph.replay))
            assert torch.equal(ref[0], wout.set_sched) and torch.equal(ref[1], sout.found) and \
                torch.equal(ref[2], sout.n_exact), "graph replay differs"
        del graph
        t_pl = timed(lambda: _paam.paam_priority_search(sub, po, pout, pws, stream))
        rm = ref[0].cpu().numpy()
        found_g = ref[1].cpu().numpy()
        evals_g = ref[2].cpu().numpy()
        found_p = pout.found.cpu().numpy()
        evals_p = pout.n_exact.cpu().numpy()
        fp = int((found_p >= 0).sum())
        entry = {
            "util_scale": util / 1000,
            "rm_analysis": {"sets_per_s": n / t_an, "ms": t_an * 1e3,
                            "schedulable_frac": float((rm == 1).mean())},
            "scoring": {"candidates_per_s": n * n_cand / t_sc, "ms": t_sc * 1e3},
            "guided_top_k": {"sets_per_s": n / (t_sc + t_gd), "search_ms": t_gd * 1e3,
                             "found_frac": float((found_g >= 0).mean()),
                             "mean_exact_evals": float(evals_g.mean()),
                             "found_frac_first_subset": float((found_g[:m] >= 0).mean()),
                             "found_vs_plain_on_subset": (float((found_g[:m] >= 0).sum() / fp)
                                                          if fp else None)},
            "graph": {"steps": "RM analysis + scoring + top-%d confirmation" % top_k,
                      "ms": float(min(t_graph)) * 1e3, "sets_per_s": n / min(t_graph)},
            "plain_subset": {"sets": m, "sets_per_s": m / t_pl, "ms": t_pl * 1e3,
                             "found_frac": float((found_p >= 0).mean()),
                             "mean_exact_evals": float(evals_p.mean())},
        }
        res[name] = entry
        log("large %s: RM %.3g sets/s (sched %.3f) | score %.3g cand/s | guided top-%d %.3g sets/s "
            "found %.3f evals %.1f | graph %.1f ms | plain (%d sets) %.3g sets/s found %.3f "
            "evals %.1f" % (
                name, entry["rm_analysis"]["sets_per_s"], entry["rm_analysis"]["schedulable_frac"],
                entry["scoring"]["candidates_per_s"], top_k, entry["guided_top_k"]["sets_per_s"],
                entry["guided_top_k"]["found_frac"], entry["guided_top_k"]["mean_exact_evals"],
                entry["graph"]["ms"], m, entry["plain_subset"]["sets_per_s"],
                entry["plain_subset"]["found_frac"], entry["plain_subset"]["mean_exact_evals"]))
        del wws, sws, gws, pws
    res["setup_s"] = time.perf_counter() - t0
    return res


def allcore_parity(args, cs, levels, outs, oracle, log):
    """The oracle on every host core over the first --allcore-sets sets at all
    levels (one single-threaded analysis per set, sets spread over a thread
    pool), compared bit-exactly with the GPU's outputs of the sweep."""
    n = min(args.allcore_sets, cs.n_sets)
    if n <= 0:
        return None
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    nc = int(cs.set_chain_off[n])
    mism, t0 = 0, time.perf_counter()
    for li, u in enumerate(levels):
        r = oracle.wcrt(cs, full=True, util_permille=u, sets=(0, n), threads=threads)
        mism += int(np.sum(outs[li].set_sched[:n].cpu().numpy() != r["sched"][:n]))
        mism += int(np.sum(outs[li].chain_R[:nc].cpu().numpy() != r["chain_R"][:nc]))
    wall = time.perf_counter() - t0
    log("oracle on %d threads: %d analyses in %.1f s; mismatches %d" % (
        threads, n * len(levels), wall, mism))
    return {"sets_per_level": n, "levels": len(levels), "analyses": n * len(levels),
            "threads": threads, "nproc": os.cpu_count(), "wall_s": wall,
            "analyses_per_s": n * len(levels) / wall, "mismatches": mism}


def other_cpu_legs(args, oracle, log):
    """The single-threaded oracle on the other workloads' fixed samples: the
    small sets (all 1,000, full mode), plain search over 256 candidate orders
    on 1,000 search sets, and the uploaded order of 100 large sets."""
    from paper_2404_06452_amd import chaingen
    res = {}
    cs = chaingen.generate("small", 1000)
    t0 = time.perf_counter()
    oracle.wcrt(cs, full=True)
    dt = time.perf_counter() - t0
    res["small_1000_sets"] = {"analyses_per_s": 1000 / dt, "s": dt}
    cs = chaingen.generate("search", 1000)
    t0 = time.perf_counter()
    r = oracle.search(cs, 256, 2404)
    dt = time.perf_counter() - t0
    res["search_1000_sets_x256"] = {"sets_per_s": 1000 / dt, "s": dt,
                                    "analyses": int(r["n_eval"].sum())}
    if args.large_sets > 0:
        cs = chaingen.generate("large", 100)
        t0 = time.perf_counter()
        oracle.wcrt(cs, full=False)
        dt = time.perf_counter() - t0
        res["large_100_sets"] = {"analyses_per_s": 100 / dt, "s": dt}
    log("oracle, other workloads: %s" % ", ".join("%s %.1f s" % (k, v["s"]) for k, v in res.items()))
    return res


def manifest(args, torch, _paam):
    """What produced the line: arguments, seeds, host and device."""
    from paper_2404_06452_amd import chaingen
    p = torch.cuda.get_device_properties(0)
    return {
        "args": vars(args),
        "seeds": {k: v.seed for k, v in chaingen.PRESETS.items()},
        "nproc": os.cpu_count(),
        "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
        "gpu": {"name": p.name, "arch": getattr(p, "gcnArchName", None),
                "compute_units": p.multi_processor_count, "memory_bytes": p.total_memory},
        "torch": torch.__version__, "hip": getattr(torch.version, "hip", None),
        "libpaam": _paam.lib().paam_version().decode(),
    }


def ablation_section(torch, dev, levels, outs, ws, stream, log):
    """Lemma 2 alone, Lemma 3 alone and their minimum (Sec. IV-F: neither
    bound dominates the other).  Per utilisation level: schedulable fraction
    under each, and the share of chains whose end-to-end bound each single
    bound makes larger than the minimum (PAAM_INF counts as larger than any
    finite bound)."""
    from paper_2404_06452_amd import _paam
    res = {}
    n_chains = int(dev.n_chains)
    o_l2 = _paam.WcrtOut(dev, True)
    o_l3 = _paam.WcrtOut(dev, True)
    for li, u in enumerate(levels):
        for out, bound in ((o_l2, _paam.PAAM_BOUND_L2), (o_l3, _paam.PAAM_BOUND_L3)):
            o = _paam.wcrt_opts(full=True, util_permille=u, bound=bound)
            with torch.cuda.stream(stream):
                _paam.paam_wcrt_batch(dev, o, out, ws, stream)
        torch.cuda.synchronize()
        rm = outs[li].chain_R[:n_chains]
        r2 = o_l2.chain_R[:n_chains]
        r3 = o_l3.chain_R[:n_chains]
        assert bool((rm <= r2).all()) and bool((rm <= r3).all()), "min bound above a single bound"
        res[str(u / 1000)] = {
            "schedulable_frac": {"min": float((outs[li].set_sched == 1).float().mean()),
                                 "lemma2_only": float((o_l2.set_sched == 1).float().mean()),
                                 "lemma3_only": float((o_l3.set_sched == 1).float().mean())},
            "chains_lemma2_only_larger": float((r2 > rm).float().mean()),
            "chains_lemma3_only_larger": float((r3 > rm).float().mean()),
            "chains_lemma2_below_lemma3": float((r2 < r3).float().mean()),
            "chains_lemma3_below_lemma2": float((r3 < r2).float().mean()),
        }
    log("ablation: level 0.10 L2-only larger %.3f, L3-only larger %.3f of chains" % (
        res[str(levels[0] / 1000)]["chains_lemma2_only_larger"],
        res[str(levels[0] / 1000)]["chains_lemma3_only_larger"]))
    del o_l2, o_l3
    return {"levels": res,
            "note": "every chain's bound of the sweep under Lemma 2 alone and Lemma 3 alone, "
                    "compared with their minimum (the analysis above); a single bound is never "
                    "below the minimum (asserted)"}


def study_section(args, torch, log, net):
    """The analytical study of the paper's Sec. V: schedulability against the
    number of chains (4 callbacks per chain, accelerator : CPU utilisation 1:1
    per chain) and against that ratio (1:9 ... 7:3 at 8 chains), 1,000 sets
    per point, on the batched analysis.  On the 8-chain 1:1 point, plain and
    guided priority-order search.  Bit-exact parity of every point against the
    CPU oracle is a GPU test (tests/test_gpu_study.py)."""
    from paper_2404_06452_amd import _paam, chaingen

    stream = torch.cuda.Stream()

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) * 1e-3

    n = args.study_sets
    t0 = time.perf_counter()

    def point(n_chains, acc, cpu):
        cs = chaingen.generate(chaingen.study_params(n_chains, acc, cpu), n)
        dev = _paam.Chainset(cs, device="cuda:0")
        o = _paam.wcrt_opts(full=False)
        out = _paam.WcrtOut(dev, False)
        ws = _paam.workspace(_paam.paam_wcrt_bytes(dev, o))
        dt = timed(lambda: _paam.paam_wcrt_batch(dev, o, out, ws, stream))
        frac = float((out.set_sched == 1).float().mean())
        return dev, frac, dt

    by_chains, t_an = {}, 0.0
    for c in chaingen.STUDY_CHAINS:
        dev, frac, dt = point(c, 1, 1)
        by_chains[str(c)] = frac
        t_an += dt
        dev.free()
    by_ratio = {}
    for acc, cpu in chaingen.STUDY_RATIOS:
        dev, frac, dt = point(chaingen.STUDY_RATIO_CHAINS, acc, cpu)
        by_ratio["%d:%d" % (acc, cpu)] = frac
        t_an += dt
        dev.free()
    vc, vr = list(by_chains.values()), list(by_ratio.values())
    res = {
        "workload": "%d sets per point; chains of 4 callbacks, each with one accelerator "
                    "segment; one accelerator; each chain on its own single-threaded executor "
                    "and core; chain utilisations UUniFast at %.2f per chain; periods "
                    "log-uniform 10-1000 ms; rate-monotonic priorities" % (
                        n, chaingen.STUDY_CHAIN_UTIL),
        "schedulable_frac_by_chains_ratio_1_1": by_chains,
        "schedulable_frac_by_ratio_%d_chains" % chaingen.STUDY_RATIO_CHAINS: by_ratio,
        "trend_chains_non_increasing": all(b <= a + 0.02 for a, b in zip(vc, vc[1:])),
        "trend_ratio_non_increasing": all(b <= a + 0.02 for a, b in zip(vr, vr[1:])),
        "analysis_ms_total": t_an * 1e3,
        "parity": "tests/test_gpu_study.py compares every set of every point with the oracle",
    }
    log("study: by chains %s | by ratio %s" % (
        " ".join("%.2f" % v for v in vc), " ".join("%.2f" % v for v in vr)))
    if net is not None:
        # priority-order search on sets that can be admitted: the 8-chain,
        # 1:1 point, 256 candidate orders per set
        n_cand, top_k, seed = 256, 16, 2404
        cs = chaingen.generate(chaingen.study_params(chaingen.STUDY_RATIO_CHAINS, 1, 1), n)
        dev = _paam.Chainset(cs, device="cuda:0")
        out = _paam.SearchOut(dev)
        scores = torch.empty(cs.n_sets * n_cand, dtype=torch.float32, device="cuda:0")

        def search(k, guided, fallback=True):
            o = _paam.search_opts(k, seed, guided=guided, top_k=top_k, fallback=fallback,
                                  scores=scores if guided else None)
            ws = _paam.workspace(_paam.paam_search_bytes(dev, o))
            dt = timed(lambda: _paam.paam_priority_search(dev, o, out, ws, stream))
            return dt, out.found.cpu().numpy(), out.n_exact.cpu().numpy()

        so = _paam.search_opts(n_cand, seed)
        sws = _paam.workspace(_paam.paam_score_bytes(dev, so))
        t_sc = timed(lambda: _paam.paam_score_candidates(dev, so, net.params, net.packed, scores,
                                                         sws, stream))
        t_p, f_p, e_p = search(n_cand, False)
        t_g, f_g, e_g = search(n_cand, True, False)
        t_i, f_i, e_i = search(top_k, False)
        fp = int((f_p >= 0).sum())
        res["search_8_chains"] = {
            "candidates": n_cand, "top_k": top_k,
            "rm_schedulable_frac": float((f_p == 0).mean()),
            "plain": {"found_frac": float((f_p >= 0).mean()),
                      "mean_exact_evals": float(e_p.mean()), "ms": t_p * 1e3},
            "guided_top_k_only": {"found_frac": float((f_g >= 0).mean()),
                                  "found_vs_plain": float((f_g >= 0).sum() / fp) if fp else None,
                                  "mean_exact_evals": float(e_g.mean()),
                                  "ms": (t_sc + t_g) * 1e3},
            "first_k_in_index_order": {"found_frac": float((f_i >= 0).mean()),
                                       "found_vs_plain": (float((f_i >= 0).sum() / fp)
                                                          if fp else None),
                                       "mean_exact_evals": float(e_i.mean())},
            "network": "the ranking network trained in the search section",
        }
        log("study search: plain found %.3f (RM %.3f) | guided top-%d %.3f | first %d %.3f" % (
            res["search_8_chains"]["plain"]["found_frac"],
            res["search_8_chains"]["rm_schedulable_frac"], top_k,
            res["search_8_chains"]["guided_top_k_only"]["found_frac"], top_k,
            res["search_8_chains"]["first_k_in_index_order"]["found_frac"]))
        dev.free()
    res["setup_s"] = time.perf_counter() - t0
    return res


def units_section(args, torch, log):
    """Several units of one accelerator type (Sec. IV-E): segments bound to
    units by worst-fit decreasing at upload, per segment, per callback or per
    chain, then analysed with each unit as its own accelerator.  Schedulable
    fraction on the study's sets against the unit count, every set compared
    with the oracle (binding and verdict); the binding kernel's rate on sweep
    sets."""
    import oracle
    from paper_2404_06452_amd import _paam, chaingen

    stream = torch.cuda.Stream()
    n = args.units_sets
    t0 = time.perf_counter()
    groups = (("segment", _paam.PAAM_UNITS_SEGMENT), ("callback", _paam.PAAM_UNITS_CALLBACK),
              ("chain", _paam.PAAM_UNITS_CHAIN))
    points = ((8, 5, 5), (8, 7, 3), (16, 5, 5))
    res, mism = {}, 0
    for n_chains, acc, cpu in points:
        cs = chaingen.generate(chaingen.study_params(n_chains, acc, cpu), n)
        key = "%d_chains_%d:%d" % (n_chains, acc, cpu)
        res[key] = {}
        for gname, g in groups:
            fr = []
            for k in (1, 2, 3, 4):
                units = np.full(int(cs.set_accel_off[-1]), k, np.int16)
                dev = _paam.Chainset(cs, device="cuda:0", units=units, unit_group=g)
                su = dev.seg_units().cpu().numpy()
                r = _paam.wcrt(dev, full=False)
                dev.free()
                ref = oracle.wfd_units(cs, units, g)
                ro = oracle.wcrt(oracle.split_units(cs, units, ref), full=False,
                                 threads=os.cpu_count() or 1)
                mism += int((su != ref).sum()) + int((r["sched"] != ro["sched"]).sum())
                fr.append(float((r["sched"] == 1).mean()))
            res[key][gname] = {str(k): v for k, v in zip((1, 2, 3, 4), fr)}
        log("units %s: %s" % (key, " | ".join(
            "%s %s" % (gn, " ".join("%.2f" % v for v in res[key][gn].values())) for gn, _ in groups)))
    # binding rate: sweep sets, 4 units, whole chains as items
    m = args.units_rate_sets
    cs = chaingen.generate("sweep", m)
    units = np.full(int(cs.set_accel_off[-1]), 4, np.int16)
    dev = _paam.Chainset(cs, device="cuda:0", units=units, unit_group=_paam.PAAM_UNITS_CHAIN)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        dev.assign_units(stream)
        a.record(stream)
        for _ in range(reps):
            dev.assign_units(stream)
        b.record(stream)
    torch.cuda.synchronize()
    dt = a.elapsed_time(b) * 1e-3 / reps
    su = dev.seg_units().cpu().numpy()
    # the oracle's binding of every sweep set, on one thread (bit-exact)
    tc = time.perf_counter()
    ref = oracle.wfd_units(cs, units, _paam.PAAM_UNITS_CHAIN)
    tc = time.perf_counter() - tc
    sample = m
    mism += int((su != ref).sum())
    dev.free()
    out = {
        "workload": "study sets (%d per point; 4 callbacks per chain, one segment per callback, "
                    "one accelerator type with 1-4 units, each chain on its own executor and "
                    "core), verdict mode" % n,
        "schedulable_frac": res,
        "binding": {"sets": m, "segments": int(cs.n_segments), "units_per_set": 4,
                    "group": "chain", "ms": dt * 1e3, "sets_per_s": m / dt,
                    "segments_per_s": cs.n_segments / dt,
                    "cpu_oracle": {"sets_per_s": m / tc, "s": tc, "threads": 1}},
        "parity_mismatches": mism,
        "parity": "every study set's binding and verdict, and the binding of all %d sweep "
                  "sets, against the oracle" % sample,
        "setup_s": time.perf_counter() - t0,
    }
    log("units binding: %d sweep sets in %.3f ms (%.3g sets/s), mismatches %d" % (
        m, dt * 1e3, m / dt, mism))
    return out


def des_section(args, torch, log):
    """Observed latencies against the bound at scale (the method of the
    paper's Case Study 1, Sec. V-A).  Two workloads: the study's 8-chain sets
    (accelerator : CPU 1:1, every chain on its own executor and core), and
    the small sets (8 chains on two executors that share a core) at 25 % of
    their utilisation, where executor blocking matters.  Every set runs 64
    scenarios (synchronous release, then random offsets), with every job at
    its WCET and again with actual times drawn from [W/2, W].  Every observed
    end-to-end latency of an admitted set is compared with the analysis
    bound (SAFE blocking), and with the bound under the printed blocking term
    of Eq. (5)/(6) for contrast; the kernel's rate; the oracle on a sample,
    bit-exact, and its single-thread rate."""
    import oracle
    from paper_2404_06452_amd import _paam, chaingen

    stream = torch.cuda.Stream()
    n, n_scen = args.des_sets, 64
    t0 = time.perf_counter()
    INF = np.iinfo(np.int64).max
    out = {}
    workloads = (
        ("study_8_chains", chaingen.generate(chaingen.study_params(8, 1, 1), n), 1000,
         "study sets: 8 chains x 4 callbacks, one segment per callback, accelerator : CPU 1:1, "
         "each chain on its own executor and core"),
        ("small_25pct", chaingen.generate("small", n), 250,
         "small sets at 25 % of their utilisation: 8 chains x 2-5 callbacks on two executors "
         "sharing a core, 30 % of callbacks with a segment"),
    )
    for name, cs, util, what in workloads:
        horizon = int(2 * cs.T.max())
        offs = chaingen.release_offsets(cs, n_scen, 2404)
        dev = _paam.Chainset(cs, device="cuda:0")
        safe = _paam.wcrt(dev, full=True, util_permille=util)
        paper = _paam.wcrt(dev, full=True, util_permille=util, blocking=_paam.PAAM_BLOCK_PAPER)
        d_off = torch.as_tensor(offs).cuda()
        obs = torch.empty(cs.n_chains * n_scen, dtype=torch.int64, device="cuda:0")
        status = torch.empty(n * n_scen, dtype=torch.int8, device="cuda:0")
        m = min(n, 2000)
        jobs = 0
        for s_ in range(m):
            c0, c1 = int(cs.set_chain_off[s_]), int(cs.set_chain_off[s_ + 1])
            blk = offs[c0 * n_scen:c1 * n_scen].reshape(n_scen, c1 - c0)
            jobs += int(((horizon - blk) // cs.T[c0:c1] + 1).sum())
        jobs_per_set = jobs / m
        chain_set = np.repeat(np.arange(n), np.diff(cs.set_chain_off))
        adm = (safe["sched"] == 1)[chain_set]
        padm_sets = paper["sched"] == 1
        res = {"workload": "%d %s; %d scenarios per set (0: synchronous release; others: offsets "
                           "uniform in [0, T)); horizon %.3f s; utilisation scale %d permille" % (
                               n, what, n_scen, horizon * 1e-9, util),
               "admitted_sets": int((safe["sched"] == 1).sum()),
               "admitted_sets_printed_blocking": int(padm_sets.sum()),
               "jobs_per_scenario_mean": jobs_per_set / n_scen}
        for label, ex in (("wcet", 1000), ("actual_50_100pct", 500)):
            o = _paam.des_opts(n_scen, horizon, exec_permille=ex, seed=7, util_permille=util)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                a.record(stream)
                _paam.paam_des_batch(dev, o, d_off, obs, status, stream)
                b.record(stream)
            torch.cuda.synchronize()
            dt = a.elapsed_time(b) * 1e-3
            g = obs.cpu().numpy()
            st = status.cpu().numpy()
            per = np.full(cs.n_chains, -1, np.int64)  # largest observation over the scenarios
            for s_ in range(n):
                c0, c1 = int(cs.set_chain_off[s_]), int(cs.set_chain_off[s_ + 1])
                per[c0:c1] = g[c0 * n_scen:c1 * n_scen].reshape(n_scen, c1 - c0).max(0)
            ok = adm & (per >= 0)
            ratio = per[ok] / safe["chain_R"][ok]
            fin = (paper["chain_R"] < INF) & (per >= 0)
            miss = np.zeros(n, bool)  # a latency above the deadline, or a chain two jobs behind
            np.logical_or.at(miss, chain_set, per > cs.D)
            miss |= (st.reshape(n, n_scen) == 1).any(1)
            r = {
                "ms": dt * 1e3, "scenarios_per_s": n * n_scen / dt,
                "jobs_per_s": jobs_per_set * n / dt,
                "status_counts": {str(k): int((st == k).sum()) for k in (0, 1, 2)},
                "chains_observed_in_admitted_sets": int(ok.sum()),
                "above_bound": int((per[ok] > safe["chain_R"][ok]).sum()),
                "observed_over_bound_mean": float(ratio.mean()) if ratio.size else None,
                "observed_over_bound_max": float(ratio.max()) if ratio.size else None,
                "above_printed_blocking_bound": int((per[fin] > paper["chain_R"][fin]).sum()),
                "printed_admitted_sets_with_observed_miss": int((padm_sets & miss).sum()),
            }
            k_sets = args.des_oracle_sets
            sub = cs.subset(range(k_sets))
            tc = time.perf_counter()
            ro = oracle.event_sim(sub, offs[:int(sub.set_chain_off[-1]) * n_scen], n_scen, horizon,
                                  exec_permille=ex, seed=7, util_permille=util)
            tc = time.perf_counter() - tc
            k = int(sub.set_chain_off[-1]) * n_scen
            r["oracle"] = {"sets": k_sets, "threads": 1, "s": tc,
                           "scenarios_per_s": k_sets * n_scen / tc,
                           "mismatches": int((ro["obs"] != g[:k]).sum()) +
                           int((ro["status"] != st[:k_sets * n_scen]).sum())}
            res[label] = r
            log("des %s %s: %d x %d scenarios in %.1f ms (%.3g/s, oracle %.3g/s on one thread, "
                "%d mismatches); above bound %d of %d chains; obs/bound mean %.3f max %.3f; above "
                "printed-blocking bound %d; printed-admitted sets with an observed miss %d" % (
                    name, label, n, n_scen, dt * 1e3, n * n_scen / dt,
                    r["oracle"]["scenarios_per_s"], r["oracle"]["mismatches"], r["above_bound"],
                    ok.sum(), r["observed_over_bound_mean"] or 0, r["observed_over_bound_max"] or 0,
                    r["above_printed_blocking_bound"], r["printed_admitted_sets_with_observed_miss"]))
        dev.free()
        out[name] = res
    out["setup_s"] = time.perf_counter() - t0
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sets", type=int, default=1_000_000)
    ap.add_argument("--cpu-sample", type=int, default=10000,
                    help="sets per level for the single-threaded oracle")
    ap.add_argument("--allcore-sets", type=int, default=100000,
                    help="sets per level compared with the oracle on all host cores (0 skips)")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--waves-per-cu", type=int, default=0)
    ap.add_argument("--search-sets", type=int, default=100_000)
    ap.add_argument("--train-sets", type=int, default=200_000)
    ap.add_argument("--train-samples", type=int, default=10_000_000)
    ap.add_argument("--train-epochs", type=int, default=2)
    ap.add_argument("--skip-search", action="store_true")
    ap.add_argument("--large-sets", type=int, default=100000,
                    help="sets of 256 chains for the large-set section (0 skips it)")
    ap.add_argument("--large-plain-sets", type=int, default=500,
                    help="sets of the large batch searched plainly for comparison")
    ap.add_argument("--study-sets", type=int, default=1000,
                    help="sets per point of the analytical study (0 skips it)")
    ap.add_argument("--units-sets", type=int, default=1000,
                    help="sets per point of the accelerator-units section (0 skips it)")
    ap.add_argument("--units-rate-sets", type=int, default=100000,
                    help="sweep sets whose unit binding is timed")
    ap.add_argument("--des-sets", type=int, default=10000,
                    help="sets of the simulation section (64 scenarios each; 0 skips it)")
    ap.add_argument("--des-oracle-sets", type=int, default=20,
                    help="sets the simulation oracle repeats, bit-exact, on one thread")
    ap.add_argument("--large-util", type=int, default=0,
                    help="optional second utilisation scale of the large-set section, in "
                         "permille (0: the workload's utilisation only)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the analysis shards across GPUs by set range with no "
              "exchange, but this benchmark runs and reports a single MI355X only (--gpus 1).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2404_06452_amd import _paam, chaingen

    levels = list(chaingen.SWEEP_LEVELS)
    t0 = time.perf_counter()
    cs = chaingen.generate("sweep", args.sets)
    log("generated %d sets (%d chains, %d callbacks, %d segments) in %.1f s" % (
        cs.n_sets, cs.n_chains, cs.n_callbacks, cs.n_segments, time.perf_counter() - t0))
    t0 = time.perf_counter()
    dev = _paam.Chainset(cs, device="cuda:0")
    log("uploaded %.2f GB arena, %d sub-chains in %.1f s" % (
        dev.arena.numel() / 1e9, dev.n_subchains, time.perf_counter() - t0))

    stream = torch.cuda.Stream()
    copy_gbs = copy_calibration(torch, stream)
    log("plain device copy: %.0f GB/s (read + write)" % copy_gbs)
    outs = [_paam.WcrtOut(dev, True) for _ in levels]
    tune = None
    wpc = args.waves_per_cu
    if wpc == 0:
        # schedule autotuner (library): persistent waves per CU, timed on the
        # middle level of the sweep
        cands = [4, 8, 12, 16, 20, 24]
        t_opts = _paam.wcrt_opts(full=True, util_permille=levels[len(levels) // 2])
        ws_t = _paam.workspace(_paam.paam_wcrt_bytes(
            dev, _paam.wcrt_opts(full=True, waves_per_cu=max(cands))))
        best_ms = _paam.paam_wcrt_autotune(dev, t_opts, cands, 1, outs[0], ws_t, stream)
        wpc = int(t_opts.waves_per_cu)  # 0: the per-class choices stored in the handle
        sched = _paam.paam_wcrt_schedule(dev)
        tune = {"candidates_waves_per_cu": cands, "candidates_evals_per_step": [1, 2, 3],
                "per_class": [{"max_chains": c, "sets": n, "waves_per_cu": w,
                               "evals_per_step": m} for c, n, w, m in sched],
                "best_ms_per_level": best_ms, "level": levels[len(levels) // 2] / 1000}
        log("autotune: %s (%.1f ms per level)" % (
            ", ".join("<=%d chains: %d waves/CU x %d" % (c, w, m) for c, n, w, m in sched),
            best_ms))
        del ws_t
    opts = [_paam.wcrt_opts(full=True, util_permille=u, waves_per_cu=wpc) for u in levels]
    ws = _paam.workspace(max(_paam.paam_wcrt_bytes(dev, o) for o in opts))

    def sweep(s):
        for o, out in zip(opts, outs):
            _paam.paam_wcrt_batch(dev, o, out, ws, s)

    graph = None
    with torch.cuda.stream(stream):
        sweep(stream)  # eager run: also the reference for the graph replays
    torch.cuda.synchronize()
    eager = [(o.set_sched.clone(), o.chain_R.clone()) for o in outs]
    if not args.no_graph:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            sweep(torch.cuda.current_stream())
        torch.cuda.synchronize()

    def step():
        if graph is not None:
            graph.replay()
        else:
            sweep(stream)

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            step()
    torch.cuda.synchronize()
    # graph replays must reproduce the eager results exactly
    for (s0, r0), o in zip(eager, outs):
        assert torch.equal(s0, o.set_sched) and torch.equal(r0, o.chain_R), "graph replay differs"

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for a, b in ev:
            a.record(stream)
            step()
            b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [a.elapsed_time(b) for a, b in ev]
    ms_per_step = wall * 1e3 / args.steps
    analyses = cs.n_sets * len(levels)
    value = analyses * args.steps / wall
    # the library launches the analysis once per size class of sets (chain
    # count up to 16, 32, 64, ...): launches per level = classes present
    sizes = np.diff(cs.set_chain_off)
    n_classes = len(np.unique(np.ceil(np.log2(np.maximum(sizes, 16) / 16)).astype(int)))
    launch_ms = float(np.mean(step_ms)) / (len(levels) * n_classes)
    log("%.1f ms/step (events %.1f), %.3g analyses/s" % (ms_per_step, np.mean(step_ms), value))

    # verdict-only mode (stops a set at its first missed deadline), one sweep
    vopts = [_paam.wcrt_opts(full=False, util_permille=u, waves_per_cu=wpc) for u in levels]
    vout = _paam.WcrtOut(dev, False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    with torch.cuda.stream(stream):
        for o in vopts:
            _paam.paam_wcrt_batch(dev, o, vout, ws, stream)
    torch.cuda.synchronize()
    verdict_rate = analyses / (time.perf_counter() - t1)

    # double-bounding ablation: the sweep again with Lemma 2 only and with
    # Lemma 3 only (every chain's bound), against the min of both used above
    ablation = ablation_section(torch, dev, levels, outs, ws, stream, log)

    # CPU oracle on a bounded sample of the same sweep (single thread), and
    # bit-exact comparison of the GPU outputs on that sample
    import oracle
    n_s = min(args.cpu_sample, cs.n_sets)
    sample = cs.subset(range(n_s))
    terms_per_level, cpu_time, mism = [], 0.0, 0
    sched_rate = []
    for li, u in enumerate(levels):
        t1 = time.perf_counter()
        r = oracle.wcrt(sample, full=True, util_permille=u)
        cpu_time += time.perf_counter() - t1
        terms_per_level.append(float(r["terms"].mean()))
        g_sched = outs[li].set_sched[:n_s].cpu().numpy()
        g_R = outs[li].chain_R[:int(sample.n_chains)].cpu().numpy()
        mism += int(np.sum(g_sched != r["sched"])) + int(np.sum(g_R != r["chain_R"]))
        sched_rate.append(float(outs[li].set_sched.float().mean().item()))
    cpu_rate = n_s * len(levels) / cpu_time
    log("oracle: %d analyses in %.1f s; mismatches %d" % (n_s * len(levels), cpu_time, mism))
    allcore = allcore_parity(args, cs, levels, outs, oracle, log)
    mism += allcore["mismatches"] if allcore else 0
    other_cpu = other_cpu_legs(args, oracle, log)

    # HBM view: the problem statement's bytes (every input field of every set
    # once) plus the outputs, per level, over the level's time
    out_bytes = cs.n_sets * (1 + 4 + 8) + cs.n_chains * 8
    level_bytes = cs.nbytes() + out_bytes
    hbm_rate = level_bytes / (launch_ms * n_classes * 1e-3)
    hbm = {"algorithmic_bytes_per_level": level_bytes, "achieved_GBps": hbm_rate / 1e9,
           "frac_of_8TBps": hbm_rate / 8e12, "frac_of_measured_copy": hbm_rate / (copy_gbs * 1e9),
           "note": "input fields of the problem statement read once per level plus outputs; "
                   "the analysis is ALU-bound (roofline)"}

    # roofline: algorithmic terms per launch (oracle count per analysis on the
    # sample x sets per launch) over the average launch duration
    terms_per_launch = float(np.mean(terms_per_level)) * cs.n_sets / n_classes
    achieved = terms_per_launch / (launch_ms * 1e-3)
    line = {
        "metric": "WCRT analyses/sec bit-exact",
        "value": value,
        "unit": "analyses/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "utilisation sweep: %d chain sets x %d levels (0.10-0.95), 4-64 chains x "
                        "2-12 callbacks, 4 executors, 1 accelerator; every chain's end-to-end "
                        "bound, cap = deadline" % (cs.n_sets, len(levels)),
            "n_sets": cs.n_sets, "levels": len(levels), "analyses_per_step": analyses,
            "chains": cs.n_chains, "callbacks": cs.n_callbacks, "segments": cs.n_segments,
            "subchains": dev.n_subchains, "hip_graph": graph is not None,
            "waves_per_cu": wpc, "autotune": tune,
            "parallelism": "single GPU",
        },
        "parity": {"sampled_analyses": n_s * len(levels), "mismatches": mism,
                   "compared": "set verdicts and every chain bound vs the CPU oracle"},
        "verdict_mode_analyses_per_s": verdict_rate,
        "bound_ablation": ablation,
        "schedulable_fraction_by_level": dict(zip([u / 1000 for u in levels], sched_rate)),
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e9,
            "peak": PEAK_TERMS / 1e9,
            "unit": "Gterm/s",
            "frac": achieved / PEAK_TERMS,
            "traffic": measured_traffic(cs.n_sets, wpc),
            "kernel": "wcrt_kernel",
            "avg_launch_ms": launch_ms,
            "launches_per_level": n_classes,
            "copy_GBps_measured": copy_gbs,
            "terms_per_analysis": float(np.mean(terms_per_level)),
        },
        "cpu_baseline": {
            "value": cpu_rate, "unit": "analyses/s", "cores": 1, "kind": "oracle",
            "sample": "first %d sets of the same batch at all %d levels (%d analyses), full "
                      "mode" % (n_s, len(levels), n_s * len(levels)),
            "all_core_parity": allcore,
            "other_workloads_single_core": other_cpu,
        },
        "hbm": hbm,
        "manifest": manifest(args, torch, _paam),
    }
    if not args.skip_search:
        del graph, eager, dev, outs, ws, vout
        torch.cuda.empty_cache()
        line["search"], net = search_section(args, torch, log)
        torch.cuda.empty_cache()
        if args.large_sets > 0:
            line["large"] = large_section(args, torch, log, net)
    else:
        net = None
    if args.study_sets > 0:
        line["study"] = study_section(args, torch, log, net)
    if args.units_sets > 0:
        line["units"] = units_section(args, torch, log)
        mism += line["units"]["parity_mismatches"]
    if args.des_sets > 0:
        line["des"] = des_section(args, torch, log)
        mism += sum(line["des"][w][k]["oracle"]["mismatches"] for w in ("study_8_chains", "small_25pct")
                    for k in ("wcet", "actual_50_100pct"))
    print(json.dumps(line), flush=True)
    if mism:
        sys.exit(1)


if __name__ == "__main__":
    main()
