"""GPU parity of paam_wcrt_batch against the CPU oracle, bit-exact (int64).

The analysis is integer arithmetic, so every bound, verdict and worst chain
must be identical to the oracle's on the same seeded inputs."""
import glob
import json
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2404_06452_amd import chaingen

pytestmark = pytest.mark.gpu

GOLDEN = sorted(glob.glob(os.path.join(os.path.dirname(__file__), "golden", "ex_*.json")))


@pytest.fixture(scope="module")
def paam():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2404_06452_amd import _paam
    return _paam


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


OPTS = [
    dict(full=True),
    dict(full=False),
    dict(full=True, blocking=1),
    dict(full=True, cap_mult=2),
    dict(full=True, bound=1),
    dict(full=True, bound=2),
    dict(full=False, cap_mult=3, blocking=1),
]


def compare(paam, cs, dev, opts, label):
    o = dict(opts)
    g = paam.wcrt(dev, **o)
    r = oracle.wcrt(cs, threads=8, **o)
    assert np.array_equal(g["sched"], r["sched"]), label
    assert np.array_equal(g["worst"], r["worst"]), label
    assert np.array_equal(g["worst_R"], r["worst_R"]), label
    if o.get("full", True):
        bad = np.nonzero(g["chain_R"] != r["chain_R"])[0]
        assert bad.size == 0, (label, bad[:10], g["chain_R"][bad[:10]], r["chain_R"][bad[:10]])
    return g


def test_worked_examples_on_gpu(paam):
    sets, expect = [], []
    for p in GOLDEN:
        fx = json.load(open(p))
        sets.append(fx["set"])
    cs = chaingen.from_sets(sets)
    dev = paam.Chainset(cs)
    note("golden: %d sets" % cs.n_sets)
    for opts in OPTS:
        compare(paam, cs, dev, opts, ("golden", opts))


@pytest.mark.parametrize("preset", ["small", "small_overheads"])
def test_small_config_all_options(paam, preset):
    cs = chaingen.generate(preset, 1000)
    dev = paam.Chainset(cs)
    for opts in OPTS:
        note("%s %s" % (preset, opts))
        compare(paam, cs, dev, opts, (preset, opts))


def test_schedulable_mix_and_multi_accelerator(paam):
    p = chaingen.PRESETS["small"].replace(seed=77, chains=(1, 9), cbs=(1, 4), n_exec=5,
                                          util=(0.02, 0.5), pseg=(0.2, 0.8), frac=(0.05, 0.9),
                                          T=(20.0, 4000.0), n_accel=3, max_seg_per_cb=3,
                                          n_buckets=3, eps=2, kappa=1, eps_hop=1)
    cs = chaingen.generate(p, 3000)
    dev = paam.Chainset(cs)
    for opts in OPTS:
        note("mix %s" % opts)
        g = compare(paam, cs, dev, opts, ("mix", opts))
    assert 0.05 < g["sched"].mean() < 0.95


@pytest.mark.parametrize("level", [100, 350, 600, 950])
def test_sweep_sets_at_levels(paam, level):
    cs = chaingen.generate("sweep", 1500)
    dev = paam.Chainset(cs)
    for full in (True, False):
        note("sweep level %d full=%s" % (level, full))
        compare(paam, cs, dev, dict(full=full, util_permille=level), ("sweep", level, full))


def test_search_shaped_sets(paam):
    for U in ((0.5, 0.9), (0.02, 0.2)):
        cs = chaingen.generate(chaingen.PRESETS["search"].replace(util=U), 2000)
        dev = paam.Chainset(cs)
        for opts in (dict(full=True), dict(full=False), dict(full=True, cap_mult=2)):
            note("search-shaped %s %s" % (U, opts))
            compare(paam, cs, dev, opts, ("search", U, opts))


def test_large_sets_sample(paam):
    cs = chaingen.generate("large", 12)
    dev = paam.Chainset(cs)
    for opts in (dict(full=True), dict(full=False), dict(full=True, cap_mult=2)):
        note("large %s" % opts)
        compare(paam, cs, dev, opts, ("large", opts))


def test_mixed_size_classes_in_one_batch(paam):
    # chain counts from 8 to 130 in one upload: the analysis and the search
    # launch once per size class (up to 16, 32, 64, 128, 256 chains), several
    # accelerators with bucket levels and overheads
    for ne, eps, util in ((6, 391_000, (0.02, 0.3)), (3, 0, (0.005, 0.05))):
        params = chaingen.PRESETS["large"].replace(
            chains=(8, 130), cbs=(2, 8), n_exec=ne, n_accel=3, max_seg_per_cb=2, n_buckets=4,
            eps=eps, kappa=eps // 3, eps_hop=eps, util=util)
        cs = chaingen.generate(params, 40)
        _mixed_classes(paam, cs, (ne, eps))


def _mixed_classes(paam, cs, tag):
    dev = paam.Chainset(cs)
    for opts in (dict(full=True), dict(full=False), dict(full=True, cap_mult=2),
                 dict(full=True, blocking=1)):
        note("mixed classes %s %s" % (tag, opts))
        compare(paam, cs, dev, opts, ("mixed classes", tag, opts))


def test_empty_and_degenerate_batches(paam):
    # a single one-callback chain, a chain with zero WCET, one executor
    sets = [
        {"chains": [{"T": 10, "D": 10, "prio": 1, "cbs": [{"E": 0, "exec": 0, "segs": []}]}],
         "exec_core": [0], "exec_prio": [1]},
        {"chains": [{"T": 10, "D": 5, "prio": 1, "cbs": [{"E": 3, "exec": 0, "segs": [(2, 0)]}]},
                    {"T": 7, "D": 7, "prio": 2, "cbs": [{"E": 0, "exec": 1, "segs": [(0, 0)]}]}],
         "exec_core": [0, 0], "exec_prio": [1, 2]},
    ]
    cs = chaingen.from_sets(sets)
    dev = paam.Chainset(cs)
    for opts in OPTS:
        compare(paam, cs, dev, opts, ("degenerate", opts))


def test_repeatable_and_schedule_independent(paam):
    """Identical results across launches and persistent-grid sizes (a data
    race or an order-dependent iteration would show up here)."""
    # 20,000 sets: the class of 33-64 chains holds more than 8,192, so at 32
    # waves per CU its grid is twice what its LDS lets the CUs hold at once
    cs = chaingen.generate("sweep", 20000, set_begin=5000)
    dev = paam.Chainset(cs)
    ref = paam.wcrt(dev, full=True, util_permille=400)
    for w in (1, 2, 4, 16, 32):
        g = paam.wcrt(dev, full=True, util_permille=400, waves_per_cu=w)
        for k in ref:
            assert np.array_equal(ref[k], g[k]), (w, k)


def test_autotune_picks_a_candidate_and_keeps_results():
    import torch

    from paper_2404_06452_amd import _paam
    cs = chaingen.generate("sweep", 300)
    dev = _paam.Chainset(cs, device="cuda:0")
    o = _paam.wcrt_opts(full=True, util_permille=300)
    out = _paam.WcrtOut(dev, True)
    ws = _paam.workspace(_paam.paam_wcrt_bytes(dev, _paam.wcrt_opts(full=True, waves_per_cu=8)))
    ms = _paam.paam_wcrt_autotune(dev, o, [2, 4, 8], 2, out, ws)
    torch.cuda.synchronize()
    assert o.waves_per_cu == 0 and ms > 0
    sched = _paam.paam_wcrt_schedule(dev)
    assert len(sched) >= 2 and sum(n for _, n, _, _ in sched) == cs.n_sets
    assert all(w in (2, 4, 8) and m in (1, 2, 3) for _, _, w, m in sched), sched
    r = oracle.wcrt(cs, full=True, util_permille=300)
    assert np.array_equal(out.chain_R.cpu().numpy()[:cs.n_chains], r["chain_R"])
    assert np.array_equal(out.set_sched.cpu().numpy(), r["sched"])
    # later calls with waves_per_cu = 0 run the tuned per-class schedule
    ws2 = _paam.workspace(_paam.paam_wcrt_bytes(dev, o))
    out.chain_R.fill_(-1)
    _paam.paam_wcrt_batch(dev, o, out, ws2)
    torch.cuda.synchronize()
    assert np.array_equal(out.chain_R.cpu().numpy()[:cs.n_chains], r["chain_R"])


@pytest.mark.gpu
def test_verdict_mode_equals_full_mode_verdicts_at_scale(paam):
    # Verdict mode stops a set at its first proven miss: lower bounds checked
    # before Lemma 2 (segments at A* + same-bucket blocking) and before the
    # iteration.  Its verdict must equal the full analysis's on every set, on
    # the sweep workload (4-64 chains) at low, middle and high levels, and on
    # the search sets, whose uploaded order is candidate 0 of a search (the
    # search's sweep analysis, with the same checks, against the full
    # analysis of the queue-driven engine).
    cs = chaingen.generate("sweep", 60_000)
    dev = paam.Chainset(cs, device="cuda:0")
    for u in (100, 300, 550, 950):
        note("sweep verdicts at %d" % u)
        f = paam.wcrt(dev, full=True, util_permille=u)
        v = paam.wcrt(dev, full=False, util_permille=u)
        assert np.array_equal(f["sched"], v["sched"]), u
        assert 0 < int(np.sum(f["sched"] == 0)) and (u > 300 or int(np.sum(f["sched"] == 1)) > 0)
    cs = chaingen.generate("search", 20_000)
    dev = paam.Chainset(cs, device="cuda:0")
    for u in (50, 200, 1000):
        note("search-set verdicts at %d" % u)
        f = paam.wcrt(dev, full=True, util_permille=u)
        g = paam.search(dev, 1, 7, util_permille=u)
        assert np.array_equal(g["found"] == 0, f["sched"] == 1), u
