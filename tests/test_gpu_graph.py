"""The analysis and the search captured in one HIP graph and replayed.

The benchmark times graph replays, so the captured launches must reproduce
the eager ones on every replay: the work-queue counters are cleared by a
kernel inside the graph, never by a memset node.  Each replay follows eager
work on the same device (other analyses, torch ops), and its outputs are
scribbled over beforehand so that a replay that writes nothing fails."""
import sys

import numpy as np
import pytest

import oracle
from paper_2404_06452_amd import chaingen

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_graph_replays_match_eager_and_oracle():
    import torch

    from paper_2404_06452_amd import _paam
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    note("graph: sweep 1500 sets (three size classes) at levels 0.02 and 0.85 + search 300 sets x 64")
    cs = chaingen.generate("sweep", 1500, set_begin=777)
    ss = chaingen.generate("search", 300, set_begin=4242)
    dev = _paam.Chainset(cs)
    sdev = _paam.Chainset(ss)
    levels = (20, 850)  # 13 % of the sets schedulable at the first, none at the second
    wo = [_paam.wcrt_opts(full=True, util_permille=u) for u in levels]
    wout = [_paam.WcrtOut(dev, True) for _ in levels]
    wws = [_paam.workspace(_paam.paam_wcrt_bytes(dev, o)) for o in wo]
    so = _paam.search_opts(64, 31, util_permille=50)
    sout = _paam.SearchOut(sdev)
    sws = _paam.workspace(_paam.paam_search_bytes(sdev, so))
    stream = torch.cuda.Stream()

    def step(s):
        for o, out, ws in zip(wo, wout, wws):
            _paam.paam_wcrt_batch(dev, o, out, ws, s)
        _paam.paam_priority_search(sdev, so, sout, sws, s)

    def snapshot():
        torch.cuda.synchronize()
        snap = [(o.set_sched.cpu().numpy(), o.set_worst.cpu().numpy(),
                 o.set_worst_R.cpu().numpy(), o.chain_R.cpu().numpy()[:cs.n_chains]) for o in wout]
        snap.append((sout.found.cpu().numpy(), sout.n_exact.cpu().numpy(),
                     sout.found_prio.cpu().numpy()[:ss.n_chains]))
        return snap

    def scribble():
        for o in wout:
            o.set_sched.fill_(-7)
            o.set_worst.fill_(-7)
            o.set_worst_R.fill_(-7)
            o.chain_R.fill_(-7)
        sout.found.fill_(-7)
        sout.n_exact.fill_(-7)
        sout.found_prio.fill_(-7)

    with torch.cuda.stream(stream):
        step(stream)
    eager = snapshot()

    # the eager outputs against the oracle
    for u, (sched, worst, worst_R, chain_R) in zip(levels, eager[:2]):
        r = oracle.wcrt(cs, full=True, util_permille=u, threads=8)
        assert np.array_equal(sched, r["sched"]), u
        assert np.array_equal(worst, r["worst"]), u
        assert np.array_equal(worst_R, r["worst_R"]), u
        assert np.array_equal(chain_R, r["chain_R"]), u
    r = oracle.search(ss, 64, 31, util_permille=50, threads=8)
    assert np.array_equal(eager[2][0], r["found"])
    assert np.array_equal(eager[2][1], r["n_eval"])
    assert (eager[2][0] >= 0).any(), "the search workload should admit some sets"

    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        step(torch.cuda.current_stream())
    torch.cuda.synchronize()

    other = _paam.wcrt_opts(full=False, util_permille=600)
    oout = _paam.WcrtOut(dev, False)
    ows = _paam.workspace(_paam.paam_wcrt_bytes(dev, other))
    x = torch.randn(512, 512, device="cuda:0")
    for rep in range(4):
        note("graph: replay %d" % rep)
        # eager work between replays: another analysis and torch kernels
        _paam.paam_wcrt_batch(dev, other, oout, ows)
        x = torch.tanh(x @ x.T / 512.0)
        torch.cuda.synchronize()
        scribble()
        torch.cuda.synchronize()
        graph.replay()
        got = snapshot()
        for a, b in zip(eager[:2], got[:2]):
            for u, v in zip(a, b):
                assert np.array_equal(u, v), "replay %d differs from the eager outputs" % rep
        assert np.array_equal(eager[2][0], got[2][0]), rep
        assert np.array_equal(eager[2][1], got[2][1]), rep
        # the found order is written for sets with a find and leaves the
        # priorities of the other sets untouched
        found_chain = np.repeat(eager[2][0] >= 0, np.diff(ss.set_chain_off))
        assert np.array_equal(got[2][2][found_chain], eager[2][2][found_chain]), rep
        assert (got[2][2][~found_chain] == -7).all(), rep
    del graph


def test_graph_replays_of_scoring_and_guided_search():
    """Features, network forward and the guided confirmation of the top 8,
    captured together: every replay reproduces the eager scores, finds and
    evaluation counts bit for bit.  (The oracle parity of each step, on
    seeded scores for the search, is covered by the surrogate and search
    tests.)"""
    import torch

    from paper_2404_06452_amd import _paam
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    note("graph: scoring + guided top-8, search 400 sets x 128")
    n_cand, seed, top_k, util = 128, 9, 8, 50
    ss = chaingen.generate("search", 400, set_begin=9100)
    sdev = _paam.Chainset(ss)
    net = _paam.Network(chaingen.mlp_init(3), device="cuda:0")
    scores = torch.empty(ss.n_sets * n_cand, dtype=torch.float32, device="cuda:0")
    so = _paam.search_opts(n_cand, seed, util_permille=util)
    go = _paam.search_opts(n_cand, seed, guided=True, top_k=top_k, fallback=False, scores=scores,
                           util_permille=util)
    sout = _paam.SearchOut(sdev, with_prio=False)
    sws = _paam.workspace(_paam.paam_score_bytes(sdev, so))
    gws = _paam.workspace(_paam.paam_search_bytes(sdev, go))
    stream = torch.cuda.Stream()

    def step(s):
        _paam.paam_score_candidates(sdev, so, net.params, net.packed, scores, sws, s)
        _paam.paam_priority_search(sdev, go, sout, gws, s)

    def snapshot():
        torch.cuda.synchronize()
        return (scores.cpu().numpy().copy(), sout.found.cpu().numpy(), sout.n_exact.cpu().numpy())

    with torch.cuda.stream(stream):
        step(stream)
    eager = snapshot()
    assert np.isfinite(eager[0]).all()
    assert (eager[1] >= 0).any(), "the guided search should admit some sets"
    assert ((eager[2] >= 1) & (eager[2] <= top_k)).all()

    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        step(torch.cuda.current_stream())
    torch.cuda.synchronize()
    x = torch.randn(256, 256, device="cuda:0")
    for rep in range(3):
        note("graph: scoring replay %d" % rep)
        x = torch.relu(x @ x.T / 256.0)
        scores.fill_(float("nan"))
        sout.found.fill_(-7)
        sout.n_exact.fill_(-7)
        torch.cuda.synchronize()
        graph.replay()
        got = snapshot()
        for u, v in zip(eager, got):
            assert np.array_equal(u, v), "scoring replay %d differs from the eager outputs" % rep
    del graph
