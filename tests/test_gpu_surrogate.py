"""GPU parity of the candidate-ranking path against the oracle.

Features, candidate analyses and guided search are integer/bit work: exact.
The network's forward pass multiplies bfloat16 operands with float32
accumulation where the oracle sums in float64 at the same rounding points; the
tolerance per candidate is 2^-7 * S with S = sum_j |w3_j * h2_j| + |b3| (the
magnitude of the output's terms): two bfloat16 ulps of it, which covers one
flipped bfloat16 rounding of an element of p or h2 and exceeds float32
accumulation error (about 256 * 2^-24 * S) by far.  Gradients are compared by
relative norm per parameter block (1e-3): float32 accumulation over a batch,
and a rare ReLU whose pre-activation sits within rounding of zero.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import features as of
from oracle import mlp as om
from paper_2404_06452_amd import _paam, chaingen
from paper_2404_06452_amd.surrogate import Trainer

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SEED = 0x5EED


def _pairs(cs, n, seed, n_cand=256, utils=(1000,)):
    rng = np.random.default_rng(seed)
    p = np.zeros((n, 3), np.int64)
    p[:, 0] = rng.integers(0, cs.n_sets, n)
    p[:, 1] = rng.integers(0, n_cand, n)
    p[:, 2] = rng.choice(utils, n)
    return p


def _check_features(cs, pairs, seed=SEED):
    dev = _paam.Chainset(cs, device=DEV)
    g = _paam.features(dev, pairs, seed)
    for i, (s, k, u) in enumerate(pairs):
        order = oracle.candidate_order(cs, int(s), seed, int(k))
        ref = of.features_bf16(cs.set_dict(int(s)), order, int(u))
        C = ref.shape[0]
        assert g["count"][i] == C
        diff = np.argwhere(g["feat"][i, :C] != ref)
        assert diff.size == 0, (i, (s, k, u), [(of.NAMES[f], g["feat"][i, c, f], ref[c, f])
                                               for c, f in diff[:4]])


# sets of up to 64 chains run the segmented scans of one pass's candidates;
# "multi" has three accelerators with three bucket levels and overheads;
# "mixed" holds sets on both sides of 64 chains in one batch
VARIANTS = {
    "multi": ("small", dict(n_accel=3, max_seg_per_cb=2, n_buckets=3, eps=391_000,
                            kappa=129_180, eps_hop=391_000, chains=(3, 20))),
    "mixed": ("large", dict(chains=(30, 90), n_accel=2, n_buckets=4, n_exec=6)),
}


@pytest.mark.parametrize("preset,n_sets,n_pairs,utils", [
    ("small_overheads", 20, 60, (1000, 250)),
    ("sweep", 30, 60, (100, 550, 950)),
    ("search", 20, 60, (1000, 50)),
    ("multi", 20, 60, (1000, 300)),
    ("mixed", 6, 24, (1000,)),
])
def test_features_bit_exact(preset, n_sets, n_pairs, utils):
    if preset in VARIANTS:
        base, kw = VARIANTS[preset]
        cs = chaingen.generate(chaingen.PRESETS[base].replace(**kw), n_sets)
    else:
        cs = chaingen.generate(preset, n_sets)
    _check_features(cs, _pairs(cs, n_pairs, 1, utils=utils))


def test_features_large_sets_and_edges():
    cs = chaingen.generate("large", 2)
    _check_features(cs, np.array([[0, 0, 1000], [1, 1023, 400]], np.int64))
    # 65-140 chains (the prefix-scan schedule over more than one 64-rank
    # chunk), three accelerators with five bucket levels each
    mid = chaingen.PRESETS["large"].replace(**MID)
    cs = chaingen.generate(mid, 3)
    _check_features(cs, _pairs(cs, 6, 8, utils=(1000, 300)))
    # a lone chain, a set with no accelerator segments, a 1-chain walk
    lone = chaingen.from_sets([
        {"chains": [{"T": 100, "D": 90, "prio": 1, "cbs": [{"E": 7, "exec": 0, "segs": [(3, 0)]}]}],
         "exec_core": [0], "exec_prio": [1]},
        {"chains": [{"T": 50, "prio": 2, "cbs": [{"E": 5, "exec": 0}]},
                    {"T": 80, "prio": 1, "cbs": [{"E": 5, "exec": 1}, {"E": 4, "exec": 0}]}],
         "exec_core": [0, 0], "exec_prio": [2, 1], "accel_buckets": [], "accel_eps": [],
         "accel_kappa": []},
    ])
    _check_features(lone, np.array([[0, 0, 1000], [0, 5, 1000], [1, 3, 700], [1, 0, 1000]],
                                   np.int64))


def test_features_bad_pairs_and_empty():
    cs = chaingen.generate("small", 3)
    dev = _paam.Chainset(cs, device=DEV)
    g = _paam.features(dev, np.array([[0, 0, 1000], [7, 0, 1000], [1, -1, 1000]], np.int64), SEED)
    assert list(g["count"]) == [8, -1, -1]
    g = _paam.features(dev, np.zeros((0, 3), np.int64), SEED)
    assert g["count"].size == 0


@pytest.mark.parametrize("preset,n_sets,n_pairs,cap", [
    ("small", 40, 80, 2), ("small_overheads", 30, 60, 2), ("sweep", 40, 60, 2), ("search", 40, 80, 1),
])
def test_candidate_wcrt_exact(preset, n_sets, n_pairs, cap):
    cs = chaingen.generate(preset, n_sets)
    dev = _paam.Chainset(cs, device=DEV)
    pairs = _pairs(cs, n_pairs, 2, utils=(1000, 300, 100))
    g = _paam.candidates(dev, pairs, SEED, cap_mult=cap)
    r = oracle.candidate_analysis(cs, pairs, SEED, cap_mult=cap)
    for k in ("sched", "worst_R", "worst_D", "ratio"):
        assert np.array_equal(g[k], r[k]), k
    bad = _paam.candidates(dev, np.array([[n_sets, 0, 1000]], np.int64), SEED)
    assert bad["sched"][0] == -2


def test_candidate_wcrt_independent_of_the_persistent_grid():
    # 6,000 pairs: at 32 waves per CU the grid holds more waves than the CUs
    # run at once; every grid gives the oracle's targets
    cs = chaingen.generate("sweep", 400, set_begin=31000)
    dev = _paam.Chainset(cs, device=DEV)
    pairs = _pairs(cs, 6000, 5, utils=(1000, 400, 60))
    r = oracle.candidate_analysis(cs, pairs, SEED, cap_mult=2)
    for w in (1, 4, 32):
        g = _paam.candidates(dev, pairs, SEED, cap_mult=2, waves_per_cu=w)
        for k in ("sched", "worst_R", "worst_D", "ratio"):
            assert np.array_equal(g[k], r[k]), (w, k)


@pytest.mark.parametrize("preset,n_sets,n_cand,top_k,fallback,util,ties", [
    ("small", 60, 64, 8, True, 100, False),
    ("small", 60, 64, 8, False, 100, True),
    ("search", 40, 128, 16, True, 50, False),
    ("search", 40, 64, 64, False, 40, True),
    ("sweep", 30, 32, 1, True, 100, False),
])
def test_guided_search_exact(preset, n_sets, n_cand, top_k, fallback, util, ties):
    cs = chaingen.generate(preset, n_sets)
    dev = _paam.Chainset(cs, device=DEV)
    sc = chaingen.random_scores(n_sets * n_cand, 3, ties=ties)
    g = _paam.search(dev, n_cand, SEED, scores=torch.from_numpy(sc).to(DEV), guided=True,
                     top_k=top_k, fallback=fallback, util_permille=util)
    r = oracle.guided_search(cs, n_cand, SEED, sc, top_k, fallback=fallback, util_permille=util)
    assert np.array_equal(g["found"], r["found"])
    assert np.array_equal(g["n_exact"], r["n_eval"])


def test_guided_search_special_scores():
    cs = chaingen.generate("small", 8)
    dev = _paam.Chainset(cs, device=DEV)
    n_cand = 16
    sc = np.tile(np.array([np.nan, -0.0, 0.0, -1.0, 5.0, np.nan, 1e-30, -1e-30] * 2, np.float32), 8)
    g = _paam.search(dev, n_cand, SEED, scores=torch.from_numpy(sc).to(DEV), guided=True,
                     top_k=5, fallback=False, util_permille=60)
    r = oracle.guided_search(cs, n_cand, SEED, sc, 5, fallback=False, util_permille=60)
    assert np.array_equal(g["found"], r["found"]) and np.array_equal(g["n_exact"], r["n_eval"])


def _network_batch(preset="sweep", n_sets=40, n=70, util=300, seed=7):
    """GPU features of n pairs, and the oracle's own features of the same
    pairs as float64 bfloat16 values (the oracle's input never comes from the
    GPU; the two are also checked equal)."""
    cs = chaingen.generate(preset, n_sets)
    dev = _paam.Chainset(cs, device=DEV)
    pairs = _pairs(cs, n, 3, utils=(util,))
    f = _paam.features(dev, pairs, seed)
    rows, ro = [], [0]
    for (s, k, u) in pairs:
        ref = of.features_bf16(cs.set_dict(int(s)), oracle.candidate_order(cs, int(s), seed, int(k)),
                               int(u))
        rows.append(ref)
        ro.append(ro[-1] + ref.shape[0])
    for i, r in enumerate(rows):
        assert np.array_equal(f["feat"][i, :r.shape[0]], r)
    x = (np.concatenate(rows).astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    feat = torch.from_numpy(f["feat"].reshape(-1).view(np.int16).copy()).to(DEV)
    count = torch.from_numpy(f["count"].astype(np.int32)).to(DEV)
    return dev, pairs, f["feat"].shape[1], feat, count, x, ro


@pytest.mark.parametrize("preset", ["sweep", "search"])
def test_forward_within_tolerance(preset):
    # search sets (16 chains) take the forward kernel's one-tile path, sweep
    # sets (4-64 chains) mostly the multi-tile path
    dev, pairs, rs, feat, count, x, ro = _network_batch(preset)
    n = len(pairs)
    for seed, b2 in ((1, 0.05), (2, 0.0)):
        theta = chaingen.mlp_init(seed)
        theta[78080:78336] = b2
        net = _paam.Network(theta, device=DEV)
        out = torch.zeros(n, dtype=torch.float32, device=DEV)
        _paam.paam_mlp_forward(net.params, net.packed, feat, count, n, rs, out)
        torch.cuda.synchronize()
        y, cache = om.forward(theta.astype(np.float64), x, ro, quant=True)
        S = np.abs(cache["h2q"] * cache["w3"]).sum(axis=1) + abs(float(theta[-1]))
        err = np.abs(out.cpu().numpy() - y)
        assert np.all(err <= 2.0 ** -7 * S + 1e-6), (err.max(), S[np.argmax(err)])


def test_backward_and_adam_match_oracle():
    dev, pairs, rs, feat, count, x, ro = _network_batch()
    n = len(pairs)
    theta = chaingen.mlp_init(3)
    theta[78080:78336] = 0.05
    net = _paam.Network(theta, device=DEV)
    out = torch.zeros(n, dtype=torch.float32, device=DEV)
    act = torch.zeros(n * 512, dtype=torch.int16, device=DEV)
    _paam.paam_mlp_forward(net.params, net.packed, feat, count, n, rs, out, act)
    t = np.random.default_rng(4).uniform(0, 2, n).astype(np.float32)
    grad = torch.zeros(78593, dtype=torch.float32, device=DEV)
    loss = torch.zeros(1, dtype=torch.float32, device=DEV)
    ws = _paam.workspace(_paam.paam_mlp_backward_bytes(n), DEV)
    _paam.paam_mlp_backward(net.params, net.packed, feat, count, n, rs, out,
                            torch.from_numpy(t).to(DEV), act, grad, loss, ws)
    torch.cuda.synchronize()
    y, cache = om.forward(theta.astype(np.float64), x, ro, quant=True)
    gref = om.backward(theta.astype(np.float64), cache, y, t.astype(np.float64))
    ge = grad.cpu().numpy().astype(np.float64)
    for a, b in ((0, 12288), (12288, 12544), (12544, 78080), (78080, 78336), (78336, 78592),
                 (78592, 78593)):
        rel = np.linalg.norm(ge[a:b] - gref[a:b]) / max(np.linalg.norm(gref[a:b]), 1e-30)
        assert rel < 1e-3, (a, b, rel)
    assert abs(loss.item() - om.loss(y, t)) <= 1e-3 * om.loss(y, t)
    # two Adam steps against the float64 reference from the same gradient
    p0 = net.params.cpu().numpy().astype(np.float64)
    m = np.zeros(78593)
    v = np.zeros(78593)
    ref = p0
    for step in (1, 2):
        net.adam(grad, 1e-3)
        ref, m, v = om.adam(ref, m, v, ge, 1e-3, 0.9, 0.999, 1e-8, step)
    torch.cuda.synchronize()
    assert np.abs(net.params.cpu().numpy() - ref).max() < 1e-6
    pk = net.packed.cpu().numpy().view(np.uint16)
    P = net.params.cpu().numpy()
    exp = np.zeros(82176, np.uint16)
    exp[:16384].reshape(256, 64)[:, :48] = of.bf16_bits(of.bf16_round(P[:12288])).reshape(256, 48)
    exp[16384:81920] = of.bf16_bits(of.bf16_round(P[12544:78080]))
    exp[81920:] = of.bf16_bits(of.bf16_round(P[78336:78592]))
    assert np.array_equal(pk, exp)


MID = dict(chains=(65, 140), n_accel=3, max_seg_per_cb=2, n_buckets=5, eps=391_000,
           kappa=129_180, eps_hop=391_000, n_exec=5)


@pytest.mark.parametrize("preset,n_sets,n_cand", [("search", 12, 70), ("mid", 3, 150),
                                                   ("mixed", 4, 80)])
def test_score_candidates_equals_explicit_path(preset, n_sets, n_cand):
    # range mode walks each run of consecutive candidates one swap at a time
    # (updated inversion counts on sets of more than 64 chains, whose tables
    # are built once per set and shared by its runs); the explicit path
    # computes every pair from scratch
    if preset == "mid":
        params = chaingen.PRESETS["large"].replace(**MID)
    elif preset in VARIANTS:
        params = chaingen.PRESETS[VARIANTS[preset][0]].replace(**VARIANTS[preset][1])
    else:
        params = preset
    cs = chaingen.generate(params, n_sets)
    dev = _paam.Chainset(cs, device=DEV)
    net = _paam.Network(chaingen.mlp_init(5), device=DEV)
    sc = _paam.score(dev, net, n_cand, SEED).cpu().numpy()
    pairs = np.array([[s, k, 1000] for s in range(cs.n_sets) for k in range(n_cand)], np.int64)
    f = _paam.features(dev, pairs, SEED)
    feat = torch.from_numpy(f["feat"].reshape(-1).view(np.int16).copy()).to(DEV)
    count = torch.from_numpy(f["count"].astype(np.int32)).to(DEV)
    out = torch.zeros(len(pairs), dtype=torch.float32, device=DEV)
    _paam.paam_mlp_forward(net.params, net.packed, feat, count, len(pairs), f["feat"].shape[1], out)
    torch.cuda.synchronize()
    assert np.array_equal(sc[:len(pairs)], out.cpu().numpy())


def test_training_lowers_loss():
    cs = chaingen.generate("sweep", 400)
    dev = _paam.Chainset(cs, device=DEV)
    pairs_np = chaingen.training_pairs(cs.n_sets, 8192, 256, 11)
    pairs_np = np.concatenate([pairs_np, np.full((len(pairs_np), 1), 0, np.int64)], axis=1)
    pairs_np[:, 2] = np.array(chaingen.SWEEP_LEVELS)[np.arange(len(pairs_np)) % 18]
    pairs = torch.from_numpy(pairs_np).to(DEV)
    net = _paam.Network(chaingen.mlp_init(2), device=DEV)
    tr = Trainer(dev, net, SEED, batch=512)
    tg = tr.targets(pairs)
    torch.cuda.synchronize()
    # targets are the oracle's on a sample
    r = oracle.candidate_analysis(cs, pairs_np[:40], SEED, cap_mult=2)
    assert np.array_equal(tg.ratio[:40].cpu().numpy(), r["ratio"])
    losses = tr.fit(pairs, tg.ratio, epochs=4, lr=2e-3, order_seed=1)
    assert losses[-1] < 0.5 * losses[0], losses


def test_trained_network_gains_over_the_search_without_it():
    """What the learned ranking adds: trained on sweep-generator sets it
    ranks the candidate orders of unseen search sets so that confirming only
    its top 16 finds more schedulable sets than an untrained network's top 16
    or the first 16 candidates in index order, and nearly every set plain
    search over all 256 candidates finds."""
    from paper_2404_06452_amd import surrogate
    n_cand, top_k, seed, util = 256, 16, 2404, 50
    tcs = chaingen.generate("sweep", 20000)
    tdev = _paam.Chainset(tcs, device=DEV)
    net = _paam.Network(chaingen.mlp_init(seed), device=DEV)
    tr = Trainer(tdev, net, seed, batch=4096)
    pairs = torch.from_numpy(surrogate.recipe_pairs(tcs.n_sets, 2_000_000, seed)).to(DEV)
    target = tr.targets(pairs).ratio[:2_000_000]
    tr.fit(pairs, target, epochs=2, lr=2e-3, lr_final=1e-4, order_seed=seed)
    untrained = _paam.Network(chaingen.mlp_init(seed + 7), device=DEV)

    cs = chaingen.generate("search", 5000, set_begin=70000)
    dev = _paam.Chainset(cs, device=DEV)
    plain = _paam.search(dev, n_cand, seed, util_permille=util)["found"] >= 0
    first = _paam.search(dev, top_k, seed, util_permille=util)["found"] >= 0

    def guided(nw):
        sc = _paam.score(dev, nw, n_cand, seed, util_permille=util)
        g = _paam.search(dev, n_cand, seed, scores=sc, guided=True, top_k=top_k, fallback=False,
                         util_permille=util)
        assert (g["n_exact"] <= top_k).all()
        return g["found"] >= 0

    trained, untr = guided(net), guided(untrained)
    print("found: plain %d, first %d in index order %d, untrained top %d %d, trained top %d %d" % (
        plain.sum(), top_k, first.sum(), top_k, untr.sum(), top_k, trained.sum()), flush=True)
    assert not (trained & ~plain).any()  # a guided find is a plain find
    assert trained.sum() > untr.sum() and trained.sum() > first.sum()
    assert trained.sum() >= 0.95 * plain.sum()
