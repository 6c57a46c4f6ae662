"""The batched simulation kernel (paam_des_batch) against the event-driven
simulation oracle, scenario by scenario and chain by chain (bit-exact), and
the property the paper's Case Study 1 checks (Sec. V-A): on sets the analysis
admits, no observed end-to-end latency exceeds the chain's bound."""
import random

import numpy as np
import pytest

import oracle
from paper_2404_06452_amd import _paam, chaingen

from des_sets import tiny_set


def _parity(cs, n_scen, horizon, label, units=None, **kw):
    print("des case", label, "sets", cs.n_sets, "scenarios", n_scen, flush=True)
    offs = chaingen.release_offsets(cs, n_scen, 7)
    dev = _paam.Chainset(cs, device="cuda:0", units=units, unit_group=_paam.PAAM_UNITS_CHAIN)
    g = _paam.simulate(dev, offs, n_scen, horizon, **kw)
    ref_cs = cs
    if units is not None:
        ref_cs = oracle.split_units(cs, units, dev.seg_units().cpu().numpy())
    dev.free()
    r = oracle.event_sim(ref_cs, offs, n_scen, horizon, threads=8, **kw)
    assert np.array_equal(g["status"], r["status"]), label
    bad = np.flatnonzero(g["obs"] != r["obs"])
    assert bad.size == 0, (label, bad[:8], g["obs"][bad[:8]], r["obs"][bad[:8]])
    return g, offs


@pytest.mark.gpu
def test_des_tiny_random_sets():
    rng = random.Random(11)
    cs = chaingen.from_sets([tiny_set(rng) for _ in range(400)])
    g, _ = _parity(cs, 8, 300, "tiny random")
    assert (g["status"] == 0).mean() > 0.5 and (g["obs"] >= 0).sum() > 1000


@pytest.mark.gpu
@pytest.mark.parametrize("exec_permille", [1000, 400])
def test_des_small_sets_with_overheads(exec_permille):
    cs = chaingen.generate("small_overheads", 60)
    horizon = int(3 * cs.T.max())
    g, _ = _parity(cs, 64, horizon, "small_overheads", exec_permille=exec_permille, seed=3,
                   util_permille=250)
    assert (g["obs"] >= 0).mean() > 0.5


@pytest.mark.gpu
def test_des_two_accelerators_units_and_hops():
    p = chaingen.PRESETS["small_overheads"].replace(seed=77, n_accel=2, max_seg_per_cb=3,
                                                   pseg=(0.6, 0.6))
    cs = chaingen.generate(p, 40)
    units = np.array([2, 1] * cs.n_sets, np.int16)
    _parity(cs, 32, int(2 * cs.T.max()), "two types, units", units=units, util_permille=200,
            exec_permille=700, seed=21)


@pytest.mark.gpu
def test_des_step_limit_and_empty_horizon():
    cs = chaingen.generate("small", 20)
    _parity(cs, 16, int(cs.T.max()), "step limit", max_steps=50)
    _parity(cs, 4, 0, "horizon 0")


@pytest.mark.gpu
def test_des_observed_within_bound_at_scale():
    """Sec. V-A at scale: the study's 8-chain sets, 64 scenarios each
    (synchronous release, random offsets, half with random actual times);
    every observed latency of an admitted set stays within its bound, and
    the GPU agrees with the oracle on a sample of the sets."""
    cs = chaingen.generate(chaingen.study_params(8, 1, 1), 500)
    R = oracle.wcrt(cs, full=True, threads=8)
    n_scen, horizon = 64, int(2 * cs.T.max())
    offs = chaingen.release_offsets(cs, n_scen, 5)
    dev = _paam.Chainset(cs, device="cuda:0")
    for ex in (1000, 500):
        g = _paam.simulate(dev, offs, n_scen, horizon, exec_permille=ex, seed=99)
        checked = 0
        for s in np.flatnonzero(R["sched"] == 1):
            c0, c1 = int(cs.set_chain_off[s]), int(cs.set_chain_off[s + 1])
            assert (g["status"][s * n_scen:(s + 1) * n_scen] == 0).all(), s
            blk = g["obs"][c0 * n_scen:c1 * n_scen].reshape(n_scen, c1 - c0)
            assert (blk <= R["chain_R"][c0:c1]).all(), s
            checked += int((blk >= 0).sum())
        assert checked > 10000
        sub = cs.subset(range(40))
        r = oracle.event_sim(sub, offs[:int(sub.set_chain_off[-1]) * n_scen], n_scen, horizon,
                             exec_permille=ex, seed=99, threads=8)
        n = int(sub.set_chain_off[-1]) * n_scen
        assert np.array_equal(g["obs"][:n], r["obs"]), ex
    dev.free()


@pytest.mark.gpu
def test_des_rejects_sets_beyond_its_limits():
    cs = chaingen.generate(chaingen.PRESETS["small"].replace(chains=(40, 40)), 2)
    dev = _paam.Chainset(cs, device="cuda:0")
    with pytest.raises(_paam.PaamError):
        _paam.simulate(dev, np.zeros(cs.n_chains * 2, np.int64), 2, 1000)
    dev.free()
    cs = chaingen.generate("small", 2)
    dev = _paam.Chainset(cs, device="cuda:0")
    with pytest.raises(_paam.PaamError):
        _paam.simulate(dev, np.zeros(cs.n_chains, np.int64), 1, 1 << 41)
    dev.free()
    # 8 chains of 600 callbacks: the set's tables exceed the 48 KB staged in LDS
    cs = chaingen.generate(chaingen.PRESETS["small"].replace(cbs=(600, 600)), 1)
    dev = _paam.Chainset(cs, device="cuda:0")
    with pytest.raises(_paam.PaamError):
        _paam.simulate(dev, np.zeros(cs.n_chains, np.int64), 1, 1000)
    dev.free()


@pytest.mark.gpu
def test_des_at_its_limits():
    """32 chains, 16 executors (pairs sharing cores), 8 segments per callback,
    two accelerators with 8 buckets each: the largest sets the kernel takes."""
    rng = random.Random(5)
    sets = []
    for _ in range(12):
        X = 16
        chains = []
        for c in range(32):
            T = rng.choice([200, 300, 500, 800, 1000, 2000]) * 1000
            cbs = [{"E": rng.randint(0, 3000), "exec": rng.randrange(X),
                    "segs": [[rng.randint(0, 2000), rng.randrange(2)] for _ in range(rng.randint(0, 8))]}
                   for _ in range(rng.randint(1, 4))]
            chains.append({"T": T, "D": T, "prio": 100 - c, "spin": rng.randint(0, 1), "cbs": cbs})
        sets.append({"chains": chains, "exec_core": [e // 2 for e in range(X)],
                     "exec_prio": [2 - (e % 2) for e in range(X)], "accel_buckets": [8, 8],
                     "accel_eps": [100, 50], "accel_kappa": [10, 0], "eps_hop": 30})
    cs = chaingen.from_sets(sets)
    g, _ = _parity(cs, 64, 6_000_000, "limits", util_permille=200, exec_permille=600, seed=8)
    assert (g["obs"] >= 0).sum() > 1000
