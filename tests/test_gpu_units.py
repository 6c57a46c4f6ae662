"""Several units of one accelerator type (Sec. IV-E) on the GPU: the unit
binding the device computes at upload equals the oracle's worst-fit
decreasing binding segment by segment, and the analysis and the priority
search of the bound batch equal the oracle's on the batch whose accelerators
are the oracle's units."""
import glob
import json
import os

import numpy as np
import pytest

import oracle
from paper_2404_06452_amd import _paam, chaingen

GOLDEN = sorted(glob.glob(os.path.join(os.path.dirname(__file__), "golden", "units_*.json")))


def _check(cs, units, group, label, search=False):
    print("units case", label, "group", group, "sets", cs.n_sets, flush=True)
    dev = _paam.Chainset(cs, device="cuda:0", units=units, unit_group=group)
    su = dev.seg_units().cpu().numpy()
    ref = oracle.wfd_units(cs, units, group)
    assert np.array_equal(su, ref), (label, group, np.flatnonzero(su != ref)[:10])
    dev.assign_units()
    assert np.array_equal(dev.seg_units().cpu().numpy(), ref), (label, "rerun")
    sp = oracle.split_units(cs, units, ref)
    g = _paam.wcrt(dev, full=True)
    r = oracle.wcrt(sp, full=True, threads=8)
    for k in ("sched", "worst", "worst_R", "chain_R"):
        assert np.array_equal(g[k], r[k]), (label, group, k)
    if search:
        gs = _paam.search(dev, 16, 11, util_permille=400)
        rs = oracle.search(sp, 16, 11, util_permille=400, threads=8)
        assert np.array_equal(gs["found"], rs["found"]), (label, group)
        assert np.array_equal(gs["n_exact"], rs["n_eval"]), (label, group)
    dev.free()
    return float((g["sched"] == 1).mean())


@pytest.mark.gpu
@pytest.mark.parametrize("path", GOLDEN, ids=[os.path.basename(p)[:-5] for p in GOLDEN])
def test_units_worked_examples_on_gpu(path):
    fx = json.load(open(path))
    cs = chaingen.from_sets([fx["set"]])
    for case in fx["cases"]:
        dev = _paam.Chainset(cs, device="cuda:0", units=case["units"], unit_group=case["group"])
        assert dev.seg_units().cpu().numpy().tolist() == case["seg_unit"], (fx["name"], case)
        if "chain_R" in case:
            assert _paam.wcrt(dev, full=True)["chain_R"].tolist() == case["chain_R"]
        dev.free()


@pytest.mark.gpu
@pytest.mark.parametrize("group", [0, 1, 2])
def test_units_on_study_sets(group):
    cs = chaingen.generate(chaingen.study_params(8, 7, 3), 500)
    fr = []
    for k in (1, 2, 4):
        units = np.full(int(cs.set_accel_off[-1]), k, np.int16)
        fr.append(_check(cs, units, group, "study 8 chains 7:3, %d units" % k))
    if group == 2:  # whole chains on their own units: fewer sets miss
        assert fr[0] < fr[1] < fr[2], fr


@pytest.mark.gpu
@pytest.mark.parametrize("group", [0, 1, 2])
def test_units_on_two_types_with_several_segments_per_callback(group):
    p = chaingen.PRESETS["small_overheads"].replace(seed=4242, n_accel=2, max_seg_per_cb=3,
                                                   pseg=(0.8, 0.8))
    cs = chaingen.generate(p, 400)
    rng = np.random.default_rng(group)
    units = np.empty(int(cs.set_accel_off[-1]), np.int16)
    for s in range(cs.n_sets):  # 1..4 units per type, mixed per set
        a0 = int(cs.set_accel_off[s])
        units[a0:a0 + 2] = rng.integers(1, 5, 2)
    _check(cs, units, group, "two types, mixed units", search=True)


@pytest.mark.gpu
def test_units_on_sweep_sets():
    cs = chaingen.generate("sweep", 600)
    units = np.full(int(cs.set_accel_off[-1]), 3, np.int16)
    for group in (0, 2):
        _check(cs, units, group, "sweep, 3 units")


@pytest.mark.gpu
def test_units_equal_sizes_and_empty_sets():
    # equal utilisations everywhere (ties decided by priority, then segment
    # order) and sets without segments
    st = {"chains": [{"T": 1000, "D": 1000, "prio": 10 - i, "spin": i % 2,
                      "cbs": [{"E": 5, "exec": i % 2, "segs": [[50, 0], [50, 0]]}]}
                     for i in range(10)],
          "exec_core": [0, 1], "exec_prio": [1, 1], "accel_buckets": [2], "accel_eps": [3],
          "accel_kappa": [1], "eps_hop": 0}
    empty = {"chains": [{"T": 100, "D": 100, "prio": 1, "spin": 0,
                         "cbs": [{"E": 5, "exec": 0, "segs": []}]}],
             "exec_core": [0], "exec_prio": [1], "accel_buckets": [1], "accel_eps": [0],
             "accel_kappa": [0], "eps_hop": 0}
    cs = chaingen.from_sets([st, empty, st])
    for group in (0, 1, 2):
        _check(cs, np.array([3, 1, 3], np.int16), group, "equal sizes")


@pytest.mark.gpu
def test_units_rejected_without_binding():
    cs = chaingen.generate("small", 4)
    dev = _paam.Chainset(cs, device="cuda:0")
    with pytest.raises(_paam.PaamError):
        dev.assign_units()
    assert np.array_equal(dev.seg_units().cpu().numpy(), cs.accel)
    dev.free()


@pytest.mark.gpu
def test_units_at_their_limits():
    # 2,000 segments per set (the limit is 2,048) over eight units in all
    p = chaingen.PRESETS["small"].replace(seed=31, chains=(200, 200), cbs=(10, 10), n_exec=4,
                                          pseg=(1.0, 1.0), n_accel=2, util=(0.3, 0.3))
    cs = chaingen.generate(p, 3)
    assert max(int(cs.cb_seg_off[cs.chain_cb_off[cs.set_chain_off[s + 1]]] -
                   cs.cb_seg_off[cs.chain_cb_off[cs.set_chain_off[s]]]) for s in range(3)) <= 2048
    for group in (0, 2):
        _check(cs, np.array([5, 3] * cs.n_sets, np.int16), group, "2,000 segments, 8 units")
