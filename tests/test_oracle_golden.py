"""The oracle against hand-derived worked examples (tests/golden/*.json).

The paper prints no numeric example of its analysis, so every fixture is a
small set whose bounds were derived by hand from the equations of Sec. IV-F;
each file carries its citation and the derivation steps."""
import glob
import json
import os

import numpy as np
import pytest

import oracle
from paper_2404_06452_amd import chaingen

GOLDEN = sorted(glob.glob(os.path.join(os.path.dirname(__file__), "golden", "ex_*.json")))


def _val(v):
    return oracle.INF if v == "INF" else v


@pytest.mark.parametrize("path", GOLDEN, ids=[os.path.basename(p)[:-5] for p in GOLDEN])
def test_worked_example(path):
    fx = json.load(open(path))
    assert fx["cite"] and fx["derivation"]
    cs = chaingen.from_sets([fx["set"]])
    for case in fx["cases"]:
        opts = dict(case["opts"])
        opts["full"] = bool(opts.get("full", 1))
        r = oracle.analyse_set(cs, 0, **opts)
        if "chain_R" in case:
            assert r["chain_R"].tolist() == [_val(v) for v in case["chain_R"]], (fx["name"], opts)
        for key in ("sched", "worst", "worst_R"):
            if key in case:
                assert r[key] == _val(case[key]), (fx["name"], key, opts)
        if "seg_H" in case:
            H = oracle.segment_H(cs, 0, **{k: v for k, v in opts.items() if k != "full"})
            assert H.tolist() == case["seg_H"], fx["name"]


def test_golden_inventory():
    names = {os.path.basename(p) for p in GOLDEN}
    assert len(names) >= 15


def test_fixture_scale_invariance():
    """Every worked example scaled to nanoseconds of milliseconds (x 10^6)
    gives the bounds scaled by the same factor (all terms are homogeneous)."""
    for path in GOLDEN:
        fx = json.load(open(path))
        st = json.loads(json.dumps(fx["set"]))
        k = 1_000_000
        for ch in st["chains"]:
            ch["T"] *= k
            ch["D"] *= k
            for cb in ch["cbs"]:
                cb["E"] *= k
                cb["segs"] = [[a * k, i] for a, i in cb["segs"]]
        st["accel_eps"] = [e * k for e in st["accel_eps"]]
        st["accel_kappa"] = [e * k for e in st["accel_kappa"]]
        st["eps_hop"] *= k
        cs = chaingen.from_sets([st])
        for case in fx["cases"]:
            if "chain_R" not in case or case["opts"].get("util_permille", 1000) != 1000:
                continue  # the floor of the utilisation scaling is not homogeneous
            opts = dict(case["opts"])
            opts["full"] = bool(opts.get("full", 1))
            r = oracle.analyse_set(cs, 0, **opts)
            want = [oracle.INF if v == "INF" else v * k for v in case["chain_R"]]
            assert r["chain_R"].tolist() == want, fx["name"]
