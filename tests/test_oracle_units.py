"""Pins of the oracle's binding of segments to accelerator units (Sec. IV-E).

The paper binds every callback/accelerator segment to one unit of its
accelerator type at registration with a bin-packing heuristic such as
worst-fit decreasing, and analyses each unit as an accelerator of its own.
Pins: hand-derived fixtures (tests/golden/units_*.json), Graham's bound for
largest-first list scheduling against a brute-force optimum, and invariances
the definition implies (one unit per type is the identity, chain order does
not matter, groups stay together, equal items spread evenly)."""
import glob
import itertools
import json
import os
import random

import numpy as np
import pytest

import oracle
from paper_2404_06452_amd import chaingen

UNITS_GOLDEN = sorted(glob.glob(os.path.join(os.path.dirname(__file__), "golden", "units_*.json")))


@pytest.mark.parametrize("path", UNITS_GOLDEN, ids=[os.path.basename(p)[:-5] for p in UNITS_GOLDEN])
def test_units_worked_example(path):
    fx = json.load(open(path))
    assert fx["cite"] and fx["derivation"]
    cs = chaingen.from_sets([fx["set"]])
    for case in fx["cases"]:
        su = oracle.wfd_units(cs, case["units"], case["group"])
        assert su.tolist() == case["seg_unit"], (fx["name"], case)
        if "chain_R" in case:
            sp = oracle.split_units(cs, case["units"], su)
            r = oracle.analyse_set(sp, 0, full=True)
            assert r["chain_R"].tolist() == case["chain_R"], (fx["name"], case)


def test_units_golden_inventory():
    assert len(UNITS_GOLDEN) >= 2


def _sizes(A, T):
    return [(a << 26) // t for a, t in zip(A, T)]


@pytest.mark.parametrize("m", [2, 3])
def test_largest_first_within_graham_bound(m):
    """Worst-fit decreasing on one type is largest-first list scheduling on
    identical units, whose largest load is at most (4/3 - 1/(3m)) of the
    optimum (Graham, 1969).  The optimum is found by brute force."""
    rng = random.Random(17 + m)
    for trial in range(60):
        n = rng.randint(m + 1, 7)
        T = [rng.choice([10, 20, 40, 100]) for _ in range(n)]
        A = [rng.randint(1, t) for t in T]
        st = {"chains": [{"T": T[i], "D": T[i], "prio": n - i, "spin": 0,
                          "cbs": [{"E": 1, "exec": 0, "segs": [[A[i], 0]]}]} for i in range(n)],
              "exec_core": [0], "exec_prio": [1], "accel_buckets": [1], "accel_eps": [0],
              "accel_kappa": [0], "eps_hop": 0}
        cs = chaingen.from_sets([st])
        su = oracle.wfd_units(cs, [m], oracle.UNITS_SEGMENT)
        assert su.min() >= 0 and su.max() < m
        size = _sizes(A, T)
        load = [0] * m
        for i, u in enumerate(su):
            load[u] += size[i]
        opt = min(max(sum(size[i] for i in range(n) if asg[i] == u) for u in range(m))
                  for asg in itertools.product(range(m), repeat=n))
        assert max(load) * 3 * m <= (4 * m - 1) * opt, (trial, A, T, su.tolist())


def test_one_unit_each_is_the_input():
    cs = chaingen.generate("small_overheads", 40)
    ones = np.ones(int(cs.set_accel_off[-1]), np.int16)
    for g in (oracle.UNITS_SEGMENT, oracle.UNITS_CALLBACK, oracle.UNITS_CHAIN):
        su = oracle.wfd_units(cs, ones, g)
        assert np.array_equal(su, cs.accel)
        sp = oracle.split_units(cs, ones, su)
        a, b = oracle.wcrt(cs, full=True), oracle.wcrt(sp, full=True)
        assert np.array_equal(a["chain_R"], b["chain_R"])


def _two_type_sets(n, seed):
    p = chaingen.PRESETS["small"].replace(seed=seed, n_accel=2, max_seg_per_cb=3, pseg=(0.8, 0.8))
    return chaingen.generate(p, n)


@pytest.mark.parametrize("group", [0, 1, 2])
def test_units_stay_within_their_type_and_groups_stay_together(group):
    cs = _two_type_sets(30, 99)
    units = np.array([3, 2] * cs.n_sets, np.int16)
    su = oracle.wfd_units(cs, units, group)
    for s in range(cs.n_sets):
        c0, c1 = int(cs.set_chain_off[s]), int(cs.set_chain_off[s + 1])
        for c in range(c0, c1):
            seen = {}
            for j in range(int(cs.chain_cb_off[c]), int(cs.chain_cb_off[c + 1])):
                seen_cb = {}
                for g in range(int(cs.cb_seg_off[j]), int(cs.cb_seg_off[j + 1])):
                    a, u = int(cs.accel[g]), int(su[g])
                    lo = 0 if a == 0 else 3
                    assert lo <= u < lo + (3 if a == 0 else 2)
                    if group == oracle.UNITS_CALLBACK:
                        assert seen_cb.setdefault(a, u) == u
                    if group == oracle.UNITS_CHAIN:
                        assert seen.setdefault(a, u) == u


@pytest.mark.parametrize("group", [0, 1, 2])
def test_chain_order_does_not_matter(group):
    """Placement depends on sizes and priorities, not on where a chain sits
    in the arrays."""
    cs = _two_type_sets(20, 5)
    units = np.array([2, 3] * cs.n_sets, np.int16)
    su = oracle.wfd_units(cs, units, group)
    for s in range(cs.n_sets):
        st = cs.set_dict(s)
        perm = list(range(len(st["chains"])))
        random.Random(s).shuffle(perm)
        st2 = dict(st, chains=[st["chains"][i] for i in perm])
        cs2 = chaingen.from_sets([st2])
        su2 = oracle.wfd_units(cs2, units[2 * s:2 * s + 2], group)
        # segments of chain perm[k] in cs2 are those of chain perm[k] in cs
        g_of = []
        for ch in range(len(st["chains"])):
            c = int(cs.set_chain_off[s]) + ch
            g_of.append(list(range(int(cs.cb_seg_off[int(cs.chain_cb_off[c])]),
                                   int(cs.cb_seg_off[int(cs.chain_cb_off[c + 1])]))))
        expect = [int(su[g]) for k in perm for g in g_of[k]]
        assert su2.tolist() == expect, s


def test_equal_items_spread_evenly():
    m, n = 3, 8
    st = {"chains": [{"T": 100, "D": 100, "prio": n - i, "spin": 0,
                      "cbs": [{"E": 1, "exec": 0, "segs": [[7, 0]]}]} for i in range(n)],
          "exec_core": [0], "exec_prio": [1], "accel_buckets": [1], "accel_eps": [0],
          "accel_kappa": [0], "eps_hop": 0}
    su = oracle.wfd_units(chaingen.from_sets([st]), [m], oracle.UNITS_SEGMENT)
    # highest priority first, each to the least-loaded (lowest on ties) unit
    assert su.tolist() == [0, 1, 2, 0, 1, 2, 0, 1]


def test_bad_unit_counts_are_rejected():
    cs = chaingen.generate("small", 2)
    with pytest.raises(ValueError):
        oracle.wfd_units(cs, np.zeros(int(cs.set_accel_off[-1]), np.int16))
    with pytest.raises(ValueError):
        oracle.wfd_units(cs, np.ones(int(cs.set_accel_off[-1]), np.int16), group=3)
