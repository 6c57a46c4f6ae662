"""Pins of oracle parts that the worked examples do not reach.

* The utilisation scaling of the sweep (the generator's reading of the
  workloads: every E and A becomes floor(x*u/1000), the platform overheads
  kappa, epsilon and the hop cost stay as they are): analysing at u equals
  analysing a copy whose E and A were floored on the host, on sets with
  non-zero overheads.  The worked example ex_k pins the same rule by hand.
* The candidate walk: SplitMix64 [Steele, Lea & Flood 2014] re-implemented
  here from its published definition and checked against its published
  reference outputs, then the oracle's walk against swaps drawn from it.
* The guided-search order: the oracle's score order against numpy's lexsort
  over an independent key (IEEE total order through the float32 bit pattern).
"""
import numpy as np
import pytest

import oracle
from paper_2404_06452_amd import chaingen

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def sm64_mix(z):
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def sm64_stream(state, n):
    out = []
    for _ in range(n):
        state = (state + GAMMA) & MASK
        out.append(sm64_mix(state))
    return out


def test_splitmix64_reference_outputs():
    # the first outputs of SplitMix64 started from state 0, as published with
    # the generator's reference code
    assert sm64_stream(0, 4) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F,
                                 0xF88BB8A8724C81EC]


def walk_by_definition(C, seed, s, n_steps, base):
    """Candidate orders 0..n_steps of set s: candidate k swaps positions
    i = u1 mod C and j = (i + 1 + u2 mod (C-1)) mod C of candidate k-1, u1 and
    u2 the outputs 2k-2 and 2k-1 of the set's stream, whose state starts at
    the first output of SplitMix64 from seed + GAMMA*s."""
    state = sm64_stream((seed + GAMMA * s) & MASK, 1)[0]
    u = sm64_stream(state, 2 * n_steps)
    order = list(base)
    orders = [list(order)]
    for k in range(1, n_steps + 1):
        if C >= 2:
            i = u[2 * k - 2] % C
            j = (i + 1 + u[2 * k - 1] % (C - 1)) % C
            order[i], order[j] = order[j], order[i]
        orders.append(list(order))
    return orders


@pytest.mark.parametrize("preset,n,seed", [("small", 6, 7), ("search", 4, 2404064522),
                                           ("sweep", 5, 123456789123)])
def test_candidate_walk_matches_splitmix64(preset, n, seed):
    cs = chaingen.generate(preset, n)
    for s in range(n):
        c0, c1 = int(cs.set_chain_off[s]), int(cs.set_chain_off[s + 1])
        C = c1 - c0
        base = oracle.candidate_order(cs, s, seed, 0).tolist()
        # candidate 0: chains by decreasing priority
        assert base == sorted(range(C), key=lambda c: -int(cs.prio[c0 + c]))
        want = walk_by_definition(C, seed, s, 12, base)
        for k in range(13):
            assert oracle.candidate_order(cs, s, seed, k).tolist() == want[k], (preset, s, k)


def test_candidate_walk_two_chains_alternates():
    # with two chains every step swaps the only pair: the order alternates
    st = {"chains": [{"T": 10, "D": 10, "spin": 0, "prio": 2, "cbs": [{"E": 1, "exec": 0,
                                                                       "segs": []}]},
                     {"T": 20, "D": 20, "spin": 0, "prio": 1, "cbs": [{"E": 1, "exec": 0,
                                                                       "segs": []}]}],
          "exec_core": [0], "exec_prio": [1], "accel_buckets": [1], "accel_eps": [0],
          "accel_kappa": [0], "eps_hop": 0}
    cs = chaingen.from_sets([st])
    for k in range(6):
        assert oracle.candidate_order(cs, 0, 99, k).tolist() == ([0, 1] if k % 2 == 0 else [1, 0])


def host_floor(cs, u):
    out = cs.subset(range(cs.n_sets))
    out.E = (np.asarray(cs.E, np.int64) * u) // 1000
    out.A = (np.asarray(cs.A, np.int64) * u) // 1000
    return out


@pytest.mark.parametrize("u", [1, 333, 500, 777, 999, 1001, 2500])
def test_utilisation_scaling_is_host_floor_of_E_and_A(u):
    cs = chaingen.generate("small_overheads", 40)
    assert int(cs.accel_kappa.max()) > 0 and int(cs.accel_eps.max()) > 0
    assert int(cs.eps_hop.max()) > 0
    ref = host_floor(cs, u)
    for full in (True, False):
        a = oracle.wcrt(cs, util_permille=u, full=full, cap_mult=2)
        b = oracle.wcrt(ref, util_permille=1000, full=full, cap_mult=2)
        for k in ("sched", "worst", "worst_R", "chain_R"):
            assert np.array_equal(a[k], b[k]), (u, full, k)


def test_utilisation_scaling_leaves_overheads_unscaled():
    # scaling the overheads as well would change the bounds of these sets
    cs = chaingen.generate("small_overheads", 40)
    u = 500
    ref = host_floor(cs, u)
    wrong = host_floor(cs, u)
    wrong.accel_kappa = (np.asarray(cs.accel_kappa) * u) // 1000
    wrong.accel_eps = (np.asarray(cs.accel_eps) * u) // 1000
    wrong.eps_hop = (np.asarray(cs.eps_hop) * u) // 1000
    a = oracle.wcrt(cs, util_permille=u, full=True, cap_mult=2)
    assert np.array_equal(a["chain_R"], oracle.wcrt(ref, full=True, cap_mult=2)["chain_R"])
    assert not np.array_equal(a["chain_R"], oracle.wcrt(wrong, full=True, cap_mult=2)["chain_R"])


def total_order_key(x):
    b = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    neg = (b >> 31) == 1
    return np.where(neg, 0xFFFFFFFF - b, b | 0x80000000)


@pytest.mark.parametrize("seed", range(6))
def test_score_order_matches_lexsort(seed):
    rng = np.random.default_rng(seed)
    n = 300
    v = rng.normal(size=n).astype(np.float32)
    pool = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, -np.nan, 1.5, -1.5], np.float32)
    pick = rng.random(n) < 0.35
    v[pick] = pool[rng.integers(0, len(pool), pick.sum())]
    v[rng.integers(0, n, 20)] = v[rng.integers(0, n, 20)]  # ties
    isnan = np.isnan(v)
    key = np.where(isnan, 0, total_order_key(v))
    want = np.lexsort((np.arange(n), key, isnan.astype(np.int8))).tolist()
    assert oracle.score_order(v) == want
