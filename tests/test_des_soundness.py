"""Brute-force soundness pin: simulated response times never exceed the bound.

The paper validates its analysis by observing that measured chain latencies
stay below the analytical bound (Sec. V-A).  Here a discrete-event simulator
(oracle/des.py) plays tiny random sets under many release offsets and
execution-time patterns; for every set the oracle calls schedulable, each
chain's largest observed response must be within its bound.  A dropped
interference or blocking term in the oracle shows up as a violation."""
import random

import pytest

import oracle
from oracle import des
from paper_2404_06452_amd import chaingen

PERIODS = [8, 12, 16, 24, 48]


def tiny_set(rng, n_exec_max=3, two_buckets=True, overheads=True):
    C = rng.randint(2, 4)
    X = rng.randint(1, n_exec_max)
    cores = [rng.randint(0, max(0, X - 2)) for _ in range(X)]
    chains = []
    for i in range(C):
        T = rng.choice(PERIODS)
        cbs = []
        for _ in range(rng.randint(1, 3)):
            segs = [(rng.randint(0, 3), 0)] if rng.random() < 0.5 else []
            if segs and rng.random() < 0.2:
                segs.append((rng.randint(0, 2), 0))
            cbs.append({"E": rng.randint(0, 2), "exec": rng.randrange(X), "segs": segs})
        chains.append({"T": T, "D": T, "prio": 0, "spin": rng.randint(0, 1), "cbs": cbs})
    for p, i in enumerate(rng.sample(range(C), C)):
        chains[i]["prio"] = p + 1
    # unique process priority per core
    eprio = list(range(1, X + 1))
    rng.shuffle(eprio)
    return {"chains": chains, "exec_core": cores, "exec_prio": eprio,
            "accel_buckets": [rng.choice([1, 2]) if two_buckets else 1],
            "accel_eps": [rng.randint(0, 1) if overheads else 0],
            "accel_kappa": [rng.randint(0, 1) if overheads else 0],
            "eps_hop": rng.randint(0, 1) if overheads else 0}


def check_sets(seed, n_sets, blocking=0, expect_sound=True, **kw):
    """Returns (sets checked, violations found)."""
    rng = random.Random(seed)
    checked = violations = 0
    for k in range(n_sets):
        st = tiny_set(rng, **kw)
        cs = chaingen.from_sets([st])
        r = oracle.analyse_set(cs, 0, full=True, blocking=blocking)
        if not r["sched"]:
            continue
        seen = des.observe(st, scenarios=12, seed=seed * 1000 + k)
        for c, (obs, bound) in enumerate(zip(seen, r["chain_R"].tolist())):
            if expect_sound:
                assert obs <= bound, ("set", k, "chain", c, "observed", obs, "bound", bound, st)
            violations += obs > bound
        checked += 1
    return checked, violations


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_observed_within_bound(seed):
    assert check_sets(seed, 300)[0] >= 40


def test_observed_within_bound_single_core_no_overheads():
    assert check_sets(11, 300, n_exec_max=2, two_buckets=False, overheads=False)[0] >= 50


def test_simulator_catches_a_dropped_term():
    """The pin has power: with the blocking term reduced to E_j (dropping the
    blocking callback's accelerator handling), random sets expose observed
    responses above the bound."""
    checked, violations = check_sets(21, 400, blocking=1, expect_sound=False,
                                     overheads=False, two_buckets=False)
    assert checked >= 40 and violations >= 1


def test_counterexample_to_execution_only_blocking():
    """Ex C: chain 2's callback holds the only executor while its 5-unit
    request runs; chain 1, released one unit later, responds in 6, above the
    bound 2 given by blocking = E_j alone, within the bound 7 that counts the
    blocking callback's accelerator handling."""
    st = {"chains": [{"T": 10, "D": 10, "prio": 2, "spin": 0, "cbs": [{"E": 1, "exec": 0, "segs": []}]},
                     {"T": 20, "D": 20, "prio": 1, "spin": 0, "cbs": [{"E": 1, "exec": 0, "segs": [(5, 0)]}]}],
          "exec_core": [0], "exec_prio": [1]}
    worst = des.simulate(st, [1, 0], horizon=60)
    assert worst[0] == 6
    cs = chaingen.from_sets([st])
    assert oracle.analyse_set(cs, 0, full=True, blocking=1)["chain_R"][0] == 2
    assert oracle.analyse_set(cs, 0, full=True, blocking=0)["chain_R"][0] == 7


def test_simulator_basics():
    # one chain alone: response = its demand; a preempting executor adds its load
    st = {"chains": [{"T": 20, "D": 20, "prio": 1, "spin": 0,
                      "cbs": [{"E": 3, "exec": 0, "segs": [(4, 0)]}]}],
          "exec_core": [0], "exec_prio": [1], "accel_eps": [1], "accel_kappa": [1]}
    assert des.simulate(st, [0], horizon=40) == [3 + 1 + 4 + 2]
    st2 = {"chains": [{"T": 20, "D": 20, "prio": 1, "spin": 1,
                       "cbs": [{"E": 2, "exec": 1, "segs": [(3, 0)]}]},
                      {"T": 40, "D": 40, "prio": 2, "spin": 0,
                       "cbs": [{"E": 4, "exec": 0, "segs": []}]}],
           "exec_core": [0, 0], "exec_prio": [2, 1]}
    # chain 0 sits on the lower process priority executor e1 and waits for
    # chain 1's 4 units on e0; with the priorities swapped it runs at once
    assert des.simulate(st2, [0, 0], horizon=40)[0] == 4 + 2 + 3
    st2["exec_prio"] = [1, 2]
    assert des.simulate(st2, [0, 0], horizon=40)[0] == 2 + 3
