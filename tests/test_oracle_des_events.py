"""Pins of the event-driven simulation oracle (oracle/paam_des.c).

It must observe exactly what the unit-step simulator (oracle/des.py, a
different formulation of the same model: one time unit per step, heaps for
the queues) observes on tiny random sets, every chain's largest response in
every scenario; the worked example Ex C (blocking by a callback that holds its
executor during its request) must show its response of 6; and every observed
response must stay within the analysis bound (Sec. V-A checks this on real
hardware)."""
import random

import numpy as np
import pytest

import oracle
import oracle.des as unit_step
from paper_2404_06452_amd import chaingen

from des_sets import tiny_set


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_events_equal_unit_steps(seed):
    rng = random.Random(seed)
    compared = observed = 0
    for _ in range(120):
        st = tiny_set(rng)
        cs = chaingen.from_sets([st])
        C, S, H = len(st["chains"]), 3, 200
        offs = [[0] * C] + [[rng.randrange(ch["T"]) for ch in st["chains"]] for _ in range(S - 1)]
        r = oracle.event_sim(cs, np.array(sum(offs, []), np.int64), S, H)
        for s in range(S):
            if r["status"][s] != 0:   # a chain fell two jobs behind: not compared
                continue
            ref = [-1 if v is None else v for v in unit_step.simulate(st, offs[s], H)]
            assert r["obs"][s * C:(s + 1) * C].tolist() == ref, (st, offs[s])
            compared += 1
            observed += sum(v >= 0 for v in ref)
    assert compared >= 250 and observed >= 600, (compared, observed)


def test_example_c_blocking_shows_six():
    st = {"chains": [{"T": 10, "D": 10, "prio": 2, "spin": 0, "cbs": [{"E": 1, "exec": 0, "segs": []}]},
                     {"T": 20, "D": 20, "prio": 1, "spin": 0,
                      "cbs": [{"E": 1, "exec": 0, "segs": [[5, 0]]}]}],
          "exec_core": [0], "exec_prio": [1], "accel_buckets": [1], "accel_eps": [0],
          "accel_kappa": [0], "eps_hop": 0}
    cs = chaingen.from_sets([st])
    r = oracle.event_sim(cs, np.array([1, 0], np.int64), 1, 40)
    assert r["status"].tolist() == [0]
    assert r["obs"][0] == 6            # above the printed bound 2, within the SAFE bound 7
    assert oracle.analyse_set(cs, 0, full=True)["chain_R"][0] == 7


def test_two_live_jobs_then_status_one():
    # one executor, a chain whose callback outlasts two periods of itself
    st = {"chains": [{"T": 10, "D": 10, "prio": 1, "spin": 0, "cbs": [{"E": 25, "exec": 0, "segs": []}]}],
          "exec_core": [0], "exec_prio": [1], "accel_buckets": [1], "accel_eps": [0],
          "accel_kappa": [0], "eps_hop": 0}
    r = oracle.event_sim(chaingen.from_sets([st]), np.array([0], np.int64), 1, 100)
    assert r["status"].tolist() == [1]


def test_actual_times_are_reproducible_and_bounded():
    cs = chaingen.generate("small", 20)
    S = 4
    rng = np.random.default_rng(0)
    offs = np.concatenate([np.stack([rng.integers(0, int(cs.T[c]), S) for c in range(
        int(cs.set_chain_off[s]), int(cs.set_chain_off[s + 1]))], 1).ravel() for s in range(20)])
    H = int(2 * cs.T.max())
    wcet = oracle.event_sim(cs, offs, S, H, util_permille=300)
    a = oracle.event_sim(cs, offs, S, H, exec_permille=500, seed=9, util_permille=300)
    b = oracle.event_sim(cs, offs, S, H, exec_permille=500, seed=9, util_permille=300)
    c = oracle.event_sim(cs, offs, S, H, exec_permille=1000, seed=123, util_permille=300)
    assert np.array_equal(a["obs"], b["obs"]) and np.array_equal(c["obs"], wcet["obs"])
    assert not np.array_equal(a["obs"], wcet["obs"])


def test_observed_within_bound_on_schedulable_sets():
    """Soundness: on sets the analysis admits, no scenario (synchronous,
    random offsets, random actual times) observes a response above a chain's
    bound."""
    cs = chaingen.generate(chaingen.study_params(4, 1, 1), 60)
    R = oracle.wcrt(cs, full=True)
    S = 6
    rng = np.random.default_rng(3)
    offs = []
    for s in range(cs.n_sets):
        c0, c1 = int(cs.set_chain_off[s]), int(cs.set_chain_off[s + 1])
        blk = np.stack([rng.integers(0, int(cs.T[c]), S) for c in range(c0, c1)], 1)
        blk[0] = 0
        offs.append(blk.ravel())
    H = int(3 * cs.T.max())
    checked = 0
    for ex in (1000, 300):
        r = oracle.event_sim(cs, np.concatenate(offs), S, H, exec_permille=ex, seed=5)
        for s in range(cs.n_sets):
            if R["sched"][s] != 1:
                continue
            c0, c1 = int(cs.set_chain_off[s]), int(cs.set_chain_off[s + 1])
            assert (r["status"][s * S:(s + 1) * S] == 0).all()
            blk = r["obs"][c0 * S:c1 * S].reshape(S, c1 - c0)
            assert (blk <= R["chain_R"][c0:c1]).all(), s
            checked += int((blk >= 0).sum())
    assert checked > 300
