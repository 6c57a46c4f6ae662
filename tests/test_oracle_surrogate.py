"""Pins of the surrogate's oracle: features, bfloat16 rounding, network, Adam.

The features and the network are not in the paper (they rank candidate orders
for the exact analysis of Sec. IV-F), so they are pinned by a hand-derived
example, invariants, a floor that the exact analysis must respect, finite
differences, and library routines (torch's CPU bfloat16 cast, autograd and
Adam) that the oracle does not use.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest
import torch

import oracle
from oracle import features as of
from oracle import mlp as om
from paper_2404_06452_amd import chaingen

Q = 65536


def two_chain_set():
    # e0 and e1 share core 0, e0 has the higher process priority; one
    # accelerator, one bucket, no overheads.
    return {
        "chains": [
            {"T": 100, "D": 100, "prio": 2, "spin": 1,
             "cbs": [{"E": 10, "exec": 0, "segs": [(20, 0)]}, {"E": 5, "exec": 1, "segs": []}]},
            {"T": 200, "D": 200, "prio": 1, "spin": 0,
             "cbs": [{"E": 30, "exec": 0, "segs": []}, {"E": 10, "exec": 0, "segs": [(40, 0)]}]},
        ],
        "exec_core": [0, 0], "exec_prio": [2, 1],
        "accel_buckets": [1], "accel_eps": [0], "accel_kappa": [0], "eps_hop": 0,
    }


def _f(x):
    return float(x)


# Hand derivation, order (chain 0, chain 1).  q = floor(x * 65536 / T):
# q(0,e0) = floor(655360/100) = 6553, q(0,e1) = 3276, qa(0,e0) = 13107,
# q(1,e0) = floor(40*65536/200) = 13107, qa(1,e0) = 13107; qA(0) = qA(1) = 13107.
EXPECT = {
    0: {  # rank 0, runs e0 (E 10 + A 20), e1 (E 5)
        0: Fr(15, 100), 1: Fr(20, 100), 2: 0, 3: 0, 4: Fr(35, 100), 5: Fr(10, 100),
        6: Fr(2, 16), 7: Fr(1, 16), 8: Fr(2, 32), 9: 1, 10: 1, 11: Fr(100, 2**30), 12: 1,
        13: Fr(9829, Q), 14: Fr(13107, Q), 15: 0, 16: Fr(1, 2), 17: 1, 18: 0, 19: 0, 20: 0,
        21: 0, 22: 0, 23: 0, 24: 0, 25: 0,
        26: Fr(30, 100),       # LP blocking on e0: max E of chain 1 there = 30; e1: none
        27: Fr(50, 100),       # SAFE-like: callback E 10 + A* 40 = 50 on e0
        28: Fr(50, 100), 29: Fr(1, 2),
        30: Fr(80, 100),       # run on e1 preempted by e0: 2 * (E 40 of suspending chain 1)
        31: Fr(13107, Q), 32: 0, 33: 0,
        34: Fr(40, 100),       # same-bucket LP request of chain 1 (A* 40)
        35: 0, 36: 0, 37: 0,
        38: Fr(22936, 2 * Q), 39: Fr(19660, Q), 40: Fr(26214, Q), 41: Fr(2, 256),
        42: Fr(2, 8), 43: Fr(1, 8), 44: 1,
        45: Fr(205, 100),      # 35 own + 50 blocking + 80 hpp + 40 same-bucket
        47: Fr(35, 115),
    },
    1: {  # rank 1, one run on e0 (E 30, E 10 + A 40)
        0: Fr(40, 200), 1: Fr(40, 200), 2: 0, 3: 0, 4: Fr(80, 200), 5: Fr(30, 200),
        6: Fr(1, 16), 7: Fr(1, 16), 8: Fr(2, 32), 9: Fr(1, 2), 10: 1, 11: Fr(200, 2**30),
        12: 0, 13: Fr(13107, Q), 14: Fr(13107, Q), 15: Fr(1, 2), 16: 0, 17: 0, 18: 1,
        19: 0, 20: 0,
        21: Fr(6553, Q), 22: Fr(13107, Q),
        23: Fr(60, 200),       # 2 jobs of chain 0 on e0: 2 * (10 + 20)
        24: Fr(19660, Q), 25: Fr(1, 2), 26: 0, 27: 0, 28: 0, 29: 0, 30: 0, 31: 0,
        32: Fr(40, 200),       # 2 requests of chain 0 (A* 20) for the one sub-chain
        33: Fr(13107, Q), 34: 0, 35: 0, 36: Fr(1, 2), 37: 1,
        38: Fr(22936, 2 * Q), 39: Fr(19660, Q), 40: Fr(26214, Q), 41: Fr(2, 256),
        42: Fr(2, 8), 43: Fr(1, 8), 44: Fr(100, 200),
        45: Fr(180, 200),      # 80 own + 60 carry-in + 40 accelerator
        47: Fr(80, 115),
    },
}


def test_features_hand_example():
    F = of.chain_features(two_chain_set(), [0, 1])
    for c, exp in EXPECT.items():
        for k, v in exp.items():
            assert F[c, k] == _f(v), (c, k, of.NAMES[k], F[c, k], _f(v))
    # feature 46 = floor estimate + utilisation terms, two roundings and a sum
    assert F[0, 46] == _f(Fr(205, 100)) + 13107 / Q
    assert F[1, 46] == _f(Fr(180, 200)) + (6553 + 13107 + 13107) / Q


def _time_scaled(st, k):
    out = {key: (list(v) if isinstance(v, list) else v) for key, v in st.items()}
    out["chains"] = [{"T": ch["T"] * k, "D": ch["D"] * k, "prio": ch["prio"], "spin": ch["spin"],
                      "cbs": [{"E": cb["E"] * k, "exec": cb["exec"],
                               "segs": [(a * k, acc) for (a, acc) in cb["segs"]]}
                              for cb in ch["cbs"]]} for ch in st["chains"]]
    out["accel_eps"] = [e * k for e in st["accel_eps"]]
    out["accel_kappa"] = [e * k for e in st["accel_kappa"]]
    out["eps_hop"] = st["eps_hop"] * k
    return out


@pytest.mark.parametrize("preset", ["small", "small_overheads", "search"])
def test_features_invariants(preset):
    cs = chaingen.generate(preset, 4)
    rng = np.random.default_rng(7)
    static = [i for i in range(48) if i not in range(15, 38) and i not in (45, 46)]
    for s in range(cs.n_sets):
        st = cs.set_dict(s)
        C = len(st["chains"])
        order = list(rng.permutation(C))
        F = of.chain_features(st, order)
        # scaling every time by 7 leaves every ratio and every floor(x*2^16/T)
        # unchanged; only T itself (feature 11) scales
        F7 = of.chain_features(_time_scaled(st, 7), order)
        keep = [i for i in range(48) if i != 11]
        assert np.array_equal(F[:, keep], F7[:, keep])
        assert np.array_equal(F[:, 11] * 7, F7[:, 11])
        # relabelling the chains (carrying the order) permutes the rows
        perm = list(rng.permutation(C))          # new index i holds old chain perm[i]
        st2 = dict(st, chains=[st["chains"][p] for p in perm])
        inv = {old: new for new, old in enumerate(perm)}
        F2 = of.chain_features(st2, [inv[c] for c in order])
        assert np.array_equal(F2, F[perm])
        # order-independent features do not move with the order
        F3 = of.chain_features(st, list(rng.permutation(C)))
        assert np.array_equal(F3[:, static], F[:, static])
        # rank features
        rank = np.empty(C, int)
        rank[order] = np.arange(C)
        assert np.array_equal(F[:, 15], rank / C)
        assert F[:, 17].sum() == 1 and F[:, 18].sum() == 1


def test_features_lone_chain_is_closed_form():
    """A chain alone in its set: feature 4 (own demand / D) equals the exact
    bound over D, the closed form of the analysis for that case."""
    cs = chaingen.generate("small_overheads", 6)
    sets = []
    for s in range(cs.n_sets):
        st = cs.set_dict(s)
        sets.append(dict(st, chains=[dict(st["chains"][0], D=st["chains"][0]["T"])]))
    lone = chaingen.from_sets(sets)
    for s in range(lone.n_sets):
        r = oracle.analyse_set(lone, s, full=True, cap_mult=100)
        F = of.chain_features(lone.set_dict(s), [0])
        assert F[0, 4] == float(r["chain_R"][0]) / float(lone.D[s])
        assert F[0, 45] == F[0, 4]


@pytest.mark.parametrize("preset,u", [("small", 300), ("small_overheads", 200), ("search", 100),
                                      ("sweep", 150)])
def test_feature_floor_below_exact_bound(preset, u):
    """Feature 45 counts two jobs of every interfering chain per sub-chain,
    SAFE blocking and same-bucket blocking: each is a lower bound of the
    matching term of Theorem 1 at its fixed point (mu >= 2 for a positive
    window), so it never exceeds the exact bound over D."""
    cs = chaingen.generate(preset, 6)
    rng = np.random.default_rng(3)
    n = 0
    for s in range(cs.n_sets):
        st = cs.set_dict(s)
        C = len(st["chains"])
        for trial in range(2):
            order = list(rng.permutation(C)) if trial else list(
                np.argsort(-np.array([ch["prio"] for ch in st["chains"]]), kind="stable"))
            r = oracle.analyse_set(cs, s, order=np.array(order, np.int32), full=True,
                                   cap_mult=1000, util_permille=u)
            F = of.chain_features(st, order, util_permille=u)
            D = np.array([ch["D"] for ch in st["chains"]], np.float64)
            R = r["chain_R"]
            fin = R != oracle.INF
            assert np.all(F[fin, 45] <= R[fin].astype(np.float64) / D[fin])
            n += int(fin.sum())
    assert n > 0


def test_bf16_rounding_pins():
    one = 1.0
    assert of.bf16_round(np.float32(one)) == 1.0
    assert of.bf16_round(np.float32(1 + 2**-8)) == 1.0               # tie -> even (1.0)
    assert of.bf16_round(np.float32(1 + 3 * 2**-8)) == 1 + 2**-6     # tie -> even
    assert of.bf16_round(np.float32(1 + 2**-8 + 2**-20)) == 1 + 2**-7
    assert of.bf16_bits(of.bf16_round(np.float32(1 / 3))) == 0x3EAB
    x = np.random.default_rng(1).standard_normal(100000).astype(np.float32) * 10
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(of.bf16_round(x), ref)


def _tiny_batch(seed, n=5, quant=True):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(1, 7, n)
    ro = np.concatenate([[0], np.cumsum(sizes)])
    x = rng.uniform(0, 1.5, (ro[-1], 48))
    if quant:
        x = of.bf16_round(x.astype(np.float32))
    t = rng.uniform(0, 2, n)
    return x, ro, t


def test_mlp_forward_hand_network():
    """A network wired by hand: y = mean over rows of max(x[:, 0], 0) + 0.5."""
    W1 = np.zeros((256, 48)); W1[0, 0] = 1.0
    W2 = np.eye(256)
    w3 = np.zeros(256); w3[0] = 1.0
    theta = om.pack({"W1": W1, "b1": np.zeros(256), "W2": W2, "b2": np.zeros(256), "w3": w3,
                     "b3": np.array([0.5])})
    x = np.zeros((5, 48)); x[:, 0] = [0.25, -1.0, 0.75, 0.5, 2.0]
    y, _ = om.forward(theta, x, [0, 2, 5], quant=True)
    assert y[0] == 0.125 + 0.5                    # (0.25 + 0) / 2
    assert y[1] == float(of.bf16_round(np.float32(3.25 / 3))) + 0.5


def test_mlp_backward_matches_finite_differences():
    x, ro, t = _tiny_batch(2, quant=False)
    theta = chaingen.mlp_init(5).astype(np.float64) * 0.5
    theta[om.N_PARAMS - 1] = 0.1
    y, cache = om.forward(theta, x, ro, quant=False)
    g = om.backward(theta, cache, y, t)
    rng = np.random.default_rng(9)
    idx = np.concatenate([rng.choice(12288, 60, replace=False),
                          12288 + rng.choice(256, 20, replace=False),
                          12544 + rng.choice(65536, 60, replace=False),
                          78080 + rng.choice(513, 40, replace=False)])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (om.loss(om.forward(tp, x, ro, quant=False)[0], t)
              - om.loss(om.forward(tm, x, ro, quant=False)[0], t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_mlp_backward_matches_autograd():
    x, ro, t = _tiny_batch(4, n=9, quant=False)
    theta = chaingen.mlp_init(6).astype(np.float64)
    y, cache = om.forward(theta, x, ro, quant=False)
    g = om.backward(theta, cache, y, t)
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    P = {}
    o = 0
    for name, shape in om.SIZES:
        n = int(np.prod(shape))
        P[name] = th[o:o + n].reshape(shape)
        o += n
    xt = torch.tensor(x)
    h1 = torch.relu(xt @ P["W1"].T + P["b1"])
    p = torch.stack([h1[ro[i]:ro[i + 1]].mean(0) for i in range(len(ro) - 1)])
    h2 = torch.relu(p @ P["W2"].T + P["b2"])
    yt = h2 @ P["w3"] + P["b3"][0]
    assert np.allclose(yt.detach().numpy(), y, rtol=1e-12, atol=1e-12)
    torch.mean((yt - torch.tensor(t)) ** 2).backward()
    assert np.allclose(th.grad.numpy(), g, rtol=1e-9, atol=1e-12)


def test_adam_first_step_and_library():
    rng = np.random.default_rng(11)
    theta = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    t1, m, v = om.adam(theta, np.zeros(50), np.zeros(50), g, lr, b1, b2, eps, 1)
    # first step: bias corrections give m^ = g, v^ = g^2
    assert np.allclose(t1, theta - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    th = torch.tensor(theta, requires_grad=True)
    opt = torch.optim.Adam([th], lr=lr, betas=(b1, b2), eps=eps)
    cur, m, v = theta.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 8):
        gs = rng.standard_normal(50)
        th.grad = torch.tensor(gs)
        opt.step()
        cur, m, v = om.adam(cur, m, v, gs, lr, b1, b2, eps, step)
    assert np.allclose(th.detach().numpy(), cur, rtol=0, atol=1e-12)
