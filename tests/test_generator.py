"""The seeded input generator: determinism, random access and workload shape."""
import numpy as np

from paper_2404_06452_amd import chaingen


def test_deterministic_and_random_access():
    a = chaingen.generate("sweep", 300)
    b = chaingen.generate("sweep", 300)
    for k, v in vars(a).items():
        if isinstance(v, np.ndarray):
            assert np.array_equal(v, getattr(b, k)), k
    for s in (0, 17, 299):
        one = chaingen.generate("sweep", 1, set_begin=s)
        assert one.set_dict(0) == a.set_dict(s)


def test_shapes_follow_the_recipes():
    cs = chaingen.generate("small", 200)
    C = np.diff(cs.set_chain_off)
    assert np.all(C == 8)
    n = np.diff(cs.chain_cb_off)
    assert n.min() >= 2 and n.max() <= 5
    assert np.all((cs.exec >= 0) & (cs.exec < 2))
    assert np.all(cs.D == cs.T)
    assert cs.T.min() >= 10**7 and cs.T.max() <= 10**9
    util = np.zeros(cs.n_sets)
    for s in range(cs.n_sets):
        for c in range(cs.set_chain_off[s], cs.set_chain_off[s + 1]):
            j0, j1 = cs.chain_cb_off[c], cs.chain_cb_off[c + 1]
            W = cs.E[j0:j1].sum() + cs.A[cs.cb_seg_off[j0]:cs.cb_seg_off[j1]].sum()
            util[s] += W / cs.T[c]
    assert np.allclose(util, 0.5, atol=2e-3)
    frac_seg = cs.n_segments / cs.n_callbacks
    assert 0.25 < frac_seg < 0.35


def test_rate_monotonic_priorities():
    cs = chaingen.generate("sweep", 50)
    for s in range(cs.n_sets):
        c0, c1 = cs.set_chain_off[s], cs.set_chain_off[s + 1]
        pr, T = cs.prio[c0:c1], cs.T[c0:c1]
        assert sorted(pr.tolist()) == list(range(1, c1 - c0 + 1))
        order = np.argsort(-pr)
        assert np.all(np.diff(T[order]) >= 0)


def test_sweep_ranges():
    cs = chaingen.generate("sweep", 2000)
    C = np.diff(cs.set_chain_off)
    assert C.min() == 4 and C.max() == 64
    n = np.diff(cs.chain_cb_off)
    assert n.min() == 2 and n.max() == 12
    assert set(np.unique(cs.exec).tolist()) == {0, 1, 2, 3}
    assert cs.exec_core.tolist()[:4] == [0, 0, 1, 1]
    assert cs.exec_prio.tolist()[:4] == [4, 3, 2, 1]


def test_study_recipe_structure():
    """The analytical study's sets: 4 callbacks per chain, one segment each,
    accelerator share of each callback's WCET = the ratio (to rounding), each
    chain on its own executor alone on its core."""
    from paper_2404_06452_amd import chaingen
    for n, (acc, cpu) in ((1, (1, 1)), (8, (1, 9)), (8, (7, 3)), (16, (1, 1))):
        cs = chaingen.generate(chaingen.study_params(n, acc, cpu), 20)
        for s in range(cs.n_sets):
            d = cs.set_dict(s)
            assert len(d["chains"]) == n
            assert d["exec_core"] == list(range(n))
            for c, ch in enumerate(d["chains"]):
                assert len(ch["cbs"]) == 4
                for cb in ch["cbs"]:
                    assert cb["exec"] == c and len(cb["segs"]) == 1
                    A, W = cb["segs"][0][0], cb["E"] + cb["segs"][0][0]
                    assert abs(A - acc / (acc + cpu) * W) <= 1.0
