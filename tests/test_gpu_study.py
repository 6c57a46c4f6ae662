"""The analytical study of Sec. V (schedulability against the number of chains
and against the accelerator : CPU utilisation ratio) on the batched analysis:
every set of the tested points bit-exact against the oracle, and the trend the
paper states (schedulability falls as chains are added and as the accelerator
share grows)."""
import numpy as np
import pytest

import oracle
from paper_2404_06452_amd import _paam, chaingen

N = 1000


def _point(n_chains, acc, cpu):
    cs = chaingen.generate(chaingen.study_params(n_chains, acc, cpu), N)
    dev = _paam.Chainset(cs, device="cuda:0")
    g = _paam.wcrt(dev, full=True)
    dev.free()
    r = oracle.wcrt(cs, full=True, threads=8)
    for k in ("sched", "worst", "worst_R", "chain_R"):
        assert np.array_equal(g[k], r[k]), (n_chains, acc, cpu, k)
    print("study point", n_chains, "chains", "%d:%d" % (acc, cpu), "schedulable",
          float((g["sched"] == 1).mean()), flush=True)
    return float((g["sched"] == 1).mean())


@pytest.mark.gpu
def test_study_by_number_of_chains():
    fr = [_point(c, 1, 1) for c in (1, 4, 8, 16)]
    assert fr[0] == 1.0  # a chain alone meets its deadline at 5 % utilisation
    assert all(b <= a for a, b in zip(fr, fr[1:])), fr
    assert fr[-1] < fr[0] - 0.5, fr


@pytest.mark.gpu
def test_study_by_accelerator_share():
    fr = [_point(chaingen.STUDY_RATIO_CHAINS, a, c) for a, c in ((1, 9), (5, 5), (7, 3))]
    assert all(b <= a for a, b in zip(fr, fr[1:])), fr
    assert fr[-1] < fr[0] - 0.3, fr
