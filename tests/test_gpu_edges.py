"""GPU parity at the edges of the input range (tests/edge_sets.py): periods
from 1 ns to just below 2^36 ns, times up to 2^36 - 1 ns, zero-length
callbacks and segments, cap_mult 64, util_permille 0 and 10^6, several
accelerators and buckets, many sub-chains.  The kernels hold times as integers
in fp64: every value a bound can reach below its cap is an integer below
2^53, the period quotient is exact for windows below 2^50 ns, and a sum whose
exact value passes the cap also passes it after rounding, so the results must
equal the oracle's int64 arithmetic bit for bit."""
import numpy as np
import pytest

import oracle
from edge_sets import edge_sets
from paper_2404_06452_amd import _paam, chaingen

OPTIONS = [
    {},
    {"cap_mult": 64},
    {"util_permille": 1000000},
    {"util_permille": 0},
    {"cap_mult": 64, "util_permille": 1000000},
    {"cap_mult": 2, "blocking": _paam.PAAM_BLOCK_PAPER, "bound": _paam.PAAM_BOUND_L3},
    {"bound": _paam.PAAM_BOUND_L2, "util_permille": 1},
]


@pytest.mark.gpu
@pytest.mark.parametrize("opt", range(len(OPTIONS)))
def test_edge_values_bit_exact(opt):
    kw = OPTIONS[opt]
    cs = chaingen.from_sets(edge_sets())
    dev = _paam.Chainset(cs, device="cuda:0")
    for full in (True, False):
        g = _paam.wcrt(dev, full=full, **kw)
        r = oracle.wcrt(cs, full=full, threads=8, **kw)
        print("edge sets", kw, "full" if full else "verdict", "schedulable",
              float((r["sched"] == 1).mean()), flush=True)
        for k in ("sched", "worst", "worst_R"):
            assert np.array_equal(g[k], r[k]), (kw, full, k)
        if full:
            assert np.array_equal(g["chain_R"], r["chain_R"]), (kw, k)
    dev.free()


@pytest.mark.gpu
def test_large_sets_thousand_bit_exact():
    """1,000 sets of the 256-chain workload (8 executors, 2-32 callbacks per
    chain), every chain's bound and the verdicts against the oracle."""
    cs = chaingen.generate("large", 1000)
    dev = _paam.Chainset(cs, device="cuda:0")
    for full in (True, False):
        g = _paam.wcrt(dev, full=full)
        r = oracle.wcrt(cs, full=full, threads=16)
        print("large sets, 1000:", "full" if full else "verdict", flush=True)
        for k in ("sched", "worst", "worst_R"):
            assert np.array_equal(g[k], r[k]), (full, k)
        if full:
            assert np.array_equal(g["chain_R"], r["chain_R"])
    dev.free()
