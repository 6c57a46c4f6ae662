"""The analysis entry point without a workspace argument (static scratch):
called through the C-ABI, its outputs equal paam_wcrt_batch's bit for bit,
on two calls in a row, the second with a smaller batch."""
import numpy as np
import pytest

from paper_2404_06452_amd import _paam, chaingen


def _run(dev, opts, entry):
    import torch
    out = _paam.WcrtOut(dev, bool(opts.full))
    for t in (out.set_sched, out.set_worst, out.set_worst_R):
        t.fill_(-7)
    if out.chain_R is not None:
        out.chain_R.fill_(-7)
    if entry == "noalloc":
        _paam.paam_wcrt_batch_noalloc(dev, opts, out)
    else:
        ws = _paam.workspace(_paam.paam_wcrt_bytes(dev, opts), dev.device)
        _paam.paam_wcrt_batch(dev, opts, out, ws)
    torch.cuda.synchronize()
    res = {"sched": out.set_sched.cpu().numpy(), "worst": out.set_worst.cpu().numpy(),
           "worst_R": out.set_worst_R.cpu().numpy()}
    if out.chain_R is not None:
        res["chain_R"] = out.chain_R.cpu().numpy()[:dev.n_chains]
    return res


@pytest.mark.gpu
def test_no_alloc_entry_point_matches_workspace_entry_point():
    # the second call analyses a smaller batch than the first: the shared
    # static scratch keeps the first call's contents
    for preset, n, util in (("sweep", 3000, 300), ("small_overheads", 400, 700)):
        cs = chaingen.generate(preset, n)
        dev = _paam.Chainset(cs, device="cuda:0")
        for full in (True, False):
            opts = _paam.wcrt_opts(full=full, util_permille=util)
            got = _run(dev, opts, "noalloc")
            ref = _run(dev, opts, "workspace")
            print("no-alloc check:", preset, n, "full" if full else "verdict", flush=True)
            for k in ref:
                assert np.array_equal(got[k], ref[k]), (preset, full, k)
        dev.free()
