"""Resuming training from a checkpoint gives the network of the
uninterrupted run, bit for bit (the training kernels are deterministic: fixed
reduction order, no atomics on the gradient)."""
import numpy as np
import pytest
import torch

from paper_2404_06452_amd import _paam, chaingen, surrogate


@pytest.mark.gpu
def test_resume_equals_uninterrupted(tmp_path):
    cs = chaingen.generate("sweep", 2000)
    dev = _paam.Chainset(cs, device="cuda:0")
    pairs = torch.from_numpy(surrogate.recipe_pairs(cs.n_sets, 12000, 5)).cuda()
    w0 = chaingen.mlp_init(9)

    net_a = _paam.Network(w0, device="cuda:0")
    tr_a = surrogate.Trainer(dev, net_a, 5)
    tg = tr_a.targets(pairs).ratio
    loss_a = tr_a.fit(pairs, tg, 3, 2e-3, 17, lr_final=2e-4)

    path = str(tmp_path / "ck.safetensors")
    net_b = _paam.Network(w0, device="cuda:0")
    tr_b = surrogate.Trainer(dev, net_b, 5)
    loss_b = tr_b.fit(pairs, tg, 3, 2e-3, 17, lr_final=2e-4, stop_epoch=1, checkpoint=path)
    # the schedule of a 3-epoch run, interrupted after epoch 1: rebuild it from the file
    net_c, ep = surrogate.load_checkpoint(path, device="cuda:0")
    assert ep == 1 and net_c.step == net_b.step
    tr_c = surrogate.Trainer(dev, net_c, 5)
    loss_c = tr_c.fit(pairs, tg, 3, 2e-3, 17, lr_final=2e-4, start_epoch=1)
    torch.cuda.synchronize()
    assert net_c.step == net_a.step
    for k in ("params", "m", "v", "packed"):
        a, c = getattr(net_a, k).cpu().numpy(), getattr(net_c, k).cpu().numpy()
        assert np.array_equal(a.view(np.uint8), c.view(np.uint8)), k
    assert loss_b == loss_a[:1] and loss_c == loss_a[1:]
    dev.free()
