"""Checkpoints of the ranking network's training state (float32 master
weights, Adam moments and step, epochs done): the file round-trips exactly,
and foreign or malformed files are refused (the loader is safetensors, which
executes nothing from the file)."""
import numpy as np
import pytest

from paper_2404_06452_amd import _paam, surrogate


def _state(seed):
    r = np.random.default_rng(seed)
    return [r.standard_normal(_paam.MLP_PARAMS).astype(np.float32) for _ in range(3)]


def test_state_round_trips(tmp_path):
    p, m, v = _state(0)
    path = str(tmp_path / "net.safetensors")
    surrogate.save_state(path, p, m, v, step=1234, epoch=3)
    st = surrogate.load_state(path)
    assert st["step"] == 1234 and st["epoch"] == 3
    for k, a in (("params", p), ("adam_m", m), ("adam_v", v)):
        assert st[k].dtype == np.float32 and np.array_equal(st[k].view(np.uint32), a.view(np.uint32))
    surrogate.save_state(path, p, m, v, step=0)
    assert surrogate.load_state(path)["epoch"] is None


def test_malformed_states_are_refused(tmp_path):
    p, m, v = _state(1)
    with pytest.raises(ValueError):
        surrogate.save_state(str(tmp_path / "a"), p[:-1], m, v, step=1)
    from safetensors.numpy import save_file
    other = str(tmp_path / "other.safetensors")
    save_file({"params": p, "adam_m": m, "adam_v": v}, other, metadata={"format": "something"})
    with pytest.raises(ValueError):
        surrogate.load_state(other)
    short = str(tmp_path / "short.safetensors")
    save_file({"params": p[:10], "adam_m": m, "adam_v": v}, short,
              metadata={"format": surrogate.CHECKPOINT_FORMAT, "step": "1", "epoch": ""})
    with pytest.raises(ValueError):
        surrogate.load_state(short)
