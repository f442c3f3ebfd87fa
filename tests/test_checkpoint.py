"""Training checkpoints: written without pickled objects, read back
unchanged, refused when the file no longer matches its recorded SHA-256."""
import numpy as np
import pytest

from paper_1606_00548_amd import train


def _state(rng):
    g = np.random.default_rng(3)
    g.permutation(10)
    return {"theta": rng.standard_normal(50).astype(np.float32), "m": rng.standard_normal(50).astype(np.float32),
            "v": rng.random(50).astype(np.float32), "adam_step": 12, "epoch": 3,
            "rng_state": g.bit_generator.state, "history": [{"epoch": 1, "train_loss": 0.5}]}


def test_checkpoint_round_trip(tmp_path):
    st = _state(np.random.default_rng(0))
    path = str(tmp_path / "ck.npz")
    train.save_checkpoint(path, st, {"lr": 1e-3})
    ck = train.load_checkpoint(path)
    for k in ("theta", "m", "v"):
        assert ck[k].dtype == np.float32 and np.array_equal(ck[k], st[k])
    assert ck["adam_step"] == 12 and ck["epoch"] == 3 and ck["history"] == st["history"]
    assert ck["meta"]["lr"] == 1e-3 and len(ck["meta"]["sha256"]) == 64
    # the generator resumes where it stopped
    g1 = np.random.default_rng(0)
    g1.bit_generator.state = ck["rng_state"]
    g2 = np.random.default_rng(3)
    g2.permutation(10)
    assert np.array_equal(g1.permutation(20), g2.permutation(20))


def test_tampered_checkpoint_is_refused(tmp_path):
    path = str(tmp_path / "ck.npz")
    train.save_checkpoint(path, _state(np.random.default_rng(1)), {})
    raw = bytearray(open(path, "rb").read())
    raw[len(raw) // 2] ^= 0xFF
    open(path, "wb").write(bytes(raw))
    with pytest.raises(ValueError):
        train.load_checkpoint(path)
