"""Window-boundary checkpoints (paper_1710_02401_amd/checkpoint.py), host
side: the description hash and the refusal of a checkpoint written for
another description, without a GPU."""
import numpy as np
import pytest

import workloads
from paper_1710_02401_amd import checkpoint


def test_config_hash_is_stable_and_sensitive():
    cfg = workloads.tiny_configs()[0]
    assert checkpoint.config_hash(cfg) == checkpoint.config_hash(dict(cfg))
    assert checkpoint.config_hash(cfg) != checkpoint.config_hash(dict(cfg, dt=cfg["dt"] * 2))
    assert checkpoint.config_hash(cfg) != checkpoint.config_hash(dict(cfg, mu=[0.0, -3.0]))


def test_checkpoint_of_another_description_is_refused(tmp_path):
    cfg = workloads.tiny_configs()[0]
    path = tmp_path / "w.npz"
    with open(path, "wb") as f:
        np.savez(f, c_end=np.zeros(4, complex), t_next=np.float64(1.0),
                 config=np.array(checkpoint.config_hash(cfg)))
    data = checkpoint.load(path, cfg)
    assert float(data["t_next"]) == 1.0
    with pytest.raises(ValueError, match="another workload description"):
        checkpoint.load(path, dict(cfg, dt=cfg["dt"] * 2))
