"""The oracle's density loop for a sample of particles (oracle.density_at,
used to check the GPU at sizes where the whole oracle pass is too slow) gives
each sampled particle what the whole pass gives it: every particle is a
candidate there, so only the order of the kernel sums differs."""
import numpy as np
import pytest

import oracle
from paper_2211_12243_amd import workloads as W


@pytest.mark.parametrize("name,st", [("sod", W.sod(n=12, seed=5)),
                                     ("clustered", W.clustered(n=16, seed=4))])
def test_sample_equals_the_whole_pass(name, st):
    cfg = {"scheme": "mfm"}
    full, cf = oracle.density(cfg, st["x"], st["y"], st["z"], st["H"])
    idx = np.random.default_rng(1).choice(st["x"].size, 200, replace=False)
    idx[0] = int(np.argmax(st["H"]))   # the widest search
    idx[1] = int(np.argmin(st["H"]))   # the densest spot
    part, cp = oracle.density_at(cfg, st["x"], st["y"], st["z"], st["H"], idx)
    for k in ("H", "V", "ncond_tilde"):
        err = np.abs(part[k] - full[k][idx]) / np.abs(full[k][idx])
        assert err.max() < 1e-12, (name, k, err.max())
    assert np.array_equal(part["nngb"], full["nngb"][idx])
    assert cp["h_noconv"] == 0


def test_bad_index_is_rejected():
    st = W.sod(n=8, seed=5)
    with pytest.raises(RuntimeError):
        oracle.density_at({}, st["x"], st["y"], st["z"], st["H"], [st["x"].size])
