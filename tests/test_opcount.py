"""The benchmark's algorithmic flop counts come from the oracle's operation
counter (oracle/opcount.cpp): the oracle compiled with a number type that
counts each add, multiply, divide, square root and power.

* the counted build computes the same face contribution as the oracle;
* bench.FLOPS_PER_FACE is the counter's mean over the benchmark's sample
  (20000 faces of the first step of the 128^3 Sedov set);
* bench.FLOPS_PER_GRAD_PAIR is the counter's per-pair figure of the
  gradient loop.
"""
import numpy as np
import pytest

import bench
import oracle
from oracle import opcount
from paper_2211_12243_amd import workloads as W


def _small_face_set():
    st = W.sod(n=8, seed=3)
    cfg = {"scheme": "mfv"}
    d, _ = oracle.density(cfg, st["x"], st["y"], st["z"], st["H"])
    g, _ = oracle.gradients(cfg, st["x"], st["y"], st["z"], d["H"], d["V"], st["m"], st["vx"],
                            st["vy"], st["vz"], st["U"])
    return st, d, g


@pytest.mark.parametrize("scheme", ["mfm", "mfv"])
def test_counted_face_equals_the_oracle_face(scheme):
    st, d, g = _small_face_set()
    cfg = {"scheme": scheme}
    fa, fb = oracle.fluxes_face_list(cfg, st["x"], st["y"], st["z"], d["H"])
    args = (st["x"], st["y"], st["z"], d["H"], d["V"], g["rho"], st["vx"], st["vy"], st["vz"],
            g["P"], g["B"], g["grad"], 1e-3)
    for f in range(0, fa.size, max(fa.size // 50, 1)):
        c_ref, _ = oracle.face(cfg, fa[f], fb[f], *args)
        k, c = opcount.face_ops(cfg, fa[f], fb[f], *args)
        assert np.array_equal(c, c_ref)
        assert k.sum() > 200 and np.all(k >= 0)


def test_mfv_face_counts_more_than_mfm():
    st, d, g = _small_face_set()
    args = (st["x"], st["y"], st["z"], d["H"], d["V"], g["rho"], st["vx"], st["vy"], st["vz"],
            g["P"], g["B"], g["grad"], 1e-3)
    fa, fb = oracle.fluxes_face_list({}, st["x"], st["y"], st["z"], d["H"])
    k_mfm, _ = opcount.face_ops({"scheme": "mfm"}, fa[0], fb[0], *args)
    k_mfv, _ = opcount.face_ops({"scheme": "mfv"}, fa[0], fb[0], *args)
    # the MFV face samples the solution and builds the full flux vector
    assert k_mfv.sum() > k_mfm.sum()


@pytest.mark.slow
def test_benchmark_flop_counts_are_the_counters():
    st = W.sedov(n=128, seed=3)
    for scheme in ("mfm", "mfv"):
        mean, k, nf = opcount.face_sample({"scheme": scheme}, st, 20000)
        print(scheme, f"{mean.sum():.2f} flop/face over {k} of {nf} faces")
        assert mean.sum() == pytest.approx(bench.FLOPS_PER_FACE[scheme], abs=0.01)
    sub = W.sedov(n=24, seed=3)
    cfg = {"scheme": "mfm"}
    d, _ = oracle.density(cfg, sub["x"], sub["y"], sub["z"], sub["H"])
    gl, _, pairs = opcount.gradients_ops(cfg, sub["x"], sub["y"], sub["z"], d["H"], d["V"],
                                         sub["m"], sub["vx"], sub["vy"], sub["vz"], sub["U"])
    assert gl.sum() / pairs == pytest.approx(bench.FLOPS_PER_GRAD_PAIR, abs=0.05)
