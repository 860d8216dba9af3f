"""GPU parity of the source terms (sec. 2.3.7-2.3.9) with the oracle's step.

Each case steps the same seeded set on both sides three times through
mfm_step / oracle.step_src and compares every particle's state, entropy and
entropy-mode flag (FP64 bar 1e-11 on the state after three steps):

* shear layers (MFV) in a uniform external field, with the entropy switch, in
  comoving coordinates (1/a = 0.9, H = 0.5): every source term at once, and
  the mass-exchange work of the MFV faces;
* cold shear layers (MFM, P = 1e-4) with the entropy switch: next to the
  shear the gas is cold against its neighbours' relative motion and its
  pressure comes from the entropy;
* a Hubble rate with gamma other than 5/3 is refused.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from gpu_helpers import _need_gpu  # noqa: E402
from paper_2211_12243_amd import mfm  # noqa: E402
from paper_2211_12243_amd import workloads as W  # noqa: E402

KEYS = ("x", "y", "z", "vx", "vy", "vz", "m", "E", "U", "H")


def _run(cfg, st, nsteps, accel=None, cosmo=None, precision="fp64"):
    n = len(st["x"])
    ctx = mfm.Context(mfm.params_from_dict(cfg, precision=precision), n)
    if cosmo:
        mfm.mfm_set_cosmology(ctx, *cosmo)
    ps = mfm.ParticleSet(st, entropy=bool(cfg.get("entropy_switch")), accel=accel)
    ref = {k: np.array(st[k], dtype=np.float64) for k in KEYS}
    S = np.zeros(n)
    emode = np.zeros(n, dtype=np.int32)
    for step in range(nsteps):
        print(f"[sources] step {step}", flush=True)
        dt = mfm.mfm_step(ctx, ps, 1.0)
        ref, dt_ref, cnt = oracle.step_src(cfg, ref, 1.0, accel=accel,
                                           inv_a=cosmo[0] if cosmo else 1.0,
                                           hubble=cosmo[1:] if cosmo else (0.0, 0.0),
                                           S=S if cfg.get("entropy_switch") else None,
                                           emode=emode if cfg.get("entropy_switch") else None)
        assert abs(dt - dt_ref) <= 1e-12 * dt_ref, (dt, dt_ref)
    torch.cuda.synchronize()
    ids = ps["id"].cpu().numpy()
    got = {}
    for k in KEYS + (("S", "emode") if cfg.get("entropy_switch") else ()):
        t = ps[k].cpu().numpy()
        a = np.empty_like(t)
        a[ids] = t
        got[k] = a
    diag = mfm.mfm_diagnostics(ctx)
    ctx.close()
    return got, ref, S, emode, diag


def _compare(got, ref, tol):
    for k in KEYS:
        d = np.abs(got[k] - ref[k])
        if k in ("x", "y", "z"):
            err = np.minimum(d, 1.0 - d).max()
        else:
            err = d.max() / max(np.abs(ref[k]).max(), 1e-300)
        print(k, f"{err:.2e}", flush=True)
        assert err <= tol, (k, err)


def test_all_sources_shear_layers_mfv():
    _need_gpu()
    st = W.kh(n=12, seed=9)
    n = len(st["x"])
    accel = np.zeros((3, n))
    accel[1] = -0.5
    cfg = {"scheme": "mfv", "entropy_switch": 1}
    got, ref, S, emode, diag = _run(cfg, st, 3, accel=accel, cosmo=(0.9, 0.5, 0.5))
    _compare(got, ref, 1e-11)
    assert np.abs(got["S"] - S).max() <= 1e-11 * np.abs(S).max()
    assert np.array_equal(got["emode"], emode)


def test_entropy_switch_cold_shear_mfm():
    _need_gpu()
    st = W.kh(n=12, seed=9, P=1e-4)
    cfg = {"scheme": "mfm", "entropy_switch": 1}
    got, ref, S, emode, diag = _run(cfg, st, 3)
    print("particles in the entropy branch:", int(emode.sum()), flush=True)
    assert emode.sum() > 0
    _compare(got, ref, 1e-11)
    assert np.array_equal(got["emode"], emode)
    on = emode == 1
    assert np.abs(got["S"][on] - S[on]).max() <= 1e-11 * np.abs(S[on]).max()


def test_hubble_needs_gamma_five_thirds():
    _need_gpu()
    st = W.sod(n=8, seed=1, gamma=1.4)
    ctx = mfm.Context(mfm.params_from_dict({"gamma": 1.4}), len(st["x"]))
    mfm.mfm_set_cosmology(ctx, 0.5, 0.0, 0.0)  # 1/a alone is fine
    with pytest.raises(mfm.MFMError, match="status -1"):
        mfm.mfm_set_cosmology(ctx, 0.5, 1.0, 1.0)
    ctx.close()
