"""mfm_step: one whole step with one synchronisation.

The step sizes its cell grid from the max H the previous step left, checks it
on the device, and rejects a density pass whose grid or candidate lists were
too small (its later kernels return at once and the state is not updated),
then repeats it.  These tests drive each path against the oracle's step:

* smoothing lengths at half their root, so the first grid is too fine;
* a particle set replaced in place (same arrays) by one with larger H, so the
  max H the previous step left is stale;
* a candidate list capacity too small: an error, with the state untouched;
* the time per step on the 8192-particle sound wave;
* steps that keep the last particle order against steps that sort.
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from gpu_helpers import _need_gpu  # noqa: E402
from paper_2211_12243_amd import mfm  # noqa: E402
from paper_2211_12243_amd import workloads as W  # noqa: E402

KEYS = ("x", "y", "z", "vx", "vy", "vz", "m", "E", "U", "H")


def _by_id(ps):
    ids = ps["id"].cpu().numpy()
    out = {}
    for k in KEYS:
        a = np.empty(len(ids))
        a[ids] = ps[k].cpu().numpy()
        out[k] = a
    return out


def _compare(got, want, tol):
    for k in KEYS:
        d = np.abs(got[k] - want[k])
        if k in ("x", "y", "z"):
            d = np.minimum(d, 1.0 - d)
            err = d.max()
        else:
            err = d.max() / max(np.abs(want[k]).max(), 1e-300)
        assert err <= tol, (k, err)


def test_step_rebuilds_a_too_fine_grid():
    _need_gpu()
    st = W.kh(n=12, seed=5)
    st["H"] = 0.5 * st["H"]
    cfg = {"scheme": "mfm"}
    ctx = mfm.Context(mfm.params_from_dict(cfg), len(st["x"]))
    ps = mfm.ParticleSet(st)
    print("[step] H at half the root", flush=True)
    dt = mfm.mfm_step(ctx, ps, 1.0)
    diag = mfm.mfm_diagnostics(ctx)
    ref, dt_ref, _ = oracle.step(cfg, st, 1.0)
    assert diag["cell_rebuilds"] >= 1
    assert abs(dt - dt_ref) <= 1e-12 * dt_ref
    _compare(_by_id(ps), ref, 1e-11)
    ctx.close()


def test_step_after_state_replaced_in_place():
    _need_gpu()
    a = W.kh(n=12, seed=5)
    b = W.kh(n=12, seed=6)
    b["H"] = 1.25 * b["H"]  # above the max H the first step leaves (and its cells)
    cfg = {"scheme": "mfv"}
    ctx = mfm.Context(mfm.params_from_dict(cfg), len(a["x"]))
    ps = mfm.ParticleSet(a)
    print("[step] state replaced in place", flush=True)
    mfm.mfm_step(ctx, ps, 1.0)
    for k in KEYS:
        ps[k].copy_(torch.as_tensor(b[k], dtype=torch.float64))
    ps["id"].copy_(torch.arange(len(a["x"]), dtype=torch.int64))
    before = mfm.mfm_diagnostics(ctx)["cell_rebuilds"]
    dt = mfm.mfm_step(ctx, ps, 1.0)
    after = mfm.mfm_diagnostics(ctx)["cell_rebuilds"]
    ref, dt_ref, _ = oracle.step(cfg, b, 1.0)
    print("rebuilds in the second step:", after - before, flush=True)
    assert abs(dt - dt_ref) <= 1e-12 * dt_ref
    _compare(_by_id(ps), ref, 1e-11)
    ctx.close()


def test_list_overflow_in_a_step_leaves_the_state():
    _need_gpu()
    st = W.sod(n=10, seed=1)
    ctx = mfm.Context(mfm.params_from_dict({"scheme": "mfv", "max_list": 8}), len(st["x"]))
    ps = mfm.ParticleSet(st)
    print("[step] max_list = 8", flush=True)
    with pytest.raises(mfm.MFMError, match="status -6"):
        mfm.mfm_step(ctx, ps, 1.0)
    got = _by_id(ps)
    # the conserved state and positions are untouched (H, the start value of
    # the smoothing-length solve, is the density pass's to overwrite)
    for k in KEYS:
        if k != "H":
            assert np.array_equal(got[k], st[k]), k
    # the error is the call's own: a later step with room succeeds
    ctx.close()
    ctx = mfm.Context(mfm.params_from_dict({"scheme": "mfv"}), len(st["x"]))
    ps = mfm.ParticleSet(st)
    mfm.mfm_step(ctx, ps, 1.0)
    ctx.close()


def test_soundwave_step_time():
    """8192 particles (the sound wave at N = 128): few flux blocks and search
    buckets must still fill the chip (sliced flux blocks, a wavefront per
    search chunk); 0.30 ms per step measured, 0.67 ms without them."""
    _need_gpu()
    st = W.soundwave(128, nyz=8, A=1e-3, gamma=1.4)
    cfg = {"scheme": "mfm", "gamma": 1.4, "limiter": 0, "box": W.soundwave_box(128, 8)}
    ctx = mfm.Context(mfm.params_from_dict(cfg), len(st["x"]))
    ps = mfm.ParticleSet(st)
    for _ in range(5):
        mfm.mfm_step(ctx, ps, 1.0)
    torch.cuda.synchronize()
    k = 50
    t0 = time.perf_counter()
    for _ in range(k):
        mfm.mfm_step(ctx, ps, 1.0)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / k * 1e3
    print(f"[step] sound wave N=128: {ms:.3f} ms per step", flush=True)
    ctx.close()
    assert ms < 0.45


def test_kept_order_steps_match_sorted_steps():
    """mfm_step may skip the Morton sort and build the tree over the order of
    its last sort (while its timed cells, search and density stages stay
    below those of that sorting step).  Such steps must give what steps that
    sort every time give (mfm_build_cells before each step clears the
    reuse), particle by particle: the order changes only the grouping of
    the search and the rounding order of the sums."""
    _need_gpu()
    st = W.kh(n=32, seed=2)
    cfg = {"scheme": "mfm"}
    n = st["x"].size
    a = mfm.Context(mfm.params_from_dict(cfg), n)
    pa = mfm.ParticleSet(st)
    b = mfm.Context(mfm.params_from_dict(cfg), n)
    pb = mfm.ParticleSet(st)
    cells_a, cells_b = [], []
    for k in range(8):
        mfm.mfm_enable_timing(a, True)
        da = mfm.mfm_step(a, pa, 1.0)
        cells_a.append(mfm.mfm_kernel_times(a)["cells"][0])
        mfm.mfm_build_cells(b, pb)
        mfm.mfm_enable_timing(b, True)
        db = mfm.mfm_step(b, pb, 1.0)
        cells_b.append(mfm.mfm_kernel_times(b)["cells"][0])
        assert abs(da - db) <= 1e-12 * db, k
    torch.cuda.synchronize()
    print("[step] cells ms, reusing:", " ".join(f"{t:.3f}" for t in cells_a), flush=True)
    print("[step] cells ms, sorting:", " ".join(f"{t:.3f}" for t in cells_b), flush=True)
    got, ref = _by_id(pa), _by_id(pb)
    for k in KEYS:
        d = np.abs(got[k] - ref[k])
        if k in ("x", "y", "z"):
            d = np.minimum(d, 1.0 - d)
            assert d.max() <= 1e-13, k
        else:
            # velocities against the flow's speed scale, the rest against
            # their own magnitude
            scale = max(np.abs(ref[k]).max(), 1.0 if k in ("vx", "vy", "vz") else 0.0)
            assert d.max() <= 1e-11 * scale, k
    a.close()
    b.close()
