"""mfm_create_static: a context on the library's own static device scratch,
for callers that cannot allocate.  Its results must be those of a context on
a caller workspace (mfm_create), to the FP64 bar, on two contexts in a row on
the same GPU, the second with a smaller particle set (the scratch keeps the
first one's contents).  Also: a request larger than the scratch and a second
static context while one exists are refused.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from gpu_helpers import _need_gpu, rel_err  # noqa: E402
from paper_2211_12243_amd import mfm  # noqa: E402
from paper_2211_12243_amd import workloads as W  # noqa: E402

FIELDS = ("H", "V", "rho", "P", "c", "ncond", "dt_i", "B", "grad", "dQ")
STATE = ("x", "y", "z", "vx", "vy", "vz", "m", "E", "U")


def _run(st, cfg, static):
    n = len(st["x"])
    params = mfm.params_from_dict(cfg)
    ctx = mfm.Context(params, n, static=static)
    ps = mfm.ParticleSet(st)
    mfm.run_pipeline(ctx, ps, 1.0, update=False)
    torch.cuda.synchronize()
    ids = ps["id"].cpu().numpy()
    out = {}
    for k in FIELDS:
        t = ps[k].cpu().numpy()
        a = np.empty_like(t)
        a[..., ids] = t
        out[k] = a
    dt = mfm.mfm_step(ctx, ps, 1.0)  # one more step through the single-sync path
    torch.cuda.synchronize()
    ids = ps["id"].cpu().numpy()
    for k in STATE:
        a = np.empty(n)
        a[ids] = ps[k].cpu().numpy()
        out["step_" + k] = a
    out["dt"] = dt
    ctx.close()
    return out


def _compare(a, b, tol):
    worst = 0.0
    for k in a:
        if k == "dt":
            e = abs(a[k] - b[k]) / b[k]
        elif a[k].ndim == 2:
            e = max(rel_err(a[k][q], b[k][q]) for q in range(a[k].shape[0]))
        else:
            e = rel_err(a[k], b[k])
        assert e <= tol, (k, e)
        worst = max(worst, e)
    return worst


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_static_context_matches_workspace_context(precision):
    _need_gpu()
    cases = (("kh14 mfv", W.kh(n=14, seed=7), {"scheme": "mfv"}),
             ("sod10 mfm", W.sod(n=10, seed=8), {"scheme": "mfm"}))
    for name, st, cfg in cases:  # the second set is smaller than the first
        print(f"[no-alloc] {name} {precision}: {len(st['x'])} particles", flush=True)
        cfg = dict(cfg, precision=precision)
        ref = _run(st, cfg, static=False)
        got = _run(st, cfg, static=True)
        worst = _compare(got, ref, 1e-12 if precision == "fp64" else 1e-6)
        print(f"[no-alloc] {name} {precision}: worst relative difference {worst:.2e}",
              flush=True)


def test_static_context_limits():
    _need_gpu()
    L = mfm.lib()
    cap = L.mfm_static_workspace_bytes()
    params = mfm.params_from_dict({"scheme": "mfm"})
    n_big = 200_000
    assert L.mfm_workspace_bytes(params, n_big) > cap
    with pytest.raises(mfm.MFMError, match="status -2"):
        mfm.Context(params, n_big, static=True)
    ctx = mfm.Context(params, 1000, static=True)
    with pytest.raises(mfm.MFMError, match="status -8"):
        mfm.Context(params, 1000, static=True)
    ctx.close()
    ctx = mfm.Context(params, 1000, static=True)  # released by mfm_destroy
    ctx.close()
