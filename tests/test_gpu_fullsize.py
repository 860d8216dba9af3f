"""GPU parity at the benchmark's full sizes, every particle compared.

The workloads are the 64^3 Kelvin-Helmholtz layers (262144 particles) and the
128^3 Sedov blast (2097152 particles, the benchmark set), run through the C
entry points with the parameters bench.py uses.  The FP64 oracle runs the
same step on the host (a few seconds with all host threads), so no sampling
is needed.  Tolerances as in the small cases: 1e-12 (FP64), 1e-5 (mixed:
fields against their largest magnitude, flux sums per particle against the
particle's own scales), exact pair and face counts.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from gpu_helpers import check_fields, run_both, _need_gpu  # noqa: E402
from paper_2211_12243_amd import mfm  # noqa: E402
from paper_2211_12243_amd import workloads as W  # noqa: E402

CASES = [
    ("kh64_mfv_fp64", lambda: W.kh(n=64, seed=2), {"scheme": "mfv"}, "fp64", 1e-12),
    ("kh64_mfm_mixed", lambda: W.kh(n=64, seed=2), {"scheme": "mfm"}, "mixed", 1e-5),
    ("sedov128_mfm_fp64", lambda: W.sedov(n=128, seed=3), {"scheme": "mfm"}, "fp64", 1e-12),
    ("sedov128_mfm_mixed", lambda: W.sedov(n=128, seed=3), {"scheme": "mfm"}, "mixed", 1e-5),
]


@pytest.mark.parametrize("name,maker,cfg,precision,tol", CASES, ids=[c[0] for c in CASES])
def test_full_size_parity(name, maker, cfg, precision, tol):
    st = maker()
    print(f"[fullsize] {name}: {len(st['x'])} particles", flush=True)
    gpu, new, dt, diag, ref = run_both(cfg, st, precision=precision)
    errs = check_fields(gpu, new, dt, diag, ref, tol, st, normwise=(precision == "mixed"))
    print(f"[fullsize] {name}: worst {max(errs.values()):.2e}", flush=True)


def _quick_guess_network():
    """A guess network trained briefly on faces of a small Sod set."""
    from oracle import mlp as omlp

    st = W.sod(n=24, seed=31)
    params = mfm.params_from_dict({"scheme": "mfv"})
    ctx = mfm.Context(params, len(st["x"]))
    ps = mfm.ParticleSet(st)
    rec = torch.zeros((2_000_000, mfm.DUMP_STRIDE), dtype=torch.float32, device="cuda")
    mfm.mfm_face_dump(ctx, rec)
    mfm.run_pipeline(ctx, ps, 1.0, update=False)
    cnt = mfm.mfm_face_dump_count(ctx)
    mfm.mfm_face_dump(ctx, None)
    ctx.close()
    rows = rec[:cnt][mfm.guess_gate(rec[:cnt])].contiguous()
    r = rows.cpu().numpy().astype(np.float64)
    norm = omlp.norm_from(r[:, :6], r[:, 6]).astype(np.float32)
    state = mfm.MLPState(omlp.init_params(3).astype(np.float32), norm)
    for _ in range(200):
        mfm.mfm_mlp_train_step(state, rows, 3e-3)
    return state


def test_full_size_learned_guess_parity():
    _need_gpu()
    state = _quick_guess_network()
    st = W.sedov(n=128, seed=3)
    print("[fullsize] sedov128 mfm mixed + learned guess", flush=True)
    gpu, new, dt, diag, ref = run_both({"scheme": "mfm", "guess": 1}, st, precision="mixed",
                                       setup=lambda ctx: mfm.mfm_mlp_attach(ctx, state))
    check_fields(gpu, new, dt, diag, ref, 1e-5, st, normwise=True)
    print(f"[fullsize] learned: fallbacks {diag['guess_fallback']} of {diag['faces']} faces",
          flush=True)
