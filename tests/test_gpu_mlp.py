"""GPU tests of the learned Riemann guess: the matrix-core network against the
FP64 reference network, the face dump against the oracle's exact solver,
training, and flux parity with the guess switched on.

Tolerances.  The matrix cores see BF16 operands (unit roundoff u = 2^-9,
about 2e-3).  The FP64 reference takes the same BF16-rounded weights and
standardised inputs, so what remains is the BF16 rounding of the three hidden
activations (and, backwards, of the three activation gradients) with FP32
accumulation: a few u.  Forward outputs and every gradient tensor are compared
normwise (||gpu - ref||_2 / ||ref||_2) at 1e-2.  The flux results with the
learned guess are held to the same bars as with the plain guess (1e-12 FP64,
1e-5 mixed): the Newton iteration finishes the solve to the same root.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from oracle import mlp as omlp  # noqa: E402
from gpu_helpers import check_fields, run_both, _need_gpu  # noqa: E402
from paper_2211_12243_amd import mfm  # noqa: E402
from paper_2211_12243_amd import workloads as W  # noqa: E402

TOL_NET = 1e-2


def _nrm(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _random_rows(seed, n):
    rng = np.random.default_rng(seed)
    X = np.stack([rng.normal(0, 1.5, n), rng.normal(0, 3.0, n), rng.normal(0, 1.0, n),
                  rng.normal(0, 0.5, n), rng.normal(0, 0.5, n), rng.normal(0, 0.7, n)], axis=1)
    t = 0.3 * X[:, 1] + 0.5 * np.tanh(X[:, 2]) + rng.normal(0, 0.1, n)
    rows = np.zeros((n, mfm.DUMP_STRIDE), dtype=np.float32)
    rows[:, :6] = X
    rows[:, 6] = t
    return rows


def _random_params(seed):
    rng = np.random.default_rng(seed)
    d = omlp.unpack(omlp.init_params(seed))
    for b in ("b1", "b2", "b3"):
        d[b][:] = rng.normal(0, 0.2, omlp.HID)
    d["b4"][:] = 0.1
    return omlp.pack(d).astype(np.float32)


@pytest.mark.parametrize("n", [1000, 64, 37])
def test_forward_matches_fp64_network(n):
    _need_gpu()
    rows = _random_rows(1, n)
    params = _random_params(2)
    norm = omlp.norm_from(rows[:, :6].astype(np.float64), rows[:, 6].astype(np.float64))
    norm32 = norm.astype(np.float32)
    print(f"[mlp] forward n={n}", flush=True)
    st = mfm.MLPState(params, norm32)
    y = mfm.mfm_mlp_predict(st, torch.from_numpy(rows).cuda()).cpu().numpy()
    ref = omlp.forward(params.astype(np.float64), norm32.astype(np.float64),
                       rows[:, :6].astype(np.float64), round_bf16=True)
    err = _nrm(y, ref)
    print(f"forward normwise error {err:.2e}", flush=True)
    assert err <= TOL_NET


@pytest.mark.parametrize("n", [1000, 33])
def test_gradient_matches_fp64_network(n):
    _need_gpu()
    rows = _random_rows(3, n)
    params = _random_params(4)
    norm = omlp.norm_from(rows[:, :6].astype(np.float64),
                          rows[:, 6].astype(np.float64)).astype(np.float32)
    print(f"[mlp] gradient n={n}", flush=True)
    st = mfm.MLPState(params, norm)
    loss = mfm.mfm_mlp_backward(st, torch.from_numpy(rows).cuda())
    p_dev, g_dev = mfm.mfm_mlp_get(st)
    assert np.array_equal(p_dev, params)
    lref, gref = omlp.loss_grad(params.astype(np.float64), norm.astype(np.float64),
                                rows[:, :6].astype(np.float64), rows[:, 6].astype(np.float64),
                                round_bf16=True)
    assert abs(loss - lref) <= TOL_NET * lref
    G, R = omlp.unpack(g_dev), omlp.unpack(gref)
    errs = {k: _nrm(G[k], R[k]) for k in ("W2", "b2", "W3", "b3", "w4", "b4", "b1")}
    errs["W1"] = _nrm(G["W1"][:6], R["W1"][:6])
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert np.all(G["W1"][6:] == 0.0)
    assert max(errs.values()) <= TOL_NET, errs


def test_adam_first_step():
    _need_gpu()
    rows = _random_rows(5, 512)
    params = _random_params(6)
    norm = omlp.norm_from(rows[:, :6].astype(np.float64),
                          rows[:, 6].astype(np.float64)).astype(np.float32)
    st = mfm.MLPState(params, norm)
    lr = 1e-2
    mfm.mfm_mlp_train_step(st, torch.from_numpy(rows).cuda(), lr)
    p1, _ = mfm.mfm_mlp_get(st)
    _, gref = omlp.loss_grad(params.astype(np.float64), norm.astype(np.float64),
                             rows[:, :6].astype(np.float64), rows[:, 6].astype(np.float64),
                             round_bf16=True)
    step = params.astype(np.float64) - p1.astype(np.float64)
    # first Adam step: lr g / (|g| + eps), i.e. lr sign(g) where |g| >> eps
    big = np.abs(gref) > 0.05 * np.abs(gref).max()
    assert big.sum() > 100
    assert np.abs(step[big] - lr * np.sign(gref[big])).max() <= 3e-5
    pad = np.zeros(omlp.NPARAM, dtype=bool)
    pad[6 * omlp.HID:16 * omlp.HID] = True  # W1 padding rows never move
    assert np.all(step[pad] == 0.0)


def _dump_faces(st, cfg, cap, precision="fp64", steps_before=0):
    params = mfm.params_from_dict(cfg, precision=precision)
    ctx = mfm.Context(params, len(st["x"]))
    ps = mfm.ParticleSet(st)
    for _ in range(steps_before):
        mfm.mfm_step(ctx, ps, 1.0)
    rec = torch.zeros((cap, mfm.DUMP_STRIDE), dtype=torch.float32, device="cuda")
    mfm.mfm_face_dump(ctx, rec)
    mfm.mfm_reset_counters(ctx)
    mfm.run_pipeline(ctx, ps, 1.0, update=False)
    count = mfm.mfm_face_dump_count(ctx)
    diag = mfm.mfm_diagnostics(ctx)
    mfm.mfm_face_dump(ctx, None)
    ctx.close()
    return rec[:count], diag


def _target_from_features(x, gamma):
    """ln(p*/P_avg) of the states that a record's features describe (right
    state rho = P = 1 at rest; the ratio depends only on the three groups)."""
    rhoL, PL = math.exp(x[0]), math.exp(x[1])
    cL, cR = math.sqrt(gamma * PL / rhoL), math.sqrt(gamma)
    du = math.copysign(math.expm1(abs(x[2])), x[2]) * 0.5 * (cL + cR)
    s, ps, _, _ = oracle.riemann(gamma, rhoL, 0.0, PL, 1.0, du, 1.0)
    return s, math.log(ps / (0.5 * (PL + 1.0)))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_face_dump_against_exact_solver(precision):
    _need_gpu()
    st = W.sedov(n=24, seed=3)
    cfg = {"scheme": "mfm"}
    print(f"[mlp] dump sedov24 {precision}", flush=True)
    rec, diag = _dump_faces(st, cfg, 2_000_000, precision)
    r = rec.cpu().numpy().astype(np.float64)
    n = r.shape[0]
    assert 0 < n <= diag["faces"] - diag["vacuum"]
    # every face's iterations are counted once: the dump holds all of them
    assert int(r[:, 7].sum()) == diag["riemann_iters"]
    assert np.all(r[:, 7] >= 1)
    # the sound-speed ratio is fixed by the density and pressure ratios
    assert np.abs(r[:, 5] - 0.5 * (r[:, 1] - r[:, 0])).max() <= 2e-5
    rng = np.random.default_rng(0)
    worst = 0.0
    for k in rng.choice(n, 1500, replace=False):
        s, y = _target_from_features(r[k], 5.0 / 3.0)
        assert s == 0
        worst = max(worst, abs(y - r[k, 6]))
    print(f"dumped target vs exact solver: max abs error {worst:.2e}", flush=True)
    assert worst <= 1e-4


def _train(rows_dev, steps, lr, batch, seed=0):
    r = rows_dev.cpu().numpy().astype(np.float64)
    norm = omlp.norm_from(r[:, :6], r[:, 6]).astype(np.float32)
    st = mfm.MLPState(omlp.init_params(seed).astype(np.float32), norm)
    n = rows_dev.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    losses = []
    for it in range(steps):
        idx = torch.randint(0, n, (batch,), generator=g).cuda()
        want = it % 50 == 0 or it == steps - 1
        l = mfm.mfm_mlp_train_step(st, rows_dev[idx].contiguous(), lr, want_loss=want)
        if want:
            losses.append(l)
    return st, losses


def test_training_and_learned_guess_parity():
    _need_gpu()
    print("[mlp] train on faces of sod24 and sedov32 (after 5 steps)", flush=True)
    parts = []
    for st, cfg, k in ((W.sod(n=24, seed=21), {"scheme": "mfv"}, 0),
                       (W.sedov(n=32, seed=11), {"scheme": "mfm"}, 5)):
        rec, _ = _dump_faces(st, cfg, 4_000_000, steps_before=k)
        parts.append(rec[mfm.guess_gate(rec)])
    rec = torch.cat(parts)
    print(f"{rec.shape[0]} training faces pass the gate", flush=True)
    assert rec.shape[0] > 1000
    st, losses = _train(rec, 400, 3e-3, 4096)
    print("losses", [f"{v:.3e}" for v in losses], flush=True)
    assert losses[-1] < 0.3 * losses[0]
    # held-out set: prediction error of ln(p*/P_avg)
    test_rows, _ = _dump_faces(W.sod(n=16, seed=12), {"scheme": "mfv"}, 2_000_000)
    test_rows = test_rows[mfm.guess_gate(test_rows)]
    y = mfm.mfm_mlp_predict(st, test_rows).cpu().numpy()
    t = test_rows[:, 6].cpu().numpy()
    print(f"held-out rms error of ln(p*/P_avg): {np.sqrt(np.mean((y - t) ** 2)):.3e}, "
          f"target std {t.std():.3e}", flush=True)

    def attach(ctx):
        mfm.mfm_mlp_attach(ctx, st)

    cases = (("sod16", W.sod(n=16, seed=1), {"scheme": "mfv"}),
             ("sedov24", W.sedov(n=24, seed=3), {"scheme": "mfm"}))
    for name, state, cfg in cases:
        for precision, tol in (("fp64", 1e-12), ("mixed", 1e-5)):
            plain_rec, plain = _dump_faces(state, cfg, 2_000_000, precision)
            hard = mfm.guess_gate(plain_rec)
            nh = max(int(hard.sum()), 1)
            it_hard_plain = float(plain_rec[hard][:, 7].sum())
            print(f"[mlp] learned-guess parity {name} {precision}", flush=True)
            gpu, new, dt, diag, ref = run_both(dict(cfg, guess=1), state, precision=precision,
                                               setup=attach)
            check_fields(gpu, new, dt, diag, ref, tol, state, normwise=(precision == "mixed"))
            saved = plain["riemann_iters"] - diag["riemann_iters"]
            print(f"{name} {precision}: {int(hard.sum())} of {diag['faces']} faces gated; Newton "
                  f"steps on them plain {it_hard_plain / nh:.3f}/face, learned "
                  f"{(it_hard_plain - saved) / nh:.3f}/face; fallbacks "
                  f"{diag['guess_fallback']}", flush=True)
            assert diag["faces"] == plain["faces"]
            assert diag["guess_fallback"] < nh


def test_garbage_weights_fall_back():
    _need_gpu()
    params = np.full(omlp.NPARAM, 50.0, dtype=np.float32)
    params[6 * omlp.HID:16 * omlp.HID] = 0.0
    norm = np.zeros(16, dtype=np.float32)
    norm[6:12] = 1.0
    norm[12], norm[13] = 0.0, 1.0
    st = mfm.MLPState(params, norm)
    cfg = {"scheme": "mfv", "guess": 1}
    sod = W.sod(n=16, seed=1)
    rec, _ = _dump_faces(sod, {"scheme": "mfv"}, 1_000_000)
    n_hard = int(mfm.guess_gate(rec).sum())
    assert n_hard > 0
    print("[mlp] garbage weights sod16", flush=True)
    gpu, new, dt, diag, ref = run_both(cfg, sod, setup=lambda ctx: mfm.mfm_mlp_attach(ctx, st))
    check_fields(gpu, new, dt, diag, ref, 1e-12, sod)
    # huge outputs overflow exp(): every face given to the network falls back
    assert diag["guess_fallback"] == n_hard


def test_learned_guess_without_network_is_an_error():
    _need_gpu()
    st = W.sod(n=8, seed=1)
    params = mfm.params_from_dict({"scheme": "mfv", "guess": 1})
    ctx = mfm.Context(params, len(st["x"]))
    ps = mfm.ParticleSet(st)
    mfm.mfm_build_cells(ctx, ps)
    mfm.mfm_density(ctx, ps)
    mfm.mfm_gradients(ctx, ps, 1.0)
    with pytest.raises(mfm.MFMError, match="status -8"):
        mfm.mfm_fluxes(ctx, ps)
    ctx.close()
