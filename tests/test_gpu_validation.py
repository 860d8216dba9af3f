"""The paper's sound-wave convergence test (sec. 3.1.1) run through the
library's C entry points for one crossing time at several resolutions
(N particles along x, 8 across, gamma = 1.4, N_NGB = 32, no gradient
limiter).  The error is the L1 norm of the density against each particle's
own estimate at t = 0; ``paper_2211_12243_amd.validation`` documents why.

Observed on MI355X (FP64, A = 1e-5, N = 16, 32, 64): MFM 1.48e-7, 2.74e-8,
5.97e-9 (orders 2.43, 2.20); MFV 5.46e-7, 1.31e-7, 3.21e-8 (orders 2.06,
2.02).  Both schemes converge at second order, as in the paper, once the
face moves with the particles' mean velocity at the half step; with their
start-of-step velocities MFV converged at first order (1.40, 1.16)."""
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from gpu_helpers import _need_gpu  # noqa: E402
from paper_2211_12243_amd import validation as V  # noqa: E402


def _series(scheme, precision, A, Ns):
    _need_gpu()
    res = []
    for N in Ns:
        print(f"[soundwave] {scheme} {precision} A={A} N={N}", flush=True)
        r = V.run_soundwave(N, scheme, precision, A=A)
        print(f"  L1 {r['L1']:.3e} (against the exact profile {r['L1_exact']:.3e}, "
              f"at t=0 {r['L1_exact_0']:.3e}), {r['steps']} steps, {r['wall_s']:.3f} s",
              flush=True)
        assert abs(r["t"] - 1.0 / 1.4 ** 0.5) <= 1e-12
        res.append(r)
    return res, V.convergence_order(res)


def test_soundwave_mfm_is_second_order():
    res, orders = _series("mfm", "fp64", 1e-5, (16, 32, 64))
    print("orders", orders, flush=True)
    assert all(o >= 1.8 for o in orders), orders


def test_soundwave_mfm_mixed_tracks_fp64():
    """Mixed precision at A = 1e-3: the same second-order decrease from N = 16
    to 32 and the same error as FP64 within 5%."""
    mixed, orders = _series("mfm", "mixed", 1e-3, (16, 32))
    fp64, _ = _series("mfm", "fp64", 1e-3, (16, 32))
    assert orders[0] >= 1.8, orders
    for a, b in zip(mixed, fp64):
        assert abs(a["L1"] - b["L1"]) <= 0.05 * b["L1"], (a["L1"], b["L1"])


def test_soundwave_mfv_is_second_order():
    res, orders = _series("mfv", "fp64", 1e-5, (16, 32, 64))
    print("orders", orders, flush=True)
    assert all(o >= 1.8 for o in orders), orders


def test_soundwave_mfv_mixed_tracks_fp64():
    """The MFV sound wave in mixed precision at A = 1e-3, as for MFM."""
    mixed, orders = _series("mfv", "mixed", 1e-3, (16, 32))
    fp64, _ = _series("mfv", "fp64", 1e-3, (16, 32))
    assert orders[0] >= 1.8, orders
    for a, b in zip(mixed, fp64):
        assert abs(a["L1"] - b["L1"]) <= 0.05 * b["L1"], (a["L1"], b["L1"])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("scheme,bound", [("mfm", 0.012), ("mfv", 0.014)])
def test_sod_shock_tube(scheme, bound, precision):
    """The paper's shock tube (sec. 3.1.2) at t = 0.13 against the exact
    solution of its Riemann problem (the oracle's exact solver, sampled at
    (x - 0.5) / t), over 0.25 < x < 0.75, away from the mirrored tube at
    x = 0.  Observed L1 of (rho, vx, P): MFM 0.0074, 0.0145, 0.0075; MFV
    0.0075, 0.0160, 0.0078, the same in mixed precision.  The plateaus between the rarefaction and the
    shock hold the exact star pressure and post-shock density within 2%."""
    import numpy as np

    import oracle

    _need_gpu()
    print(f"[sod] {scheme} {precision}", flush=True)
    r = V.run_sod(scheme, precision)
    g, rl, pl, rr, pr = 1.4, 1.0, 1.0, r["rho_right"], 0.1795
    st, ps, us, _ = oracle.riemann(g, rl, 0.0, pl, rr, 0.0, pr)
    assert st == 0
    x = r["x"]
    w = (x > 0.25) & (x < 0.75)
    ex = np.array([oracle.riemann_sample(g, rl, 0.0, pl, rr, 0.0, pr, ps, us, (xi - 0.5) / r["t"])
                   for xi in x[w]])
    l1 = [float(np.mean(np.abs(a - b))) for a, b in
          ((r["rho"][w], ex[:, 0]), (r["vx"][w], ex[:, 1]), (r["P"][w], ex[:, 2]))]
    print(f"  {r['n']} particles, {r['steps']} steps, {r['wall_s']:.3f} s; "
          f"L1 rho {l1[0]:.4f}, vx {l1[1]:.4f}, P {l1[2]:.4f}", flush=True)
    assert abs(r["t"] - 0.13) <= 1e-12
    assert l1[0] <= bound and l1[1] <= 2.0 * bound and l1[2] <= bound
    # plateaus: the star pressure between the rarefaction tail and the
    # shock, the post-shock density between the contact and the shock
    star = (x > 0.50) & (x < 0.66)
    post = (x > 0.60) & (x < 0.66)
    shock_rho = oracle.riemann_sample(g, rl, 0.0, pl, rr, 0.0, pr, ps, us, (0.63 - 0.5) / r["t"])[0]
    assert abs(np.median(r["P"][star]) - ps) <= 0.02 * ps
    assert abs(np.median(r["rho"][post]) - shock_rho) <= 0.02 * shock_rho


def _radial_peak(r, bins_per_unit=128):
    """Radius and value of the largest mean density in shells around the
    blast particle's start position (periodic separations)."""
    import numpy as np

    c = np.array(r["center"])
    d = np.stack([r["x"], r["y"], r["z"]]) - c[:, None]
    d -= np.round(d)
    rad = np.sqrt((d ** 2).sum(0))
    b = np.floor(rad * bins_per_unit).astype(int)
    s = np.bincount(b, weights=r["rho"])
    k = np.bincount(b)
    prof = np.where(k > 0, s / np.maximum(k, 1), 0.0)[: bins_per_unit // 2]
    i = int(np.argmax(prof))
    return (i + 0.5) / bins_per_unit, float(prof[i])


@pytest.mark.parametrize("scheme,precision", [("mfm", "fp64"), ("mfv", "fp64"),
                                              ("mfm", "mixed")])
def test_sedov_point_explosion(scheme, precision):
    """The paper's Sedov test (sec. 3.1.5): unit energy in one particle of a
    uniform 64^3 lattice, to t = 0.1.  The shell's radius against the
    Sedov-Taylor radius 1.15167 (E t^2 / rho)^(1/5) (gamma = 5/3), its
    density contrast (the exact value is 4; the paper reaches ~2.7), and
    total energy to roundoff, in both precisions (the mixed path adds every
    FP32 face contribution to both sides in FP64).  Observed on MI355X: MFM
    301 steps in 1.5 s, peak 2.96 at R = 0.449 (R_ST 0.459); MFV 618 steps,
    3.02 at 0.457; MFM mixed 302 steps, 2.99 at 0.449; energy drift below
    5e-16 in all three."""
    _need_gpu()
    print(f"[sedov] {scheme} {precision} 64^3 to t = 0.1", flush=True)
    r = V.run_sedov(scheme, precision, n=64, t_end=0.1, progress=100)
    R, peak = _radial_peak(r)
    R_st = 1.15167 * (1.0 * r["t"] ** 2) ** 0.2
    drift = abs(r["energy1"] - r["energy0"]) / r["energy0"]
    print(f"  {r['steps']} steps, {r['wall_s']:.2f} s; peak density {peak:.3f} at R = {R:.4f} "
          f"(Sedov-Taylor {R_st:.4f}); energy drift {drift:.1e}", flush=True)
    assert abs(r["t"] - 0.1) <= 1e-12
    assert drift <= 1e-12
    assert 0.93 * R_st <= R <= 1.05 * R_st
    assert 2.4 <= peak <= 4.0


def test_sedov_32_stays_finite():
    """The same explosion on a 32^3 lattice to t = 0.1, where a cavity of a
    few particles forms next to the blast particle.  Under the dual-energy
    switch tested on the integrated U this run turned non-finite near
    t = 0.09; with the test on E - E_kin (and the positivity guard) it runs
    through with total energy conserved (observed: 148 steps, peak 2.45 at
    R = 0.430, drift 2e-16)."""
    _need_gpu()
    print("[sedov] mfm fp64 32^3 to t = 0.1", flush=True)
    r = V.run_sedov("mfm", "fp64", n=32, t_end=0.1, progress=100)
    drift = abs(r["energy1"] - r["energy0"]) / r["energy0"]
    R, peak = _radial_peak(r, bins_per_unit=64)
    R_st = 1.15167 * (1.0 * r["t"] ** 2) ** 0.2
    print(f"  {r['steps']} steps, {r['wall_s']:.2f} s; peak density {peak:.3f} at R = {R:.4f} "
          f"(Sedov-Taylor {R_st:.4f}); energy drift {drift:.1e}", flush=True)
    import numpy as np

    assert abs(r["t"] - 0.1) <= 1e-12
    assert all(np.isfinite(r[k]).all() for k in ("x", "y", "z", "rho", "vx", "vy", "vz"))
    assert drift <= 1e-12
    assert 0.85 * R_st <= R <= 1.1 * R_st


@pytest.mark.parametrize("scheme,precision", [("mfm", "fp64"), ("mfv", "fp64"),
                                              ("mfm", "mixed")])
def test_gresho_vortex(scheme, precision):
    """The paper's Gresho-Chan vortex (sec. 3.1.3): 64^2 particles per plane
    of side 2 on a Cartesian grid, 8 planes, both limiters, t = 3 (2.4 orbits
    of the peak).  The tangential velocity about the centre against the
    initial profile, which the exact solution keeps: observed L1 0.087 (MFM)
    and 0.084 (MFV) over r < 0.5 (MFM mixed: 0.087), the binned peak down
    from 1 to 0.69 for all three.  Most of that decay is the pairwise limiter's (0.74 with it alone,
    1.11 with the Barth-Jespersen limiter alone, 1.20 and a noisy profile
    with neither)."""
    import numpy as np

    from paper_2211_12243_amd import workloads as W

    _need_gpu()
    print(f"[gresho] {scheme} {precision}", flush=True)
    r = V.run_gresho(scheme, precision, progress=500)
    w = r["r"] < 0.5
    l1 = float(np.mean(np.abs(r["vphi"][w] - W.gresho_vphi(r["r"][w]))))
    b = np.floor(r["r"][w] / 0.02).astype(int)
    prof = np.bincount(b, weights=r["vphi"][w]) / np.maximum(np.bincount(b), 1)
    print(f"  {r['steps']} steps, {r['wall_s']:.2f} s; L1 v_phi {l1:.4f}, peak {prof.max():.3f} "
          f"at r = {(np.argmax(prof) + 0.5) * 0.02:.2f}", flush=True)
    assert abs(r["t"] - 3.0) <= 1e-12
    assert l1 <= 0.12
    assert prof.max() >= 0.6
    assert 0.14 <= (np.argmax(prof) + 0.5) * 0.02 <= 0.26
