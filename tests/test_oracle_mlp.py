"""Pins of the FP64 guess-network reference (oracle/mlp.py), CPU only."""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import mlp

HERE = os.path.dirname(os.path.abspath(__file__))


def _random_case(seed, n=8):
    rng = np.random.default_rng(seed)
    p = mlp.unpack(mlp.init_params(seed))
    for b in ("b1", "b2", "b3"):
        p[b][:] = rng.normal(0, 0.3, mlp.HID)
    p["b4"][:] = 0.2
    params = mlp.pack(p)
    X = rng.normal(0, 1.5, (n, mlp.NIN))
    t = rng.normal(0, 1.0, n)
    norm = mlp.norm_from(X, t)
    return params, norm, X, t


@pytest.mark.parametrize("seed", [1, 2])
def test_gradient_matches_central_differences(seed):
    params, norm, X, t = _random_case(seed)
    loss, g = mlp.loss_grad(params, norm, X, t)
    rng = np.random.default_rng(100 + seed)
    idx = np.concatenate([rng.choice(mlp.NPARAM, 300, replace=False),
                          [mlp.NPARAM - 1, 0, 6 * mlp.HID + 3]])  # b4, W1[0,0], W1 padding row
    h = 1e-6
    fd = np.empty(idx.size)
    for q, k in enumerate(idx):
        pp, pm = params.copy(), params.copy()
        pp[k] += h
        pm[k] -= h
        fd[q] = (mlp.loss_grad(pp, norm, X, t)[0] - mlp.loss_grad(pm, norm, X, t)[0]) / (2 * h)
    scale = np.abs(g).max()
    assert np.abs(fd - g[idx]).max() <= 1e-6 * scale
    assert g[6 * mlp.HID + 3] == 0.0  # padding rows of W1 see zero inputs
    assert loss > 0


def test_single_path_network_by_hand():
    """One non-zero weight per layer: the output is a nested scalar
    expression, evaluated here with the math module.  A transposed or shifted
    weight matrix routes the signal elsewhere and gives b4 instead."""
    d = {k: np.zeros(s) for k, s in mlp.SHAPES}
    a_, b_, c_, w_, e_ = 0.7, -1.3, 0.9, 1.7, 0.25
    d["W1"][2, 5] = a_
    d["W2"][5, 7] = b_
    d["W3"][7, 3] = c_
    d["w4"][3] = w_
    d["b4"][0] = e_
    params = mlp.pack(d)
    norm = np.zeros(16)
    norm[:6] = [0.1, 0.2, 0.3, 0.4, 0.5, 0.6]
    norm[6:12] = [1.0, 2.0, 4.0, 1.0, 1.0, 1.0]
    norm[12], norm[13] = -0.5, 3.0
    x = np.array([[9.0, 9.0, 2.3, 9.0, 9.0, 9.0]])

    def s(z):
        return z / (1.0 + math.exp(-z))

    xs = (2.3 - 0.3) / 4.0
    ref = -0.5 + 3.0 * (e_ + w_ * s(c_ * s(b_ * s(a_ * xs))))
    assert abs(mlp.forward(params, norm, x)[0] - ref) <= 1e-15 * abs(ref)


def test_silu_derivative_against_differences():
    z = np.linspace(-6, 6, 49)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.abs(fd - mlp.dsilu(z)).max() < 1e-8
    assert mlp.silu(0.0) == 0.0
    assert abs(mlp.silu(1.0) - 1.0 / (1.0 + math.exp(-1.0))) < 1e-16


def test_bf16_rounding_ties_to_even():
    one = 1.0
    vals = np.array([one, one + 2.0**-8, one + 3 * 2.0**-8, one + 2.0**-8 + 2.0**-20, -2.5,
                     3.0e-39 * 0 + 1e-30])
    r = mlp.bf16(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                    # halfway, even neighbour is 1
    assert r[2] == 1.0 + 2.0**-6          # halfway, even neighbour is 1 + 2^-6
    assert r[3] == 1.0 + 2.0**-7          # above halfway
    assert r[4] == -2.5
    assert abs(r[5] - 1e-30) <= 2.0**-8 * 1e-30


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    p1, m1, v1 = mlp.adam(p, g, m, v, 1, 1e-2)
    # bias correction makes the first step lr * g / (|g| + eps)
    assert np.allclose(p - p1, 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    # a constant gradient keeps the step at lr (m_hat = g, v_hat = g^2)
    p2, _, _ = mlp.adam(p1, g, m1, v1, 2, 1e-2)
    assert np.allclose(p1 - p2, 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def _guess(g, rL, uL, pL, rR, uR, pR):
    out = [oracle.riemann_guess(g, *s, with_branch=True) for s in zip(rL, uL, pL, rR, uR, pR)]
    return np.array([o[0] for o in out]), np.array([o[1] for o in out])


def test_feature_mirror_symmetry():
    """The mirrored problem (left and right swapped, velocities reversed) has
    the same p*, the same velocity jump and the same starting value and
    branch: only the two ratios change sign.  Identical states at rest give
    zero features (the primitive-variable estimate is their pressure)."""
    rng = np.random.default_rng(9)
    rL, rR, pL, pR = rng.uniform(0.1, 3, (4, 20))
    uL, uR = rng.normal(0, 2, (2, 20))
    g = 5.0 / 3.0
    cL, cR = np.sqrt(g * pL / rL), np.sqrt(g * pR / rR)
    p0, b = _guess(g, rL, uL, pL, rR, uR, pR)
    p0m, bm = _guess(g, rR, -uR, pR, rL, -uL, pL)
    np.testing.assert_allclose(p0m, p0, rtol=1e-14)
    assert np.array_equal(bm, b)
    f = mlp.features(rL, pL, rR, pR, uR - uL, cL, cR, p0, b)
    m = mlp.features(rR, pR, rL, pL, (-uL) - (-uR), cR, cL, p0m, bm)
    np.testing.assert_allclose(m, np.stack([-f[:, 0], -f[:, 1], f[:, 2], f[:, 3], f[:, 4],
                                            f[:, 5]], axis=1), rtol=1e-13, atol=1e-15)
    assert set(np.unique(b)) >= {1, 2}  # both outer estimates occur in the sample
    p0s, bs = _guess(g, rL, 0 * uL, pL, rL, 0 * uL, pL)
    same = mlp.features(rL, pL, rL, pL, 0 * uL, cL, cL, p0s, bs)
    assert np.all(same == 0.0)


def test_target_of_printed_sod_solution():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "toro_exact_riemann.txt"))
            if l.strip() and not l.startswith("#")]
    for r in rows:
        rhoL, uL, PL, rhoR, uR, PR, pstar = map(float, r[1:8])
        st, ps, _, _ = oracle.riemann(1.4, rhoL, uL, PL, rhoR, uR, PR)
        assert st == 0
        y = math.log(ps / (0.5 * (PL + PR)))
        # five printed digits: relative error of p* below 1e-4
        assert abs(y - math.log(pstar / (0.5 * (PL + PR)))) < 1e-4
