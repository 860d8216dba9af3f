"""Pins of the oracle's exact Riemann solver (Toro's solver, sec. 2.3.3).

Closed forms that do not use the solver's own code paths: identical states,
the two-rarefaction formula (exact when p* is below both pressures), the
symmetric two-shock quadratic, the vacuum condition, mirror symmetry, the
Rankine-Hugoniot conditions across a sampled shock and the Riemann invariant
across a sampled rarefaction, and two printed textbook solutions.
"""
import math
import os

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def test_identical_states():
    for g in (1.4, 5.0 / 3.0):
        st, ps, us, it = oracle.riemann(g, 1.3, 0.7, 2.2, 1.3, 0.7, 2.2)
        assert st == 0 and ps == 2.2 and us == pytest.approx(0.7, abs=1e-15)


@pytest.mark.parametrize("uL,uR,PL,PR", [(-1.0, 1.0, 1.0, 1.0), (-0.5, 1.2, 0.8, 1.5),
                                          (0.0, 2.0, 2.0, 0.6)])
def test_two_rarefaction_closed_form(uL, uR, PL, PR):
    g = 1.4
    rhoL, rhoR = 1.0, 0.7
    cL, cR = math.sqrt(g * PL / rhoL), math.sqrt(g * PR / rhoR)
    z = (g - 1) / (2 * g)
    p_tr = ((cL + cR - 0.5 * (g - 1) * (uR - uL)) / (cL / PL ** z + cR / PR ** z)) ** (1 / z)
    assert p_tr < min(PL, PR)  # both waves are rarefactions, so the formula is exact
    st, ps, us, it = oracle.riemann(g, rhoL, uL, PL, rhoR, uR, PR)
    assert st == 0
    assert ps == pytest.approx(p_tr, rel=1e-12)
    # velocity from the left rarefaction's Riemann invariant
    u_exp = uL - 2 * cL / (g - 1) * ((p_tr / PL) ** z - 1)
    assert us == pytest.approx(u_exp, rel=1e-10, abs=1e-12)


@pytest.mark.parametrize("U,rho,P", [(1.0, 1.0, 1.0), (5.0, 0.5, 0.2), (30.0, 1.0, 1e-3)])
def test_symmetric_collision_two_shock(U, rho, P):
    # equal states with u_L = U = -u_R: two shocks, u* = 0, and p* solves
    # (p - P)^2 A = U^2 (p + B), A = 2/((g+1) rho), B = (g-1) P/(g+1)
    g = 5.0 / 3.0
    A = 2 / ((g + 1) * rho)
    B = (g - 1) / (g + 1) * P
    # A p^2 - (2 A P + U^2) p + A P^2 - U^2 B = 0, larger root
    a, b, c = A, -(2 * A * P + U * U), A * P * P - U * U * B
    p_exp = (-b + math.sqrt(b * b - 4 * a * c)) / (2 * a)
    st, ps, us, it = oracle.riemann(g, rho, U, P, rho, -U, P)
    assert st == 0
    assert ps == pytest.approx(p_exp, rel=1e-12)
    assert abs(us) < 1e-12 * U


def test_vacuum_condition():
    g = 1.4
    cL = cR = math.sqrt(g)
    du_crit = 2 / (g - 1) * (cL + cR)
    st, *_ = oracle.riemann(g, 1, -0.5 * du_crit - 1e-9, 1, 1, 0.5 * du_crit + 1e-9, 1)
    assert st == 1
    st, *_ = oracle.riemann(g, 1, -0.5 * du_crit * 0.999, 1, 1, 0.5 * du_crit * 0.999, 1)
    assert st == 0


def test_mirror_symmetry():
    rng = np.random.default_rng(0)
    for _ in range(50):
        rL, rR = rng.uniform(0.1, 3, 2)
        PL, PR = 10 ** rng.uniform(-3, 2, 2)
        uL, uR = rng.normal(0, 1, 2)
        a = oracle.riemann(5 / 3, rL, uL, PL, rR, uR, PR)
        b = oracle.riemann(5 / 3, rR, -uR, PR, rL, -uL, PL)
        if a[0] == 1:
            assert b[0] == 1
            continue
        assert a[1] == pytest.approx(b[1], rel=1e-12)
        assert a[2] == pytest.approx(-b[2], rel=1e-9, abs=1e-12)


def test_printed_textbook_solutions():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "toro_exact_riemann.txt"))
            if l.strip() and not l.startswith("#")]
    for name, *vals in rows:
        rL, uL, PL, rR, uR, PR, ps_ref, us_ref = map(float, vals)
        st, ps, us, it = oracle.riemann(1.4, rL, uL, PL, rR, uR, PR)
        assert st == 0
        assert ps == pytest.approx(ps_ref, rel=2e-5), name
        assert us == pytest.approx(us_ref, rel=2e-5), name


def test_sampled_sod_satisfies_jump_conditions():
    # The paper's shock tube states (sec. 3.1.2): (1, 0, 1) | (0.25, 0, 0.1795), gamma 1.4
    g = 1.4
    rL, uL, PL, rR, uR, PR = 1.0, 0.0, 1.0, 0.25, 0.0, 0.1795
    st, ps, us, it = oracle.riemann(g, rL, uL, PL, rR, uR, PR)
    assert st == 0 and PR < ps < PL and us > 0
    # right shock: find its speed from the sampled profile and check mass and
    # momentum fluxes across it
    xis = np.linspace(us + 1e-6, 3.0, 20001)
    rho = np.array([oracle.riemann_sample(g, rL, uL, PL, rR, uR, PR, ps, us, x)[0] for x in xis])
    k = np.nonzero(rho <= rR * (1 + 1e-12))[0][0]
    S = 0.5 * (xis[k - 1] + xis[k])
    r2, u2, p2 = oracle.riemann_sample(g, rL, uL, PL, rR, uR, PR, ps, us, xis[k - 1])
    m1 = rR * (uR - S)
    m2 = r2 * (u2 - S)
    assert m1 == pytest.approx(m2, rel=2e-3)
    assert (m1 * uR + PR) == pytest.approx(m2 * u2 + p2, rel=2e-3)
    # left rarefaction: u + 2c/(g-1) is constant through the fan
    cL = math.sqrt(g * PL / rL)
    inv0 = uL + 2 * cL / (g - 1)
    for xi in np.linspace(uL - cL + 1e-6, us - math.sqrt(g * ps / (rL * (ps / PL) ** (1 / g))),
                          7):
        r, u, p = oracle.riemann_sample(g, rL, uL, PL, rR, uR, PR, ps, us, xi)
        assert u + 2 * math.sqrt(g * p / r) / (g - 1) == pytest.approx(inv0, rel=1e-12)
        assert p / r ** g == pytest.approx(PL / rL ** g, rel=1e-12)  # isentropic


def test_strong_pressure_ratio_converges():
    # Sedov-like faces: pressure ratios up to 1e11
    for ratio in (1e3, 1e7, 1e11):
        st, ps, us, it = oracle.riemann(5 / 3, 1.0, 0.0, ratio, 1.0, 0.0, 1.0)
        assert st == 0 and it < 30
        st2, ps2, us2, _ = oracle.riemann(5 / 3, 1.0, 0.0, 1.0, 1.0, 0.0, ratio)
        assert ps == pytest.approx(ps2, rel=1e-12)


@pytest.mark.parametrize("uL,uR,PL,PR", [(-1.0, 1.0, 1.0, 1.0), (-0.5, 1.2, 0.8, 1.5),
                                          (0.0, 2.0, 2.0, 0.6)])
def test_starting_value_is_exact_for_two_rarefactions(uL, uR, PL, PR):
    """Toro's adaptive starting value takes the two-rarefaction estimate
    when the primitive-variable one falls below both pressures; that
    estimate is the exact p* when both waves are rarefactions."""
    g = 1.4
    st, ps, _, _ = oracle.riemann(g, 1.0, uL, PL, 0.7, uR, PR)
    assert st == 0 and ps < min(PL, PR)
    assert oracle.riemann_guess(g, 1.0, uL, PL, 0.7, uR, PR) == pytest.approx(ps, rel=1e-12)


def test_starting_value_of_close_states():
    """Identical states at rest: the primitive-variable estimate is the
    common pressure.  A small pressure jump delta: its error is of second
    order (the estimate linearises the wave curves about the mean state), so
    halving delta divides it by about four."""
    g = 5.0 / 3.0
    assert oracle.riemann_guess(g, 1.2, 0.0, 0.9, 1.2, 0.0, 0.9) == 0.9
    err = []
    for d in (0.2, 0.1, 0.05):
        st, ps, _, _ = oracle.riemann(g, 1.0, 0.0, 1.0 + d, 1.0, 0.0, 1.0)
        assert st == 0
        err.append(abs(oracle.riemann_guess(g, 1.0, 0.0, 1.0 + d, 1.0, 0.0, 1.0) - ps) / ps)
    assert all(3.0 < a / b < 5.0 for a, b in zip(err, err[1:])), err


def test_starting_value_of_strong_shocks_and_floor():
    """Colliding flows (two shocks, p* above both pressures): the two-shock
    estimate, evaluated at the primitive-variable pressure, lies between the
    states' pressure and p*; within 10% of p* for a weak collision, while for
    hypersonic ones it falls far short (0.37 p* at Mach 7, 0.03 p* at Mach
    800) -- the faces where Newton needs the most steps.  Near vacuum the
    value is kept above the pressure floor 1e-10 (P_L + P_R) / 2."""
    g = 5.0 / 3.0
    for U, rho, P in ((1.0, 1.0, 1.0), (5.0, 0.5, 0.2), (30.0, 1.0, 1e-3)):
        st, ps, _, _ = oracle.riemann(g, rho, U, P, rho, -U, P)
        p0 = oracle.riemann_guess(g, rho, U, P, rho, -U, P)
        assert st == 0 and P < p0 < ps
        if U == 1.0:
            assert abs(p0 - ps) < 0.1 * ps
    c = math.sqrt(g)
    du = 2.0 / (g - 1.0) * 2 * c * (1 - 1e-9)  # just short of the vacuum condition
    p0 = oracle.riemann_guess(g, 1.0, -0.5 * du, 1.0, 1.0, 0.5 * du, 1.0)
    assert p0 >= 1e-10
