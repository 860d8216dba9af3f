"""The sound-wave input set against its defining formulas (sec. 3.1.1)."""
import math

import numpy as np

from paper_2211_12243_amd import workloads as W


def test_soundwave_set():
    N, nyz, A, gamma = 16, 8, 1e-3, 1.4
    st = W.soundwave(N, nyz=nyz, A=A, gamma=gamma)
    box = W.soundwave_box(N, nyz)
    n = N * nyz * nyz
    assert box == (1.0, 0.5, 0.5)
    assert all(len(st[k]) == n for k in st)
    for k, L in zip("xyz", box):
        assert st[k].min() > 0.0 and st[k].max() < L
    D = 1.0 / N
    w = np.cos(2.0 * math.pi * st["x"])
    rho = 1.0 + A * w
    # mass over the lattice cell, the wave velocity, and the pressure through U
    assert np.allclose(st["m"], rho * D ** 3, rtol=0, atol=1e-15)
    assert np.allclose(st["vx"], A * math.sqrt(gamma) * w, rtol=0, atol=1e-15)
    assert not st["vy"].any() and not st["vz"].any()
    P = (gamma - 1.0) * st["U"] * rho / st["m"]
    assert np.allclose(P, 1.0 + A * gamma * w, rtol=1e-13, atol=0)
    kin = 0.5 * st["m"] * st["vx"] ** 2
    assert np.allclose(st["E"], st["U"] + kin, rtol=1e-15, atol=0)
    # the mean mass density is the background density
    assert abs(st["m"].sum() / (box[0] * box[1] * box[2]) - 1.0) < 1e-12
    # H encloses N_NGB lattice particles on average: (4 pi / 3) H^3 N^3 = 32
    assert abs(4.0 * math.pi / 3.0 * st["H"][0] ** 3 * N ** 3 - 32.0) < 1e-9


def test_sod_tube_set():
    st, rho_r = W.sod_tube()
    box = W.sod_tube_box()
    n = len(st["x"])
    assert box == (1.0, 0.08, 0.08)
    for k, L in zip("xyz", box):
        assert st[k].min() > 0.0 and st[k].max() < L
    # equal masses; the density jump through the number density
    assert np.all(st["m"] == st["m"][0])
    left = st["x"] < 0.5
    nl, nr = left.sum(), n - left.sum()
    vol = 0.5 * box[1] * box[2]
    assert abs(nl * st["m"][0] / vol - 1.0) < 1e-12
    assert abs(nr * st["m"][0] / vol - rho_r) < 1e-12
    assert abs(rho_r - 0.25) < 0.01
    rho = np.where(left, 1.0, rho_r)
    P = (1.4 - 1.0) * st["U"] * rho / st["m"]
    assert np.allclose(P, np.where(left, 1.0, 0.1795), rtol=1e-13, atol=0)
    assert not st["vx"].any() and np.array_equal(st["E"], st["U"])


def test_sedov_point_set():
    st, c = W.sedov_point(16)
    n = 16 ** 3
    assert len(st["x"]) == n
    # the blast particle is the lattice point (8, 8, 8) + 1/2, next to the centre
    assert (st["x"][c], st["y"][c], st["z"][c]) == (8.5 / 16, 8.5 / 16, 8.5 / 16)
    assert st["U"][c] == 1.0
    others = np.delete(st["U"], c)
    assert np.all(others == others[0]) and abs(others.sum() + others[0] - 1e-5) < 1e-18
    assert abs(st["m"].sum() - 1.0) < 1e-12
    assert np.array_equal(st["E"], st["U"]) and not st["vx"].any()


def test_gresho_set():
    st = W.gresho(32, 4)
    box = W.gresho_box(32, 4)
    assert box == (2.0, 2.0, 0.25) and len(st["x"]) == 32 * 32 * 4
    dx, dy = st["x"] - 1.0, st["y"] - 1.0
    r = np.sqrt(dx * dx + dy * dy)
    vphi = (dx * st["vy"] - dy * st["vx"]) / r
    assert np.allclose(vphi, W.gresho_vphi(r), rtol=0, atol=1e-14)
    assert np.allclose(dx * st["vx"] + dy * st["vy"], 0.0, atol=1e-14)
    P = 0.4 * st["U"] / st["m"]  # density 1
    # hydrostatic equilibrium: dP/dr = v_phi^2 / r, by finite differences of
    # the profile the set uses, and continuity at r = 0.2 and 0.4
    def prof(x):
        return np.where(x <= 0.2, 5.0 + 12.5 * x * x,
                        np.where(x < 0.4, 9.0 + 12.5 * x * x - 20.0 * x
                                 + 4.0 * np.log(np.maximum(5.0 * x, 1e-300)),
                                 3.0 + 4.0 * math.log(2.0)))
    assert np.allclose(P, prof(r), rtol=1e-13, atol=0)
    for x in (0.05, 0.15, 0.25, 0.35, 0.45):
        h = 1e-6
        dP = (prof(x + h) - prof(x - h)) / (2 * h)
        assert abs(dP - W.gresho_vphi(x) ** 2 / x) < 1e-6
    for x in (0.2, 0.4):
        assert abs(prof(x - 1e-12) - prof(x + 1e-12)) < 1e-9
    assert abs(prof(0.0) - 5.0) < 1e-15
