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
