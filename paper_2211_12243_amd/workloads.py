"""Seeded synthetic particle sets shaped like the paper's hydro tests.

This module only draws inputs: positions, masses, velocities and energies.  It
holds none of the hydro method's arithmetic, and both the GPU library's tests
and the CPU oracle's tests take their inputs from here.

Recipes (all in a periodic unit box, lattice spacing D = 1/n, each particle at
((i, j, k) + 1/2) D plus a seeded uniform jitter of up to 0.1 D per axis):

* ``sod``    -- planar jump at x = 0.5 of the unjittered lattice: density 1 |
  0.125 set through the particle mass, pressure 1 | 0.1, at rest (a Sod-like
  shock tube, cf. sec. 3.1.2).
* ``kh``     -- shear layers: density 2 for |y - 0.5| < 0.25 (through the mass),
  1 outside; vx = +0.5 inside, -0.5 outside; vy = 0.01 sin(4 pi x); P = 2.5.
* ``sedov``  -- uniform density 1 and pressure 1e-6; a unit energy added to the
  internal energy of the 33 particles nearest the box centre with cubic-spline
  weights of support equal to the distance of the 34th nearest (cf. sec. 3.1.5).
* ``uniform`` -- uniform gas (density 1, pressure 1), optional bulk velocity;
  with ``jitter = 0`` a perfect lattice.
* ``soundwave`` -- a linear sound wave along x (sec. 3.1.1): an unjittered
  lattice of N particles along x and ``nyz`` across y and z, in the periodic
  box (1, nyz / N, nyz / N); density 1 + A cos(2 pi x) through the particle
  mass, vx = A c cos(2 pi x), pressure 1 + A gamma cos(2 pi x), with
  c = sqrt(gamma) (unit background density and pressure).  Not cubic: its box
  comes from ``soundwave_box``.
* ``sod_tube`` -- the paper's shock tube (sec. 3.1.2): (rho, v, P) = (1, 0, 1)
  for x < 0.5 and (0.25, 0, 0.1795) beyond, gamma = 1.4, the density jump set
  by the number density of equal-mass particles (an unjittered lattice of
  spacing D = 0.5 / nx_left on the left; on the right ``k_right`` particles
  across and the x spacing that gives a quarter of the left number density,
  rounded to whole layers, so the right density is within a few per cent of
  0.25 and is returned exactly).  The box is periodic, so a mirrored tube sits
  at x = 0; its box comes from ``sod_tube_box``.
* ``sedov_point`` -- the paper's Sedov validation set (sec. 3.1.5): an
  unjittered n^3 lattice of density 1, gamma 5/3, a background of total
  energy E0 = 1e-5 spread evenly, and unit internal energy in one particle,
  the one at lattice index (n/2, n/2, n/2) (the lattice has no particle at
  the exact centre).
* ``gresho`` -- the paper's Gresho-Chan vortex (sec. 3.1.3): an unjittered
  lattice of n x n particles per plane of side 2 and ``nz`` planes, centred
  on (1, 1); v_phi = 5r (r <= 0.2), 2 - 5r (0.2 < r < 0.4), 0 beyond;
  density 1, gamma 1.4, and the pressure of hydrostatic equilibrium with
  p(0) = 5: 5 + 12.5 r^2, then 9 + 12.5 r^2 - 20 r + 4 ln(5 r), then
  3 + 4 ln 2.  Its box comes from ``gresho_box``.
* ``clustered`` -- log-normal density field with a k^-2 spectrum, particles
  Poisson-sampled per grid cell, Zel'dovich-like velocities (a stand-in for the
  clustered cosmological gas the paper's scaling runs use, which are not
  available here).

A state is a dict of float64 numpy arrays: x, y, z, vx, vy, vz, m, E, U, H with
E and U extensive (total and internal energy of the particle).  H is a start
value for the smoothing-length solve: the support radius that encloses n_ngb
particles at the mean number density.
"""
from __future__ import annotations

import math

import numpy as np


def _lattice(n: int, jitter: float, rng: np.random.Generator):
    D = 1.0 / n
    g = (np.arange(n, dtype=np.float64) + 0.5) * D
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    lat = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    pos = lat.copy()
    if jitter > 0:
        pos += rng.uniform(-jitter * D, jitter * D, size=pos.shape)
    pos = np.mod(pos, 1.0)
    pos[pos >= 1.0] -= 1.0
    return lat, pos, D


def _finish(pos, m, v, P, gamma, rho_nominal, n_ngb, N):
    U = m * P / ((gamma - 1.0) * rho_nominal)
    E = U + 0.5 * m * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2)
    H0 = (3.0 * n_ngb / (4.0 * math.pi * N)) ** (1.0 / 3.0)
    return {
        "x": pos[0].copy(), "y": pos[1].copy(), "z": pos[2].copy(),
        "vx": v[0].copy(), "vy": v[1].copy(), "vz": v[2].copy(),
        "m": m, "E": E, "U": U, "H": np.full(N, H0),
    }


def sod(n: int = 16, seed: int = 1, gamma: float = 5.0 / 3.0, n_ngb: float = 32.0,
        jitter: float = 0.1, rho=(1.0, 0.125), P=(1.0, 0.1)):
    rng = np.random.default_rng(seed)
    lat, pos, D = _lattice(n, jitter, rng)
    N = pos.shape[1]
    left = lat[0] < 0.5
    rho_n = np.where(left, rho[0], rho[1])
    Pn = np.where(left, P[0], P[1])
    m = rho_n * D ** 3
    v = np.zeros((3, N))
    return _finish(pos, m, v, Pn, gamma, rho_n, n_ngb, N)


def soundwave_box(N: int, nyz: int = 8):
    """The periodic box of ``soundwave(N, nyz)``: unit length along x."""
    return (1.0, nyz / N, nyz / N)


def soundwave(N: int = 32, nyz: int = 8, A: float = 1e-3, gamma: float = 1.4,
              n_ngb: float = 32.0):
    D = 1.0 / N
    gx = (np.arange(N, dtype=np.float64) + 0.5) * D
    gy = (np.arange(nyz, dtype=np.float64) + 0.5) * D
    X, Y, Z = np.meshgrid(gx, gy, gy, indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    n = pos.shape[1]
    cs = math.sqrt(gamma)
    wave = np.cos(2.0 * math.pi * pos[0])
    rho = 1.0 + A * wave
    P = 1.0 + A * gamma * wave
    v = np.zeros((3, n))
    v[0] = A * cs * wave
    m = rho * D ** 3
    st = _finish(pos, m, v, P, gamma, rho, n_ngb, n)
    # _finish sizes H for n particles in a unit volume; here the number
    # density is N^3
    st["H"] = np.full(n, (3.0 * n_ngb / (4.0 * math.pi)) ** (1.0 / 3.0) * D)
    return st


def sod_tube_box(nx_left: int = 100, nyz: int = 16):
    """The periodic box of ``sod_tube(nx_left, nyz)``: unit length along x."""
    T = nyz * 0.5 / nx_left
    return (1.0, T, T)


def sod_tube(nx_left: int = 100, nyz: int = 16, k_right: int = 10, gamma: float = 1.4,
             n_ngb: float = 64.0, rho=(1.0, 0.25), P=(1.0, 0.1795)):
    """Returns (state, rho_right): the right density the lattice realises."""
    D = 0.5 / nx_left
    T = nyz * D
    m = rho[0] * D ** 3
    dy_r = T / k_right
    n_r = max(1, int(round(0.5 / (m / (rho[1] * dy_r ** 2)))))
    dx_r = 0.5 / n_r
    rho_r = m / (dx_r * dy_r ** 2)
    gl = (np.arange(nyz, dtype=np.float64) + 0.5) * D
    X, Y, Z = np.meshgrid((np.arange(nx_left, dtype=np.float64) + 0.5) * D, gl, gl, indexing="ij")
    gr = (np.arange(k_right, dtype=np.float64) + 0.5) * dy_r
    Xr, Yr, Zr = np.meshgrid(0.5 + (np.arange(n_r, dtype=np.float64) + 0.5) * dx_r, gr, gr,
                             indexing="ij")
    pos = np.concatenate([np.stack([X.ravel(), Y.ravel(), Z.ravel()]),
                          np.stack([Xr.ravel(), Yr.ravel(), Zr.ravel()])], axis=1)
    n = pos.shape[1]
    left = pos[0] < 0.5
    rho_n = np.where(left, rho[0], rho_r)
    Pn = np.where(left, P[0], P[1])
    masses = np.full(n, m)
    st = _finish(pos, masses, np.zeros((3, n)), Pn, gamma, rho_n, n_ngb, n)
    st["H"] = (3.0 * n_ngb * masses / (4.0 * math.pi * rho_n)) ** (1.0 / 3.0)
    return st, rho_r


def sedov_point(n: int = 64, gamma: float = 5.0 / 3.0, n_ngb: float = 32.0, E0: float = 1e-5,
                E_blast: float = 1.0):
    """Returns (state, index of the blast particle)."""
    lat, pos, D = _lattice(n, 0.0, np.random.default_rng(0))
    N = pos.shape[1]
    m = np.full(N, D ** 3)
    st = _finish(pos, m, np.zeros((3, N)), np.zeros(N), gamma, np.ones(N), n_ngb, N)
    st["U"] = np.full(N, E0 / N)
    c = (n // 2) * n * n + (n // 2) * n + n // 2
    st["U"][c] = E_blast
    st["E"] = st["U"].copy()
    return st, c


def gresho_box(n: int = 64, nz: int = 8):
    """The periodic box of ``gresho(n, nz)``."""
    return (2.0, 2.0, nz * 2.0 / n)


def gresho_vphi(r):
    """The vortex's tangential velocity profile."""
    r = np.asarray(r, dtype=np.float64)
    return np.where(r <= 0.2, 5.0 * r, np.where(r < 0.4, 2.0 - 5.0 * r, 0.0))


def gresho(n: int = 64, nz: int = 8, gamma: float = 1.4, n_ngb: float = 32.0):
    D = 2.0 / n
    g = (np.arange(n, dtype=np.float64) + 0.5) * D
    gz = (np.arange(nz, dtype=np.float64) + 0.5) * D
    X, Y, Z = np.meshgrid(g, g, gz, indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    N = pos.shape[1]
    dx, dy = pos[0] - 1.0, pos[1] - 1.0
    r = np.sqrt(dx * dx + dy * dy)
    vphi = gresho_vphi(r)
    rs = np.where(r > 0.0, r, 1.0)
    v = np.zeros((3, N))
    v[0] = -vphi * dy / rs
    v[1] = vphi * dx / rs
    mid = 9.0 + 12.5 * r * r - 20.0 * r + 4.0 * np.log(np.maximum(5.0 * r, 1e-300))
    P = np.where(r <= 0.2, 5.0 + 12.5 * r * r, np.where(r < 0.4, mid, 3.0 + 4.0 * math.log(2.0)))
    m = np.full(N, D ** 3)
    st = _finish(pos, m, v, P, gamma, np.ones(N), n_ngb, N)
    st["H"] = np.full(N, (3.0 * n_ngb / (4.0 * math.pi)) ** (1.0 / 3.0) * D)
    return st


def kh(n: int = 64, seed: int = 2, gamma: float = 5.0 / 3.0, n_ngb: float = 32.0,
       jitter: float = 0.1, P: float = 2.5):
    rng = np.random.default_rng(seed)
    lat, pos, D = _lattice(n, jitter, rng)
    N = pos.shape[1]
    inside = np.abs(lat[1] - 0.5) < 0.25
    rho_n = np.where(inside, 2.0, 1.0)
    m = rho_n * D ** 3
    v = np.zeros((3, N))
    v[0] = np.where(inside, 0.5, -0.5)
    v[1] = 0.01 * np.sin(4.0 * math.pi * pos[0])
    Pn = np.full(N, P)
    return _finish(pos, m, v, Pn, gamma, rho_n, n_ngb, N)


def _spline_shape(q):
    """Cubic B-spline shape used only to spread the deposited blast energy."""
    q = np.asarray(q, dtype=np.float64)
    out = np.where(q < 0.5, 1.0 - 6.0 * q ** 2 + 6.0 * q ** 3, 2.0 * (1.0 - q) ** 3)
    return np.where(q < 1.0, out, 0.0)


def sedov(n: int = 128, seed: int = 3, gamma: float = 5.0 / 3.0, n_ngb: float = 32.0,
          jitter: float = 0.1, P0: float = 1e-6, E_blast: float = 1.0, n_dep: int = 33):
    rng = np.random.default_rng(seed)
    lat, pos, D = _lattice(n, jitter, rng)
    N = pos.shape[1]
    rho_n = np.ones(N)
    m = rho_n * D ** 3
    v = np.zeros((3, N))
    st = _finish(pos, m, v, np.full(N, P0), gamma, rho_n, n_ngb, N)
    d = pos - 0.5
    r = np.sqrt((d ** 2).sum(axis=0))
    order = np.lexsort((np.arange(N), r))  # by distance, ties by index
    near = order[:n_dep]
    h_dep = r[order[n_dep]]
    w = _spline_shape(r[near] / h_dep)
    w = w / w.sum()
    st["U"][near] += E_blast * w
    st["E"][near] += E_blast * w
    return st


def uniform(n: int = 16, seed: int = 0, gamma: float = 5.0 / 3.0, n_ngb: float = 32.0,
            jitter: float = 0.1, rho: float = 1.0, P: float = 1.0, v0=(0.0, 0.0, 0.0)):
    rng = np.random.default_rng(seed)
    lat, pos, D = _lattice(n, jitter, rng)
    N = pos.shape[1]
    m = np.full(N, rho * D ** 3)
    v = np.zeros((3, N))
    for k in range(3):
        v[k] += v0[k]
    return _finish(pos, m, v, np.full(N, P), gamma, np.full(N, rho), n_ngb, N)


def random_gas(N: int = 2000, seed: int = 0, gamma: float = 5.0 / 3.0, n_ngb: float = 32.0,
               box: float = 1.0):
    """Uniform random positions, random smooth-ish states (for parity tests)."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, box, size=(3, N))
    rho_n = rng.uniform(0.5, 2.0, size=N)
    m = rho_n * box ** 3 / N
    v = rng.normal(0.0, 0.3, size=(3, N))
    P = rng.uniform(0.5, 2.0, size=N)
    st = _finish(pos, m, v, P, gamma, rho_n, n_ngb, N)
    st["H"] *= box
    return st


def _h_from_cell_counts(counts, n_ngb, steps=(0, 1, 2, 3, 4, 6, 8, 12, 16, 24, 32)):
    """Start values of H (in cells) from the particle counts of a periodic
    grid: for each cell, the smallest cube of 2k + 1 cells around it that
    holds the number of particles a sphere of N_NGB neighbours needs
    (N_NGB * 6 / pi in the cube), with H scaled inside it as for uniform
    density.  Cells between clumps and voids take the clump into account,
    where the density of their own cell alone would not."""
    n = counts.shape[0]
    K = min(max(steps), (n - 1) // 2)
    cs = np.pad(counts.astype(np.int64), K, mode="wrap")
    for ax in range(3):
        cs = cs.cumsum(axis=ax)
    cs = np.pad(cs, ((1, 0), (1, 0), (1, 0)))
    target = n_ngb * 6.0 / math.pi
    H = np.full(counts.shape, np.nan)
    C = None
    for k in steps:
        if k > K:
            break
        a0, a1 = slice(K - k, K - k + n), slice(K + k + 1, K + k + 1 + n)
        C = (cs[a1, a1, a1] - cs[a0, a1, a1] - cs[a1, a0, a1] - cs[a1, a1, a0]
             + cs[a0, a0, a1] + cs[a0, a1, a0] + cs[a1, a0, a0] - cs[a0, a0, a0])
        pick = np.isnan(H) & (C >= target)
        H[pick] = (k + 0.5) * (target / C[pick]) ** (1.0 / 3.0)
        last = k
    rest = np.isnan(H)
    H[rest] = (last + 0.5) * (target / np.maximum(C[rest], 1)) ** (1.0 / 3.0)
    return H


def clustered(n: int = 256, seed: int = 4, gamma: float = 5.0 / 3.0, n_ngb: float = 32.0,
              sigma_ln: float = 1.5, vrms_over_cs: float = 10.0):
    """Log-normal clustered gas on an n^3 grid with N = n^3 particles in total."""
    rng = np.random.default_rng(seed)
    N = n ** 3
    k = np.fft.fftfreq(n, d=1.0 / n)
    KX, KY, KZ = np.meshgrid(k, k, k, indexing="ij")
    K2 = KX ** 2 + KY ** 2 + KZ ** 2
    K2[0, 0, 0] = 1.0
    white = rng.standard_normal((n, n, n))
    wk = np.fft.fftn(white)
    amp = 1.0 / np.sqrt(K2)  # sqrt of P(k) ~ k^-2
    amp[0, 0, 0] = 0.0
    dk = wk * amp
    delta = np.real(np.fft.ifftn(dk))
    delta /= delta.std()
    lnrho = sigma_ln * delta - 0.5 * sigma_ln ** 2
    rho = np.exp(lnrho)
    prob = (rho / rho.sum()).ravel()
    counts = rng.multinomial(N, prob)
    cells = np.repeat(np.arange(n ** 3), counts)
    ci = np.stack(np.unravel_index(cells, (n, n, n))).astype(np.float64)
    pos = (ci + rng.uniform(0.0, 1.0, size=ci.shape)) / n
    pos = np.mod(pos, 1.0)
    # Zel'dovich-like displacement field psi(k) = i k delta(k) / k^2 on the
    # grid (cell centres), interpolated trilinearly to the particles: a
    # continuous velocity field, so neighbours in one cell do not share a
    # velocity exactly
    g = pos * n - 0.5
    g0 = np.floor(g).astype(np.int64)
    f = g - g0
    vel = []
    for K in (KX, KY, KZ):
        psik = 1j * K * dk / K2
        psik[0, 0, 0] = 0.0
        field = np.real(np.fft.ifftn(psik))
        v = np.zeros(N)
        for cx in (0, 1):
            wx = f[0] if cx else 1.0 - f[0]
            ix = (g0[0] + cx) % n
            for cy in (0, 1):
                wy = f[1] if cy else 1.0 - f[1]
                iy = (g0[1] + cy) % n
                for cz in (0, 1):
                    wz = f[2] if cz else 1.0 - f[2]
                    v += wx * wy * wz * field[ix, iy, (g0[2] + cz) % n]
        vel.append(v)
    vel = np.stack(vel)
    u0 = 1.0 / (gamma * (gamma - 1.0))  # sound speed 1 in code units
    vrms = np.sqrt((vel ** 2).sum(axis=0).mean())
    vel *= vrms_over_cs / vrms
    m = np.full(N, 1.0 / N)
    U = m * u0
    E = U + 0.5 * m * (vel ** 2).sum(axis=0)
    # start values of H from the particle counts around each cell (an
    # initial condition carries its smoothing lengths)
    H = _h_from_cell_counts(counts.reshape(n, n, n), n_ngb).ravel()[cells] / n
    return {"x": pos[0].copy(), "y": pos[1].copy(), "z": pos[2].copy(),
            "vx": vel[0].copy(), "vy": vel[1].copy(), "vz": vel[2].copy(),
            "m": m, "E": E, "U": U, "H": H}


# The five configurations of the benchmark set, by name.
CONFIGS = {
    "sod16": dict(maker="sod", n=16, seed=1, scheme="mfv"),
    "kh64": dict(maker="kh", n=64, seed=2, scheme="mfv"),
    "sedov128": dict(maker="sedov", n=128, seed=3, scheme="mfm"),
    "clustered256": dict(maker="clustered", n=256, seed=4, scheme="mfm"),
}


def make(name: str, **over):
    spec = dict(CONFIGS[name])
    spec.update(over)
    maker = spec.pop("maker")
    spec.pop("scheme", None)
    return globals()[maker](**spec)


def params_for(name: str, **over) -> dict:
    """Plain-dict hydro parameters of a named configuration (gamma 5/3, N_NGB 32)."""
    cfg = {"scheme": CONFIGS[name]["scheme"], "gamma": 5.0 / 3.0, "n_ngb": 32.0,
           "box": (1.0, 1.0, 1.0)}
    cfg.update(over)
    return cfg
