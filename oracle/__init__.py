"""FP64 CPU oracle of the MFV/MFM neighbour loops (arXiv 2211.12243, sec. 2.3).

TEST INFRASTRUCTURE ONLY.  This package is the independent checker that the GPU
library is compared against.  Only the tests, the smoke check and the CPU
baseline of the benchmark may import it; the product package never does.  It
shares no code with the HIP library: the arithmetic lives in ``mfm_oracle.c``
(plain C, FP64, compiled with gcc) and this module only marshals numpy arrays.

Pins (what fixes each function independently of itself) are in
``tests/test_oracle_*.py``.  Functions without such a pin are marked
"parity unpinned" in their docstring.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mfm_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
             "-ffp-contract=off", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("scheme", ctypes.c_int32), ("limiter", ctypes.c_int32),
        ("max_boosts", ctypes.c_int32), ("h_maxit", ctypes.c_int32),
        ("riemann_maxit", ctypes.c_int32), ("pad0", ctypes.c_int32),
        ("gamma", ctypes.c_double), ("n_ngb", ctypes.c_double),
        ("ncond_max", ctypes.c_double), ("ngb_boost", ctypes.c_double),
        ("h_tol", ctypes.c_double), ("c_cfl", ctypes.c_double),
        ("psi1", ctypes.c_double), ("psi2", ctypes.c_double),
        ("riemann_tol", ctypes.c_double), ("alpha1", ctypes.c_double),
        ("box", ctypes.c_double * 3),
        ("alpha2", ctypes.c_double), ("alpha3", ctypes.c_double),
        ("entropy_switch", ctypes.c_int32), ("pad1", ctypes.c_int32),
    ]


class Sources(ctypes.Structure):
    """Source terms of one step (sec. 2.3.7-2.3.9)."""
    _fields_ = [
        ("accel", ctypes.c_void_p), ("inv_a", ctypes.c_double),
        ("hubble_n", ctypes.c_double), ("hubble_np1", ctypes.c_double),
        ("S", ctypes.c_void_p), ("emode", ctypes.c_void_p),
    ]


class Counters(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "h_noconv", "ncond_boosts", "ncond_fail", "h_fallback", "grad_pairs", "faces",
        "riemann_iters", "riemann_maxit", "vacuum", "positivity", "neg_mass", "singular_e",
        "u_guard")]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


def make_params(cfg: dict) -> Params:
    """Build the oracle's parameter struct from a plain dict of values."""
    p = Params()
    p.scheme = 1 if cfg.get("scheme", "mfv") == "mfm" else 0
    p.limiter = int(cfg.get("limiter", 3))
    p.max_boosts = int(cfg.get("max_boosts", 5))
    p.h_maxit = int(cfg.get("h_maxit", 64))
    p.riemann_maxit = int(cfg.get("riemann_maxit", 100))
    p.gamma = float(cfg.get("gamma", 5.0 / 3.0))
    p.n_ngb = float(cfg.get("n_ngb", 32.0))
    p.ncond_max = float(cfg.get("ncond_max", 100.0))
    p.ngb_boost = float(cfg.get("ngb_boost", 1.2))
    p.h_tol = float(cfg.get("h_tol", 1e-13))
    p.c_cfl = float(cfg.get("c_cfl", 0.2))
    p.psi1 = float(cfg.get("psi1", 0.5))
    p.psi2 = float(cfg.get("psi2", 0.25))
    p.riemann_tol = float(cfg.get("riemann_tol", 1e-10))
    p.alpha1 = float(cfg.get("alpha1", 0.01))
    p.alpha2 = float(cfg.get("alpha2", 1e-3))
    p.alpha3 = float(cfg.get("alpha3", 1e-3))
    p.entropy_switch = int(cfg.get("entropy_switch", 0))
    box = cfg.get("box", (1.0, 1.0, 1.0))
    for k in range(3):
        p.box[k] = float(box[k])
    return p


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)
_I32 = ctypes.POINTER(ctypes.c_int32)


def lib():
    global _lib
    if _lib is None:
        # (re)build when the library is missing or older than its source
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


@contextlib.contextmanager
def use_library(path: str):
    """Run the oracle from another build of its source (the mutation tests
    check that the pins reject deliberately broken copies)."""
    global _lib
    saved = lib()
    _lib = _bind(ctypes.CDLL(path))
    try:
        yield
    finally:
        _lib = saved


def build_variant(src_text: str, out_path: str) -> str:
    """Compile C source text with the oracle's flags into out_path."""
    src = out_path + ".c"
    with open(src, "w") as fh:
        fh.write(src_text)
    subprocess.check_call(
        ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
         "-ffp-contract=off", "-I", _HERE, "-o", out_path, src, "-lm"])
    return out_path


def source() -> str:
    with open(_SRC) as fh:
        return fh.read()


def _bind(L):
    """Declare the argument and result types of the oracle's C functions."""
    P = ctypes.POINTER(Params)
    C = ctypes.POINTER(Counters)
    i64 = ctypes.c_int64
    L.orc_kernel_W.restype = ctypes.c_double
    L.orc_kernel_W.argtypes = [ctypes.c_double, ctypes.c_double]
    L.orc_neighbours.argtypes = [P, i64, _D, _D, _D, _D, ctypes.c_int, _I64, _I32]
    L.orc_density.argtypes = [P, i64, _D, _D, _D, _D, _D, _D, _D, C]
    L.orc_density_at.argtypes = [P, i64, _D, _D, _D, _D, i64, _I64, _D, _D, _D, _D, C]
    L.orc_gradients.argtypes = [P, i64] + [_D] * 10 + [_D] * 8 + [C]
    L.orc_riemann.argtypes = [ctypes.c_double] * 8 + [ctypes.c_int, _D, _D,
                                                        ctypes.POINTER(ctypes.c_int)]
    L.orc_riemann_sample.argtypes = [ctypes.c_double] * 10 + [_D, _D, _D]
    L.orc_riemann_guess.argtypes = [ctypes.c_double] * 7 + [ctypes.POINTER(ctypes.c_int)]
    L.orc_riemann_guess.restype = ctypes.c_double
    L.orc_face_list_copy.argtypes = [P, i64, _D, _D, _D, _D, i64, _I64, _I64, _I64]
    L.orc_face_list_copy.restype = ctypes.c_int
    L.orc_pair_limit.restype = ctypes.c_double
    L.orc_pair_limit.argtypes = [ctypes.c_double] * 5
    L.orc_face.argtypes = [P, i64, i64, i64] + [_D] * 12 + [ctypes.c_double, _D, C]
    L.orc_fluxes.argtypes = [P, i64] + [_D] * 12 + [ctypes.c_double, _D, _D, C]
    L.orc_update.argtypes = [P, i64] + [_D] * 9 + [_D, ctypes.c_double, C]
    L.orc_step.argtypes = [P, i64] + [_D] * 10 + [ctypes.c_double, _D, C]
    SP = ctypes.POINTER(Sources)
    L.orc_fluxes_src.argtypes = ([P, i64] + [_D] * 12 + [ctypes.c_double, ctypes.c_double, _D,
                                 _D, _D, C])
    L.orc_ekin_max.argtypes = [P, i64] + [_D] * 8
    L.orc_entropy_pressure.argtypes = [P, i64, _D, _D, _D, _D, _I32]
    L.orc_update_src.argtypes = ([P, i64] + [_D] * 9 + [_D, ctypes.c_double, SP, _D, _D, _D, _D,
                                 C])
    L.orc_step_src.argtypes = [P, i64] + [_D] * 10 + [ctypes.c_double, SP, _D, C]
    L.orc_rungs.argtypes = [P, i64, _D, _D, _D, _D, _D, ctypes.c_double, _I32]
    L.orc_step_rungs.argtypes = ([P, i64] + [_D] * 10 + [ctypes.c_double, _I32, ctypes.c_int,
                                                        _I64, C])
    for f in ("orc_fluxes_src", "orc_ekin_max", "orc_entropy_pressure", "orc_update_src",
              "orc_step_src", "orc_rungs", "orc_step_rungs"):
        getattr(L, f).restype = ctypes.c_int
    for f in ("orc_neighbours", "orc_density", "orc_density_at", "orc_gradients", "orc_riemann",
              "orc_riemann_sample", "orc_face", "orc_fluxes", "orc_update", "orc_step"):
        getattr(L, f).restype = ctypes.c_int
    return L


def _p(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def kernel_W(r: float, H: float) -> float:
    """Cubic-spline kernel with compact support H (sec. 2.3.2)."""
    return lib().orc_kernel_W(float(r), float(H))


def neighbours(cfg: dict, x, y, z, R, use_grid: bool = True):
    """Neighbour sets N_i = {j : |x_j - x_i| < R_i} as CSR (start, idx), self included."""
    p = make_params(cfg)
    x, y, z, R = (_f64(a) for a in (x, y, z, R))
    n = x.size
    start = np.zeros(n + 1, dtype=np.int64)
    L = lib()
    rc = L.orc_neighbours(ctypes.byref(p), n, _p(x), _p(y), _p(z), _p(R), int(use_grid),
                          start.ctypes.data_as(_I64), None)
    assert rc == 0
    idx = np.zeros(max(int(start[-1]), 1), dtype=np.int32)
    rc = L.orc_neighbours(ctypes.byref(p), n, _p(x), _p(y), _p(z), _p(R), int(use_grid),
                          start.ctypes.data_as(_I64), idx.ctypes.data_as(_I32))
    assert rc == 0
    return start, idx[: int(start[-1])]


def density(cfg: dict, x, y, z, H):
    """Loop (1): smoothing length, volume and unweighted condition number."""
    p = make_params(cfg)
    x, y, z = (_f64(a) for a in (x, y, z))
    H = _f64(H).copy()
    n = x.size
    V, nc, nngb = (np.empty(n) for _ in range(3))
    cnt = Counters()
    rc = lib().orc_density(ctypes.byref(p), n, _p(x), _p(y), _p(z), _p(H), _p(V), _p(nc),
                           _p(nngb), ctypes.byref(cnt))
    if rc:
        raise RuntimeError(f"orc_density failed: {rc}")
    return {"H": H, "V": V, "ncond_tilde": nc, "nngb": nngb}, cnt.as_dict()


def density_at(cfg: dict, x, y, z, H, idx):
    """Loop (1) for the particles idx only (every particle a candidate): the
    H, V, ncond and N_NGB that density() gives them."""
    p = make_params(cfg)
    x, y, z, H = (_f64(a) for a in (x, y, z, H))
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    nq = idx.size
    Ho, V, nc, nngb = (np.empty(nq) for _ in range(4))
    cnt = Counters()
    rc = lib().orc_density_at(ctypes.byref(p), x.size, _p(x), _p(y), _p(z), _p(H), nq,
                              idx.ctypes.data_as(_I64), _p(Ho), _p(V), _p(nc), _p(nngb),
                              ctypes.byref(cnt))
    if rc:
        raise RuntimeError(f"orc_density_at failed: {rc}")
    return {"H": Ho, "V": V, "ncond_tilde": nc, "nngb": nngb}, cnt.as_dict()


def gradients(cfg: dict, x, y, z, H, V, m, vx, vy, vz, U):
    """Loops (2) and (4): primitives, B = E^-1, limited gradients, dt_i."""
    p = make_params(cfg)
    arrs = [_f64(a) for a in (x, y, z, H, V, m, vx, vy, vz, U)]
    n = arrs[0].size
    rho, P, c, nc, dti = (np.empty(n) for _ in range(5))
    B = np.empty((6, n))
    grad = np.empty((15, n))
    alpha = np.empty((5, n))
    cnt = Counters()
    rc = lib().orc_gradients(ctypes.byref(p), n, *[_p(a) for a in arrs], _p(rho), _p(P), _p(c),
                             _p(B), _p(grad), _p(alpha), _p(nc), _p(dti), ctypes.byref(cnt))
    if rc:
        raise RuntimeError(f"orc_gradients failed: {rc}")
    return {"rho": rho, "P": P, "c": c, "B": B, "grad": grad, "alpha": alpha, "ncond": nc,
            "dt_i": dti}, cnt.as_dict()


def riemann(gamma, rhoL, uL, PL, rhoR, uR, PR, tol=1e-10, maxit=100):
    """Exact Riemann solve: returns (status, p*, u*, iterations)."""
    ps, us = ctypes.c_double(), ctypes.c_double()
    it = ctypes.c_int()
    st = lib().orc_riemann(float(gamma), float(rhoL), float(uL), float(PL), float(rhoR),
                           float(uR), float(PR), float(tol), int(maxit), ctypes.byref(ps),
                           ctypes.byref(us), ctypes.byref(it))
    return st, ps.value, us.value, it.value


def riemann_guess(gamma, rhoL, uL, PL, rhoR, uR, PR, with_branch=False):
    """Starting value of the exact solver's Newton iteration (Toro's adaptive
    choice, floored at 1e-10 of the mean pressure); with_branch: also the
    estimate it came from (0 primitive-variable, 1 two-rarefaction, 2
    two-shock)."""
    b = ctypes.c_int()
    p0 = lib().orc_riemann_guess(*(float(v) for v in (gamma, rhoL, uL, PL, rhoR, uR, PR)),
                                 ctypes.byref(b))
    return (p0, b.value) if with_branch else p0


def riemann_sample(gamma, rhoL, uL, PL, rhoR, uR, PR, ps, us, xi):
    """Exact solution at speed xi: returns (rho, u, P)."""
    r, u, P = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().orc_riemann_sample(*(float(v) for v in (gamma, rhoL, uL, PL, rhoR, uR, PR, ps, us, xi)),
                             ctypes.byref(r), ctypes.byref(u), ctypes.byref(P))
    return r.value, u.value, P.value


def pair_limit(qf, qo, qn, psi1=0.5, psi2=0.25):
    """Pairwise limiter of face value qf from the own side qo towards qn (sec. 2.3.6)."""
    return lib().orc_pair_limit(float(qf), float(qo), float(qn), float(psi1), float(psi2))


def face(cfg: dict, i, j, x, y, z, H, V, rho, vx, vy, vz, P, B, grad, dt):
    """Contribution c = |A_ij| F_ij of one face, oriented from i to j."""
    p = make_params(cfg)
    arrs = [_f64(a) for a in (x, y, z, H, V, rho, vx, vy, vz, P)]
    B = _f64(B)
    grad = _f64(grad)
    n = arrs[0].size
    c = np.zeros(5)
    cnt = Counters()
    lib().orc_face(ctypes.byref(p), n, int(i), int(j), *[_p(a) for a in arrs], _p(B), _p(grad),
                   float(dt), _p(c), ctypes.byref(cnt))
    return c, cnt.as_dict()


def fluxes_face_list(cfg: dict, x, y, z, H):
    """The flux loop's faces {i, j}, r_ij < max(H_i, H_j), as (lower, higher) index arrays."""
    p = make_params(cfg)
    x, y, z, H = (_f64(a) for a in (x, y, z, H))
    nf = ctypes.c_int64()
    L = lib()
    rc = L.orc_face_list_copy(ctypes.byref(p), x.size, _p(x), _p(y), _p(z), _p(H), 0, None,
                              None, ctypes.byref(nf))
    assert rc == 0
    fa = np.zeros(max(nf.value, 1), dtype=np.int64)
    fb = np.zeros(max(nf.value, 1), dtype=np.int64)
    rc = L.orc_face_list_copy(ctypes.byref(p), x.size, _p(x), _p(y), _p(z), _p(H), nf.value,
                              fa.ctypes.data_as(_I64), fb.ctypes.data_as(_I64), ctypes.byref(nf))
    assert rc == 0
    return fa[:nf.value], fb[:nf.value]


def fluxes(cfg: dict, x, y, z, H, V, rho, vx, vy, vz, P, B, grad, dt):
    """Loop (3): dQ (5, n) and its per-component scale dt * sum_j |c_ij|."""
    p = make_params(cfg)
    arrs = [_f64(a) for a in (x, y, z, H, V, rho, vx, vy, vz, P)]
    B = _f64(B)
    grad = _f64(grad)
    n = arrs[0].size
    dQ = np.empty((5, n))
    scale = np.empty((5, n))
    cnt = Counters()
    rc = lib().orc_fluxes(ctypes.byref(p), n, *[_p(a) for a in arrs], _p(B), _p(grad), float(dt),
                          _p(dQ), _p(scale), ctypes.byref(cnt))
    if rc:
        raise RuntimeError(f"orc_fluxes failed: {rc}")
    return {"dQ": dQ, "scale": scale}, cnt.as_dict()


def update(cfg: dict, state: dict, dQ, dt):
    """Close of the step on a copy of ``state`` (keys x,y,z,m,vx,vy,vz,E,U)."""
    p = make_params(cfg)
    s = {k: _f64(state[k]).copy() for k in ("x", "y", "z", "m", "vx", "vy", "vz", "E", "U")}
    n = s["x"].size
    dQ = _f64(dQ)
    cnt = Counters()
    rc = lib().orc_update(ctypes.byref(p), n, *[_p(s[k]) for k in
                                                ("x", "y", "z", "m", "vx", "vy", "vz", "E", "U")],
                          _p(dQ), float(dt), ctypes.byref(cnt))
    if rc:
        raise RuntimeError(f"orc_update failed: {rc}")
    return s, cnt.as_dict()


STATE_KEYS = ("x", "y", "z", "m", "vx", "vy", "vz", "E", "U", "H")


def step(cfg: dict, state: dict, dt_max: float):
    """One full step on a copy of ``state``; returns (new_state, dt, counters)."""
    p = make_params(cfg)
    s = {k: _f64(state[k]).copy() for k in STATE_KEYS}
    n = s["x"].size
    dt = ctypes.c_double()
    cnt = Counters()
    rc = lib().orc_step(ctypes.byref(p), n, *[_p(s[k]) for k in STATE_KEYS], float(dt_max),
                        ctypes.byref(dt), ctypes.byref(cnt))
    if rc:
        raise RuntimeError(f"orc_step failed: {rc}")
    return s, dt.value, cnt.as_dict()


RUNG_MAX = 30


def rungs(cfg: dict, x, y, z, H, dt_i, dt0: float):
    """Rungs from the particles' own steps dt_i (sec. 2.3.10) with the
    |r_i - r_j| <= 2 limiter over the flux pairs at H."""
    p = make_params(cfg)
    x, y, z, H, dt_i = (_f64(a) for a in (x, y, z, H, dt_i))
    r = np.zeros(x.size, dtype=np.int32)
    rc = lib().orc_rungs(ctypes.byref(p), x.size, _p(x), _p(y), _p(z), _p(H), _p(dt_i),
                         float(dt0), r.ctypes.data_as(_I32))
    if rc:
        raise RuntimeError(f"orc_rungs failed: {rc}")
    return r


def step_rungs(cfg: dict, state: dict, dt0: float, rungs=None):
    """One base step dt0 on individual steps, on a copy of ``state``; returns
    (new_state, rungs, number of sub-steps, counters).  ``rungs`` given:
    used as they are (no criterion, no limiter)."""
    p = make_params(cfg)
    s = {k: _f64(state[k]).copy() for k in STATE_KEYS}
    n = s["x"].size
    given = rungs is not None
    r = np.array(rungs, dtype=np.int32) if given else np.zeros(n, dtype=np.int32)
    nsub = ctypes.c_int64()
    cnt = Counters()
    rc = lib().orc_step_rungs(ctypes.byref(p), n, *[_p(s[k]) for k in STATE_KEYS], float(dt0),
                              r.ctypes.data_as(_I32), int(given), ctypes.byref(nsub),
                              ctypes.byref(cnt))
    if rc:
        raise RuntimeError(f"orc_step_rungs failed: {rc}")
    return s, r, nsub.value, cnt.as_dict()


def pipeline(cfg: dict, state: dict, dt_max: float):
    """Every stage of one step, keeping the intermediate fields (for parity tests)."""
    d, c1 = density(cfg, state["x"], state["y"], state["z"], state["H"])
    g, c2 = gradients(cfg, state["x"], state["y"], state["z"], d["H"], d["V"], state["m"],
                      state["vx"], state["vy"], state["vz"], state["U"])
    dt = min(float(dt_max), float(np.min(g["dt_i"])))
    f, c3 = fluxes(cfg, state["x"], state["y"], state["z"], d["H"], d["V"], g["rho"],
                   state["vx"], state["vy"], state["vz"], g["P"], g["B"], g["grad"], dt)
    new, c4 = update(cfg, state, f["dQ"], dt)
    new["H"] = d["H"].copy()
    counters = {k: c1[k] + c2[k] + c3[k] + c4[k] for k in c1}
    out = {"density": d, "gradients": g, "fluxes": f, "dt": dt, "state": new,
           "counters": counters}
    return out


# --- source terms (sec. 2.3.7-2.3.9) -------------------------------------------------------

def _opt(a):
    return a.ctypes.data_as(_D) if a is not None else None


def make_sources(n, accel=None, inv_a=1.0, hubble=(0.0, 0.0), S=None, emode=None):
    """Sources struct plus the numpy arrays it points at (kept alive by the caller)."""
    src = Sources()
    keep = {}
    if accel is not None:
        keep["accel"] = _f64(accel).reshape(3, n)
        src.accel = keep["accel"].ctypes.data
    src.inv_a = float(inv_a)
    src.hubble_n, src.hubble_np1 = float(hubble[0]), float(hubble[1])
    if S is not None:
        keep["S"] = S
        src.S = S.ctypes.data
        keep["emode"] = emode
        src.emode = emode.ctypes.data
    return src, keep


def step_src(cfg: dict, state: dict, dt_max: float, accel=None, inv_a=1.0, hubble=(0.0, 0.0),
             S=None, emode=None):
    """One full step with source terms on a copy of ``state``; S (float64) and
    emode (int32) arrays, when given, are updated in place.  Returns
    (new_state, dt, counters)."""
    p = make_params(cfg)
    s = {k: _f64(state[k]).copy() for k in STATE_KEYS}
    n = s["x"].size
    src, keep = make_sources(n, accel, inv_a, hubble, S, emode)
    dt = ctypes.c_double()
    cnt = Counters()
    rc = lib().orc_step_src(ctypes.byref(p), n, *[_p(s[k]) for k in STATE_KEYS], float(dt_max),
                            ctypes.byref(src), ctypes.byref(dt), ctypes.byref(cnt))
    if rc:
        raise RuntimeError(f"orc_step_src failed: {rc}")
    return s, dt.value, cnt.as_dict()


def ekin_max(cfg: dict, x, y, z, H, m, vx, vy, vz):
    """E_kin^max_i = max_j 1/2 m_i |v_j - v_i|^2 over r_ij < H_i (sec. 2.3.7)."""
    p = make_params(cfg)
    arrs = [_f64(a) for a in (x, y, z, H, m, vx, vy, vz)]
    out = np.empty(arrs[0].size)
    rc = lib().orc_ekin_max(ctypes.byref(p), arrs[0].size, *[_p(a) for a in arrs], _p(out))
    assert rc == 0
    return out


def fluxes_src(cfg: dict, x, y, z, H, V, rho, vx, vy, vz, P, B, grad, dt, inv_a=1.0,
               gwork=False):
    """Flux loop with the comoving factor; returns dQ, scale and (if asked)
    gwork[3, n] = sum_j dm_ij (x_j - x_i)."""
    p = make_params(cfg)
    arrs = [_f64(a) for a in (x, y, z, H, V, rho, vx, vy, vz, P)]
    B = _f64(B)
    grad = _f64(grad)
    n = arrs[0].size
    dQ = np.empty((5, n))
    scale = np.empty((5, n))
    gw = np.empty((3, n)) if gwork else None
    cnt = Counters()
    rc = lib().orc_fluxes_src(ctypes.byref(p), n, *[_p(a) for a in arrs], _p(B), _p(grad),
                              float(dt), float(inv_a), _p(dQ), _p(scale), _opt(gw),
                              ctypes.byref(cnt))
    if rc:
        raise RuntimeError(f"orc_fluxes_src failed: {rc}")
    return {"dQ": dQ, "scale": scale, "gwork": gw}, cnt.as_dict()


def update_src(cfg: dict, state: dict, dQ, dt, accel=None, inv_a=1.0, hubble=(0.0, 0.0),
               S=None, emode=None, gwork=None, ekin_max=None, V=None, H=None):
    """Close of the step with source terms on a copy of ``state``."""
    p = make_params(cfg)
    s = {k: _f64(state[k]).copy() for k in ("x", "y", "z", "m", "vx", "vy", "vz", "E", "U")}
    n = s["x"].size
    src, keep = make_sources(n, accel, inv_a, hubble, S, emode)
    cnt = Counters()
    rc = lib().orc_update_src(ctypes.byref(p), n, *[_p(s[k]) for k in
                                                    ("x", "y", "z", "m", "vx", "vy", "vz", "E",
                                                     "U")],
                              _p(_f64(dQ)), float(dt), ctypes.byref(src),
                              _opt(None if gwork is None else _f64(gwork)),
                              _opt(None if ekin_max is None else _f64(ekin_max)),
                              _opt(None if V is None else _f64(V)),
                              _opt(None if H is None else _f64(H)), ctypes.byref(cnt))
    if rc:
        raise RuntimeError(f"orc_update_src failed: {rc}")
    return s, cnt.as_dict()


def entropy_pressure(cfg: dict, m, V, U, S, emode):
    """U and S after a density pass (in place on U and S)."""
    p = make_params(cfg)
    rc = lib().orc_entropy_pressure(ctypes.byref(p), U.size, _p(_f64(m)), _p(_f64(V)), _p(U),
                                    _p(S), emode.ctypes.data_as(_I32))
    assert rc == 0
