"""Python binding of libmfm (include/mfm.h): argument marshalling only.

Every step of the hydro path runs in the HIP kernels of ``libmfm.so``.  This
module loads that library with ctypes, mirrors its structs, and offers
functions with the same names as the C entry points.  PyTorch supplies the
device memory (tensors) and the stream.  If the library is not built, or no
HIP device is visible, the calls raise; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmfm.so")

MFM_OK = 0
MFM_SCHEME_MFV, MFM_SCHEME_MFM = 0, 1
MFM_FP64, MFM_MIXED = 0, 1
MFM_GUESS_PLAIN, MFM_GUESS_LEARNED = 0, 1
MFM_LIMIT_BJ, MFM_LIMIT_PAIRWISE = 1, 2
MFM_NSTAGES = 8
STAGES = ("cells", "search", "density", "gradients", "fluxes", "update", "flux_kernel",
          "flux_hard")


class mfm_params(ctypes.Structure):
    _fields_ = [
        ("scheme", ctypes.c_int32), ("precision", ctypes.c_int32), ("limiter", ctypes.c_int32),
        ("max_boosts", ctypes.c_int32), ("h_maxit", ctypes.c_int32),
        ("riemann_maxit", ctypes.c_int32), ("guess", ctypes.c_int32),
        ("max_list", ctypes.c_int32),
        ("gamma", ctypes.c_double), ("n_ngb", ctypes.c_double), ("ncond_max", ctypes.c_double),
        ("ngb_boost", ctypes.c_double), ("h_tol", ctypes.c_double), ("c_cfl", ctypes.c_double),
        ("psi1", ctypes.c_double), ("psi2", ctypes.c_double), ("riemann_tol", ctypes.c_double),
        ("alpha1", ctypes.c_double), ("box", ctypes.c_double * 3),
        ("cell_margin", ctypes.c_double), ("reserved", ctypes.c_int32),
        ("pad0", ctypes.c_int32), ("alpha2", ctypes.c_double), ("alpha3", ctypes.c_double),
        ("entropy_switch", ctypes.c_int32), ("pad1", ctypes.c_int32),
        ("mixed_jump", ctypes.c_double),
    ]


_PTR = ctypes.c_void_p
_STATE = ("x", "y", "z", "vx", "vy", "vz", "m", "E", "U", "H")
_DERIVED = ("V", "rho", "P", "c", "ncond")


class mfm_particles(ctypes.Structure):
    _fields_ = ([("n", ctypes.c_int64)] + [(k, _PTR) for k in _STATE + _DERIVED]
                + [(k, _PTR) for k in ("B", "grad", "dQ", "dt_i", "id", "S", "emode", "accel")])


_DIAG_INT = ("h_noconv", "ncond_boosts", "ncond_fail", "cell_rebuilds", "list_overflow",
             "grad_pairs", "faces", "riemann_iters", "riemann_maxit", "vacuum", "positivity",
             "neg_mass", "singular_e", "guess_fallback", "fp64_inverse", "u_guard",
             "hard_faces", "hard_overflow")


class mfm_diag(ctypes.Structure):
    _fields_ = ([(k, ctypes.c_int64) for k in _DIAG_INT]
                + [(k, ctypes.c_double) for k in ("mass", "px", "py", "pz", "energy")])

    def as_dict(self):
        d = {k: int(getattr(self, k)) for k in _DIAG_INT}
        d.update({k: float(getattr(self, k)) for k in ("mass", "px", "py", "pz", "energy")})
        return d


class MFMError(RuntimeError):
    pass


_lib = None


def lib():
    """Load libmfm.so (raises if it is missing: nothing falls back to the CPU)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise MFMError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, PP, C = ctypes.POINTER(mfm_params), ctypes.POINTER(mfm_particles), _PTR
        L.mfm_default_params.argtypes = [P]
        L.mfm_default_params.restype = None
        L.mfm_workspace_bytes.argtypes = [P, ctypes.c_int64]
        L.mfm_workspace_bytes.restype = ctypes.c_size_t
        L.mfm_create.argtypes = [P, ctypes.c_int64, _PTR, ctypes.c_size_t, _PTR,
                                 ctypes.POINTER(_PTR)]
        L.mfm_destroy.argtypes = [C]
        L.mfm_set_cosmology.argtypes = [C, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.mfm_set_cosmology.restype = ctypes.c_int
        L.mfm_create_static.argtypes = [P, ctypes.c_int64, _PTR, ctypes.POINTER(_PTR)]
        L.mfm_create_static.restype = ctypes.c_int
        L.mfm_static_workspace_bytes.argtypes = []
        L.mfm_static_workspace_bytes.restype = ctypes.c_size_t
        L.mfm_build_cells.argtypes = [C, PP, _PTR]
        L.mfm_density.argtypes = [C, PP]
        L.mfm_gradients.argtypes = [C, PP, ctypes.c_double, _PTR]
        L.mfm_fluxes.argtypes = [C, PP, _PTR]
        L.mfm_update.argtypes = [C, PP, _PTR]
        L.mfm_step.argtypes = [C, PP, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
        L.mfm_step_rungs.argtypes = [C, PP, ctypes.c_double, _PTR, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_int64)]
        L.mfm_diagnostics.argtypes = [C, PP, ctypes.POINTER(mfm_diag)]
        L.mfm_reset_counters.argtypes = [C]
        L.mfm_enable_timing.argtypes = [C, ctypes.c_int]
        L.mfm_kernel_times.argtypes = [C, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int64)]
        for f in ("mfm_create", "mfm_destroy", "mfm_build_cells", "mfm_density", "mfm_gradients",
                  "mfm_fluxes", "mfm_update", "mfm_step", "mfm_diagnostics",
                  "mfm_reset_counters", "mfm_enable_timing", "mfm_kernel_times"):
            getattr(L, f).restype = ctypes.c_int
        F, I64 = ctypes.POINTER(ctypes.c_float), ctypes.c_int64
        L.mfm_mlp_state_bytes.argtypes = []
        L.mfm_mlp_state_bytes.restype = ctypes.c_size_t
        L.mfm_mlp_param_count.argtypes = []
        L.mfm_mlp_param_count.restype = ctypes.c_int
        L.mfm_mlp_init.argtypes = [_PTR, F, F, _PTR]
        L.mfm_mlp_backward.argtypes = [_PTR, _PTR, I64, I64, F, _PTR]
        L.mfm_mlp_adam.argtypes = [_PTR, ctypes.c_float, ctypes.c_int, _PTR]
        L.mfm_mlp_train_step.argtypes = [_PTR, _PTR, I64, I64, ctypes.c_float, ctypes.c_int, F,
                                         _PTR]
        L.mfm_mlp_predict.argtypes = [_PTR, _PTR, I64, I64, _PTR, _PTR]
        L.mfm_mlp_get.argtypes = [_PTR, F, F, _PTR]
        L.mfm_mlp_attach.argtypes = [C, _PTR]
        L.mfm_face_dump.argtypes = [C, _PTR, I64]
        L.mfm_face_dump_count.argtypes = [C, ctypes.POINTER(I64)]
        for f in ("mfm_mlp_init", "mfm_mlp_backward", "mfm_mlp_adam", "mfm_mlp_train_step",
                  "mfm_mlp_predict",
                  "mfm_mlp_get", "mfm_mlp_attach", "mfm_face_dump", "mfm_face_dump_count"):
            getattr(L, f).restype = ctypes.c_int
        L.mfm_strerror.argtypes = [ctypes.c_int]
        L.mfm_strerror.restype = ctypes.c_char_p
        L.mfm_last_error.argtypes = [C]
        L.mfm_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


EXPORTED = ("mfm_default_params", "mfm_workspace_bytes", "mfm_create", "mfm_destroy",
            "mfm_create_static", "mfm_static_workspace_bytes", "mfm_set_cosmology",
            "mfm_build_cells", "mfm_density", "mfm_gradients", "mfm_fluxes", "mfm_update",
            "mfm_step", "mfm_step_rungs", "mfm_diagnostics", "mfm_reset_counters", "mfm_enable_timing",
            "mfm_kernel_times", "mfm_strerror", "mfm_last_error", "mfm_mlp_state_bytes",
            "mfm_mlp_param_count", "mfm_mlp_init", "mfm_mlp_backward", "mfm_mlp_adam",
            "mfm_mlp_train_step",
            "mfm_mlp_predict", "mfm_mlp_get", "mfm_mlp_attach", "mfm_face_dump",
            "mfm_face_dump_count")


def mfm_default_params(**over) -> mfm_params:
    p = mfm_params()
    lib().mfm_default_params(ctypes.byref(p))
    for k, v in over.items():
        if k == "box":
            for a in range(3):
                p.box[a] = float(v[a])
        elif k == "scheme" and isinstance(v, str):
            p.scheme = MFM_SCHEME_MFM if v == "mfm" else MFM_SCHEME_MFV
        elif k == "precision" and isinstance(v, str):
            p.precision = MFM_MIXED if v == "mixed" else MFM_FP64
        else:
            setattr(p, k, v)
    return p


def params_from_dict(cfg: dict, **over) -> mfm_params:
    """The library's parameter struct from the plain dict the tests share."""
    keys = ("scheme", "limiter", "max_boosts", "h_maxit", "riemann_maxit", "gamma", "n_ngb",
            "ncond_max", "ngb_boost", "h_tol", "c_cfl", "psi1", "psi2", "riemann_tol", "alpha1",
            "box", "precision", "max_list", "cell_margin", "guess",
            "mixed_jump", "alpha2", "alpha3", "entropy_switch")
    d = {k: cfg[k] for k in keys if k in cfg}
    d.update(over)
    return mfm_default_params(**d)


def _check(rc, ctx=None):
    if rc != MFM_OK:
        msg = lib().mfm_strerror(rc).decode()
        if ctx is not None:
            msg += ": " + (lib().mfm_last_error(ctx).decode() or "")
        raise MFMError(f"libmfm status {rc}: {msg}")
    return rc


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class ParticleSet:
    """Device arrays of one particle set (torch tensors) and their C struct."""

    def __init__(self, state: dict, device="cuda", ids: bool = True, entropy: bool = False,
                 accel=None):
        """state: host arrays x..H.  entropy: allocate S and emode (the
        entropy switch; S is set from U by the first density pass).  accel:
        optional (3, n) external acceleration."""
        n = int(len(state["x"]))
        self.n = n
        self.device = device
        f64 = dict(dtype=torch.float64, device=device)
        self.t = {k: torch.as_tensor(state[k], **f64).contiguous().clone() for k in _STATE}
        for k in _DERIVED + ("dt_i",):
            self.t[k] = torch.zeros(n, **f64)
        self.t["B"] = torch.zeros(6, n, **f64)
        self.t["grad"] = torch.zeros(15, n, **f64)
        self.t["dQ"] = torch.zeros(5, n, **f64)
        self.t["id"] = (torch.arange(n, dtype=torch.int64, device=device) if ids else None)
        self.t["S"] = torch.zeros(n, **f64) if entropy else None
        self.t["emode"] = (torch.zeros(n, dtype=torch.int32, device=device) if entropy
                           else None)
        self.t["accel"] = (torch.as_tensor(accel, **f64).reshape(3, n).contiguous().clone()
                           if accel is not None else None)
        self.s = mfm_particles()
        self.s.n = n
        for k in _STATE + _DERIVED + ("B", "grad", "dQ", "dt_i", "id", "S", "emode", "accel"):
            t = self.t[k]
            setattr(self.s, k, t.data_ptr() if t is not None else None)

    def __getitem__(self, k):
        return self.t[k]

    def host(self, keys=None) -> dict:
        keys = keys or [k for k in self.t if self.t[k] is not None]
        return {k: self.t[k].detach().cpu().numpy() for k in keys}


class Context:
    """A libmfm context with its workspace tensor, bound to one stream."""

    def __init__(self, params: mfm_params, n_max: int, stream=None, device="cuda",
                 static: bool = False):
        L = lib()
        self.params = params
        self.n_max = int(n_max)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.h = ctypes.c_void_p()
        self.dt_dev = torch.zeros(1, dtype=torch.float64, device=device)
        if static:
            # the library's own device scratch: mfm_create_static allocates nothing
            self.ws = None
            _check(L.mfm_create_static(ctypes.byref(params), self.n_max,
                                       ctypes.c_void_p(self.stream.cuda_stream),
                                       ctypes.byref(self.h)))
            return
        nbytes = L.mfm_workspace_bytes(ctypes.byref(params), self.n_max)
        if nbytes == 0:
            raise MFMError("invalid parameters (mfm_workspace_bytes returned 0)")
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) // 256 * 256
        _check(L.mfm_create(ctypes.byref(params), self.n_max, ctypes.c_void_p(self.ws_ptr),
                            nbytes, ctypes.c_void_p(self.stream.cuda_stream),
                            ctypes.byref(self.h)))

    def close(self):
        if self.h:
            lib().mfm_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --- entry points with the C names --------------------------------------------------------

def mfm_create(params: mfm_params, n_max: int, stream=None) -> Context:
    return Context(params, n_max, stream)


def mfm_destroy(ctx: Context):
    ctx.close()


def mfm_set_cosmology(ctx: Context, inv_a: float, hubble_n: float, hubble_np1: float):
    _check(lib().mfm_set_cosmology(ctx.h, float(inv_a), float(hubble_n), float(hubble_np1)),
           ctx.h)


def mfm_build_cells(ctx: Context, ps: ParticleSet, perm=None):
    _check(lib().mfm_build_cells(ctx.h, ctypes.byref(ps.s), _ptr(perm)), ctx.h)


def mfm_density(ctx: Context, ps: ParticleSet):
    _check(lib().mfm_density(ctx.h, ctypes.byref(ps.s)), ctx.h)


def mfm_gradients(ctx: Context, ps: ParticleSet, dt_max: float, dt_dev=None):
    dt_dev = ctx.dt_dev if dt_dev is None else dt_dev
    _check(lib().mfm_gradients(ctx.h, ctypes.byref(ps.s), float(dt_max), _ptr(dt_dev)), ctx.h)
    return dt_dev


def mfm_fluxes(ctx: Context, ps: ParticleSet, dt_dev=None):
    dt_dev = ctx.dt_dev if dt_dev is None else dt_dev
    _check(lib().mfm_fluxes(ctx.h, ctypes.byref(ps.s), _ptr(dt_dev)), ctx.h)


def mfm_update(ctx: Context, ps: ParticleSet, dt_dev=None):
    dt_dev = ctx.dt_dev if dt_dev is None else dt_dev
    _check(lib().mfm_update(ctx.h, ctypes.byref(ps.s), _ptr(dt_dev)), ctx.h)


def mfm_step(ctx: Context, ps: ParticleSet, dt_max: float) -> float:
    dt = ctypes.c_double()
    _check(lib().mfm_step(ctx.h, ctypes.byref(ps.s), float(dt_max), ctypes.byref(dt)), ctx.h)
    return dt.value


RUNG_MAX = 24


def mfm_step_rungs(ctx: Context, ps: ParticleSet, dt0: float, rungs=None):
    """One base step dt0 on individual time steps.  ``rungs`` (torch int32 on
    the device, in the particles' current order) given: used as they are
    (and permuted with the particles).  Returns (number of sub-steps, rungs
    in the particles' order after the call)."""
    import torch

    given = rungs is not None
    if given:
        if rungs.dtype != torch.int32 or not rungs.is_cuda or rungs.numel() != ps.n:
            raise MFMError("rungs must be a device int32 tensor of one entry per particle")
        r = rungs.contiguous()
    else:
        r = torch.zeros(ps.n, dtype=torch.int32, device=ps.device)
    nsub = ctypes.c_int64()
    _check(lib().mfm_step_rungs(ctx.h, ctypes.byref(ps.s), float(dt0),
                                ctypes.c_void_p(r.data_ptr()), int(given), ctypes.byref(nsub)),
           ctx.h)
    return nsub.value, r


def mfm_diagnostics(ctx: Context, ps: ParticleSet | None = None) -> dict:
    d = mfm_diag()
    _check(lib().mfm_diagnostics(ctx.h, ctypes.byref(ps.s) if ps is not None else None,
                                 ctypes.byref(d)), ctx.h)
    return d.as_dict()


def mfm_reset_counters(ctx: Context):
    _check(lib().mfm_reset_counters(ctx.h), ctx.h)


def mfm_enable_timing(ctx: Context, on: bool = True):
    _check(lib().mfm_enable_timing(ctx.h, int(bool(on))), ctx.h)


def mfm_kernel_times(ctx: Context) -> dict:
    ms = (ctypes.c_double * MFM_NSTAGES)()
    cnt = (ctypes.c_int64 * MFM_NSTAGES)()
    _check(lib().mfm_kernel_times(ctx.h, ms, cnt), ctx.h)
    return {STAGES[s]: (ms[s], int(cnt[s])) for s in range(MFM_NSTAGES)}


def run_pipeline(ctx: Context, ps: ParticleSet, dt_max: float, update: bool = True):
    """All loops of one step through the C entry points; returns dt (host float)."""
    mfm_build_cells(ctx, ps)
    for _ in range(4):
        try:
            mfm_density(ctx, ps)
            break
        except MFMError as e:
            if "status -5" not in str(e):
                raise
            mfm_build_cells(ctx, ps)
    else:
        raise MFMError("cell grid kept overflowing")
    mfm_gradients(ctx, ps, dt_max)
    mfm_fluxes(ctx, ps)
    dt = float(ctx.dt_dev.item())
    if update:
        mfm_update(ctx, ps)
    return dt


# --- learned Riemann guess ------------------------------------------------------------------

MLP_NIN, MLP_K1, MLP_HID, MLP_NNORM = 6, 16, 64, 16
DUMP_STRIDE = 8  # floats per face record: 6 features, ln(p*/p0), Newton iterations


GATE_LOG_P = 0.69314718  # ln 2: pressure ratio above 2
GATE_DU = 0.40546511     # ln 1.5: |u_R - u_L| above half the mean sound speed


def guess_gate(rows):
    """Rows (torch tensor [n, 8] of face records) the flux loop would hand to
    the network: the same test as the kernel's, on the stored features."""
    return (rows[:, 1].abs() > GATE_LOG_P) | (rows[:, 2].abs() > GATE_DU)


def mlp_param_layout() -> dict:
    """Offsets and shapes of the FP32 parameter vector (order fixed by the C ABI)."""
    shapes = [("W1", (MLP_K1, MLP_HID)), ("b1", (MLP_HID,)), ("W2", (MLP_HID, MLP_HID)),
              ("b2", (MLP_HID,)), ("W3", (MLP_HID, MLP_HID)), ("b3", (MLP_HID,)),
              ("w4", (MLP_HID,)), ("b4", (1,))]
    out, off = {}, 0
    for name, shp in shapes:
        size = 1
        for d in shp:
            size *= d
        out[name] = (off, shp)
        off += size
    assert off == mfm_mlp_param_count()
    return out


def mfm_mlp_param_count() -> int:
    return int(lib().mfm_mlp_param_count())


def mfm_mlp_state_bytes() -> int:
    return int(lib().mfm_mlp_state_bytes())


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _stream_ptr(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class MLPState:
    """Device state of the guess network (one tensor of mfm_mlp_state_bytes bytes)."""

    def __init__(self, params, norm, stream=None, device="cuda"):
        import numpy as np
        nb = mfm_mlp_state_bytes()
        self.buf = torch.empty(nb + 256, dtype=torch.uint8, device=device)
        self.ptr = (self.buf.data_ptr() + 255) // 256 * 256
        self.stream = stream
        self.step = 0
        p = np.ascontiguousarray(params, dtype=np.float32)
        q = np.ascontiguousarray(norm, dtype=np.float32)
        if p.size != mfm_mlp_param_count() or q.size != MLP_NNORM:
            raise MFMError("parameter or normalisation vector has the wrong length")
        _check(lib().mfm_mlp_init(ctypes.c_void_p(self.ptr), _fptr(p), _fptr(q),
                                  _stream_ptr(stream)))

    @property
    def handle(self):
        return ctypes.c_void_p(self.ptr)


def mfm_mlp_init(params, norm, stream=None) -> MLPState:
    return MLPState(params, norm, stream)


def mfm_mlp_backward(st: MLPState, rows, n=None, stride=DUMP_STRIDE) -> float:
    n = int(rows.shape[0]) if n is None else int(n)
    loss = ctypes.c_float()
    _check(lib().mfm_mlp_backward(st.handle, _ptr(rows), n, int(stride), ctypes.byref(loss),
                                  _stream_ptr(st.stream)))
    return float(loss.value)


def mfm_mlp_adam(st: MLPState, lr: float):
    st.step += 1
    _check(lib().mfm_mlp_adam(st.handle, float(lr), st.step, _stream_ptr(st.stream)))


def mfm_mlp_train_step(st: MLPState, rows, lr: float, n=None, stride=DUMP_STRIDE,
                       want_loss=False):
    n = int(rows.shape[0]) if n is None else int(n)
    st.step += 1
    loss = ctypes.c_float()
    _check(lib().mfm_mlp_train_step(st.handle, _ptr(rows), n, int(stride), float(lr), st.step,
                                    ctypes.byref(loss) if want_loss else None,
                                    _stream_ptr(st.stream)))
    return float(loss.value) if want_loss else None


def mfm_mlp_predict(st: MLPState, rows, n=None, stride=DUMP_STRIDE):
    n = int(rows.shape[0]) if n is None else int(n)
    y = torch.empty(n, dtype=torch.float32, device=rows.device)
    _check(lib().mfm_mlp_predict(st.handle, _ptr(rows), n, int(stride), _ptr(y),
                                 _stream_ptr(st.stream)))
    return y


def mfm_mlp_get(st: MLPState):
    import numpy as np
    n = mfm_mlp_param_count()
    p = np.zeros(n, dtype=np.float32)
    g = np.zeros(n, dtype=np.float32)
    _check(lib().mfm_mlp_get(st.handle, _fptr(p), _fptr(g), _stream_ptr(st.stream)))
    return p, g


def mfm_mlp_attach(ctx: Context, st: MLPState | None):
    ctx.mlp = st  # keeps the state alive while attached
    _check(lib().mfm_mlp_attach(ctx.h, st.handle if st is not None else None), ctx.h)


def mfm_face_dump(ctx: Context, records=None):
    """Arm (records: float32 device tensor [cap, 8]) or disarm (None) the face dump."""
    ctx.dump = records
    cap = int(records.shape[0]) if records is not None else 0
    _check(lib().mfm_face_dump(ctx.h, _ptr(records), cap), ctx.h)


def mfm_face_dump_count(ctx: Context) -> int:
    c = ctypes.c_int64()
    _check(lib().mfm_face_dump_count(ctx.h, ctypes.byref(c)), ctx.h)
    return int(c.value)
