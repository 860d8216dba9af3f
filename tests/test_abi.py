"""The C ABI on the CPU: libmfm.so loads, exports every function that
include/mfm.h declares, and rejects invalid arguments in its host-side checks.
No call here launches a kernel or touches a device."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2211_12243_amd import build as hipbuild
from paper_2211_12243_amd import mfm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mfm.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mfm_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(hipbuild.LIB):
        hipbuild.build()
    return mfm.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("mfm_build_cells", "mfm_density", "mfm_gradients", "mfm_fluxes",
                     "mfm_update", "mfm_step", "mfm_create", "mfm_workspace_bytes",
                     "mfm_mlp_train_step", "mfm_face_dump", "mfm_mlp_attach"):
        assert required in names


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    out = subprocess.run(["nm", "-D", "--defined-only", hipbuild.LIB], capture_output=True,
                         text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(L, n)
    # the Python binding names every declared function
    assert sorted(set(mfm.EXPORTED) | {"mfm_default_params"}) == names


def test_default_params_are_the_papers(L):
    p = mfm.mfm_default_params()
    assert p.n_ngb == 32.0 and p.ncond_max == 100.0 and p.ngb_boost == 1.2
    assert p.psi1 == 0.5 and p.psi2 == 0.25 and p.alpha1 == 0.01
    assert p.riemann_tol == 1e-10 and p.guess == mfm.MFM_GUESS_PLAIN
    assert tuple(p.box) == (1.0, 1.0, 1.0)
    # sec. 2.3.7: alpha_2 = alpha_3 = 1/1000; the entropy switch is off by default
    assert p.alpha2 == 1e-3 and p.alpha3 == 1e-3 and p.entropy_switch == 0


@pytest.mark.parametrize("field,value", [
    ("gamma", 1.0), ("n_ngb", 5.0), ("box", (1.0, 0.0, 1.0)), ("max_list", 5000),
    ("reserved", 1), ("cell_margin", 0.5), ("scheme", 7), ("precision", 3), ("guess", 2),
    ("riemann_maxit", 0), ("h_maxit", 0), ("c_cfl", 0.0), ("alpha2", -1.0),
    ("entropy_switch", 2), ("mixed_jump", 0.5),
])
def test_invalid_parameters_give_no_workspace(L, field, value):
    p = mfm.mfm_default_params(**{field: value})
    assert L.mfm_workspace_bytes(ctypes.byref(p), 1000) == 0


def test_workspace_size_grows_with_n_and_list(L):
    p = mfm.mfm_default_params()
    a = L.mfm_workspace_bytes(ctypes.byref(p), 1000)
    b = L.mfm_workspace_bytes(ctypes.byref(p), 2000)
    p2 = mfm.mfm_default_params(max_list=256)
    c = L.mfm_workspace_bytes(ctypes.byref(p2), 1000)
    assert 0 < a < b and a < c
    assert L.mfm_workspace_bytes(ctypes.byref(p), 0) == 0


def test_create_rejects_bad_arguments_without_a_device(L):
    p = mfm.mfm_default_params()
    h = ctypes.c_void_p()
    nb = L.mfm_workspace_bytes(ctypes.byref(p), 100)
    # no workspace
    assert L.mfm_create(ctypes.byref(p), 100, None, nb, None, ctypes.byref(h)) == -2
    # workspace too small
    assert L.mfm_create(ctypes.byref(p), 100, ctypes.c_void_p(256), nb - 1, None,
                        ctypes.byref(h)) == -2
    # null output handle / null params
    assert L.mfm_create(ctypes.byref(p), 100, ctypes.c_void_p(256), nb, None, None) == -1
    assert L.mfm_create(None, 100, ctypes.c_void_p(256), nb, None, ctypes.byref(h)) == -1


def test_null_context_is_an_argument_error(L):
    for f in (L.mfm_density, L.mfm_destroy, L.mfm_reset_counters):
        args = [None] * len(f.argtypes)
        assert f(*args) == -1
    assert L.mfm_mlp_attach(None, None) == -1
    assert L.mfm_face_dump(None, None, 0) == -1
    assert L.mfm_mlp_init(None, None, None, None) == -1
    assert L.mfm_mlp_backward(None, None, 0, 8, None, None) == -1


def test_status_texts(L):
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8):
        assert L.mfm_strerror(code)
    assert L.mfm_strerror(-99)
    assert L.mfm_mlp_param_count() == 16 * 64 + 64 + 2 * (64 * 64 + 64) + 64 + 1
    assert L.mfm_mlp_state_bytes() % 256 == 0
