"""The C-ABI library loads, exports every symbol its header declares, and
rejects bad input before touching the GPU (no compute calls here)."""

import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fsim.h")
LIBPATH = os.path.join(ROOT, "paper_2510_24968_amd", "libfsim.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fsim_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def so():
    if not os.path.exists(LIBPATH):
        pytest.fail("libfsim.so not built (run python -m paper_2510_24968_amd.build)")
    return ctypes.CDLL(LIBPATH)


def test_exports_every_declared_symbol(so):
    names = _declared()
    assert "fsim_fock_build" in names and "fsim_schwarz_screen" in names and \
        "fsim_scf_step" in names
    for n in names:
        assert hasattr(so, n), n


def _create(so, basis, **opt):
    from paper_2510_24968_amd.fsim import _Options, basis_struct
    b, keep = basis_struct(basis)
    o = _Options(opt.get("tau", 0.0), opt.get("tau_fp32", 0.0), opt.get("diis_m", 8), 1e-8, 1e-10,
                 50)
    h = ctypes.c_void_p()
    so.fsim_ctx_create.restype = ctypes.c_int
    so.fsim_last_error.restype = ctypes.c_char_p
    st = so.fsim_ctx_create(ctypes.byref(b), ctypes.byref(o), ctypes.byref(h))
    return st, so.fsim_last_error().decode()


@pytest.mark.parametrize("mutate,needle", [
    (lambda b: b["shell_l"].__setitem__(0, 3), "shell_l"),
    (lambda b: b["exps"].__setitem__(0, -1.0), "exponent"),
    (lambda b: b["exps"].__setitem__(0, float("nan")), "exponent"),
    (lambda b: b.__setitem__("nelec", 7), "nelec"),
    (lambda b: b.__setitem__("nelec", 0), "nelec"),
    (lambda b: b["shell_nprim"].__setitem__(0, 9), "shell_nprim"),
    (lambda b: b["shell_atom"].__setitem__(0, 99), "shell_atom"),
    (lambda b: b["xyz"].__setitem__((0, 0), float("inf")), "coordinate"),
])
def test_invalid_input_is_rejected_on_the_host(so, mutate, needle):
    b = synth.h_chain(4)
    for k in ("shell_l", "exps", "shell_nprim", "shell_atom", "xyz"):
        b[k] = np.array(b[k])
    mutate(b)
    st, msg = _create(so, b)
    assert st == -1 and needle in msg


def test_negative_threshold_rejected(so):
    st, msg = _create(so, synth.h_chain(4), tau=-1.0)
    assert st == -1 and "threshold" in msg


def test_null_arguments(so):
    so.fsim_ctx_create.restype = ctypes.c_int
    assert so.fsim_ctx_create(None, None, None) == -1
    so.fsim_ctx_destroy.restype = ctypes.c_int
    assert so.fsim_ctx_destroy(None) == 0
    so.fsim_fock_build.restype = ctypes.c_int
    assert so.fsim_fock_build(None, None, None, None, None, None, 0, None) == -1
