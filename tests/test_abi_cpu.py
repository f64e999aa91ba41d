"""The C-ABI library loads on the CPU host and exports what include/le.h declares.

No kernel is launched here: only symbol lookup, struct layout and the
argument validation that runs before any device call.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_0710_5912_amd import le

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"\b(le_\w+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_core_abi():
    names = declared_functions()
    for core in ("le_create", "le_step", "le_observables", "le_destroy"):
        assert core in names


def test_library_exports_every_declared_symbol():
    lib = le.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_symbols_match_header():
    assert set(le.SYMBOLS) <= set(declared_functions())


def test_struct_layouts():
    # int32 nx, ny; 10 doubles; int32 precision (+pad); pointer
    assert C.sizeof(le.LeParams) == 8 + 10 * 8 + 8 + 8
    assert le.LeParams.stream.offset == 96
    assert le.LeObs.finite.offset == C.sizeof(le.LeObs) - 8


def test_strerror_names_codes():
    assert le.strerror(le.LE_OK) == "ok"
    assert "invalid" in le.strerror(le.LE_EINVAL)
    assert le.strerror(-99) == "unknown error"


BASE = dict(nx=64, ny=64, lx=64.0, ly=64.0, gdot=0.01, A=1.0, B=1.0, kappa=1.0, M=1.0,
            eta=1.0, rho=1.0, dt=0.005)


@pytest.mark.parametrize("bad", [dict(nx=48), dict(ny=4), dict(nx=8192), dict(lx=0.0),
                                 dict(dt=-1.0), dict(eta=0.0), dict(rho=-1.0),
                                 dict(kappa=float("nan")), dict(nx=32, ny=64, gdot=0.1)])
def test_invalid_parameters_rejected_before_any_device_call(bad):
    p = dict(BASE, **bad)
    phi = np.zeros((p["ny"], p["nx"]))
    with pytest.raises(le.LeError) as ei:
        le.Context(p, phi)
    assert ei.value.code == le.LE_EINVAL


def test_null_arguments_rejected():
    lib = le.lib()
    h = C.c_void_p()
    p = le.make_params(BASE)
    assert lib.le_create(C.byref(p), None, None, C.byref(h)) == le.LE_EINVAL
    assert lib.le_step(None, 1) == le.LE_EINVAL
    assert lib.le_observables(None, None, None, 0) == le.LE_EINVAL
    assert lib.le_tuning(None, None, 0) == le.LE_EINVAL
    assert lib.le_batch_tuning(None, None, 0) == le.LE_EINVAL
    assert lib.le_corrector_audit(None, 10, 2, 0.02) == le.LE_EINVAL
    assert lib.le_corrector_status(None, None, None, None) == le.LE_EINVAL
    assert lib.le_set_recovery(None, 1) == le.LE_EINVAL
    assert lib.le_set_scheme(None, 0) == le.LE_EINVAL
    lib.le_destroy(None)   # NULL-safe


def test_stage_timer_validates_arguments():
    lib = le.lib()
    ms = C.c_double()
    assert lib.le_time_stage(None, 0, 1, C.byref(ms)) == le.LE_EINVAL


@pytest.mark.parametrize("header", ["le.h", "le_train.h"])
@pytest.mark.parametrize("lang,std", [("c", "c99"), ("c++", "c++11")])
def test_header_compiles_standalone(lang, std, header, tmp_path):
    """The headers are plain C: each compiles on its own as C99 and as C++11."""
    import shutil
    import subprocess
    cc = shutil.which("gcc" if lang == "c" else "g++")
    if cc is None:
        pytest.skip("no host compiler")
    r = subprocess.run([cc, "-x", lang, f"-std={std}", "-Wall", "-Wextra", "-Werror",
                        "-fsyntax-only", os.path.join(ROOT, "include", header)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
