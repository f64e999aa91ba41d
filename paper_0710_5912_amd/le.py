"""ctypes binding of the C ABI in include/le.h (argument marshalling only).

Every step of the method runs in the HIP library; this module converts NumPy
arrays and dicts to the C structs and back.  It loads ``libmodelh.so`` from
this package directory and raises if the library has not been built: there is
no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmodelh.so")

LE_OK, LE_EINVAL, LE_ENOMEM, LE_EDEVICE, LE_ENONFINITE, LE_ESTATE = 0, -1, -2, -3, -4, -5
LE_SCHEME_F_HALF, LE_SCHEME_MIDPOINT_S, LE_SCHEME_UPWIND3, LE_SCHEME_BANDED = 1, 2, 4, 8
LE_FP64, LE_FP32 = 0, 1

SYMBOLS = ("le_create", "le_step", "le_corrector_projection", "le_step_noalloc", "le_checkpoint_size",
           "le_checkpoint_save", "le_checkpoint_load", "le_observables", "le_destroy", "le_get_state",
           "le_set_state", "le_strerror", "le_profile", "le_stage_times", "le_last_error",
           "le_batch_create", "le_batch_step", "le_batch_observables", "le_batch_get_state",
           "le_batch_profile", "le_batch_stage_times", "le_batch_destroy",
           "le_tuning", "le_batch_tuning", "le_time_stage",
           "le_corrector_load", "le_step_corrected", "le_restrict", "le_set_fields",
           "le_corrector_audit", "le_corrector_status", "le_set_scheme", "le_set_recovery",
           "le_batch_set_scheme",
           "le_cnn_nparams", "le_cnn_create", "le_cnn_destroy", "le_cnn_set_params",
           "le_cnn_get_params", "le_cnn_forward", "le_cnn_grad", "le_cnn_adam",
           "le_cnn_layer_fwd", "le_cnn_layer_bwd", "le_cnn_mfma_probe")
LE_NSTAGES = 6
STAGES = ("row_inv_flow", "advect", "column_ch", "row_inv_phi", "mu_source", "column_flow")
LE_TUNING_FIELDS = 10
TUNING_KEYS = ("nx", "ny", "precision", "inertial", "advect", "mu_source", "column_ch",
               "column_flow", "row", "row_fwd")


class LeParams(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("lx", C.c_double),
                ("ly", C.c_double), ("gdot", C.c_double), ("A", C.c_double),
                ("B", C.c_double), ("kappa", C.c_double), ("M", C.c_double),
                ("eta", C.c_double), ("rho", C.c_double), ("dt", C.c_double),
                ("precision", C.c_int32), ("stream", C.c_void_p)]


class LeObs(C.Structure):
    _fields_ = [("step", C.c_int64), ("wraps", C.c_int64), ("t", C.c_double),
                ("strain", C.c_double), ("s", C.c_double), ("mean_phi", C.c_double),
                ("phi2", C.c_double), ("Ls", C.c_double), ("Dxx", C.c_double),
                ("Dxy", C.c_double), ("Dyy", C.c_double), ("L_par", C.c_double),
                ("L_perp", C.c_double), ("sigma_xy", C.c_double),
                ("sigma_xy_re", C.c_double), ("nbins", C.c_int32), ("dk", C.c_double),
                ("finite", C.c_int32)]


def _tuning(fn, h, what):
    """Per-group kernel variants chosen at creation (list of dicts)."""
    n = fn(h, None, 0)
    if n < 0:
        raise LeError(n, what)
    buf = (C.c_int32 * (n * LE_TUNING_FIELDS))()
    rc = fn(h, buf, n * LE_TUNING_FIELDS)
    if rc < 0:
        raise LeError(rc, what)
    return [dict(zip(TUNING_KEYS, buf[i * LE_TUNING_FIELDS:(i + 1) * LE_TUNING_FIELDS]))
            for i in range(n)]


class LeError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = f"{what}: {strerror(code)} ({code})"
        if code == LE_EDEVICE:
            msg += f" [{lib().le_last_error().decode()}]"
        super().__init__(msg)
        self.code = code


_LIB = None
_DP = C.POINTER(C.c_double)


def lib():
    """Load the HIP library once; raise if it is missing."""
    global _LIB
    if _LIB is None:
        # torch carries its own HIP runtime next to the system one this
        # library links; both work in one process only when torch has
        # initialised the device first, so let it do so before loading.
        try:
            import torch
            if torch.cuda.is_available():
                torch.cuda.init()
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_0710_5912_amd.build`")
        L = C.CDLL(LIB_PATH)
        L.le_create.argtypes = [C.POINTER(LeParams), _DP, _DP, C.POINTER(C.c_void_p)]
        L.le_create.restype = C.c_int
        L.le_step.argtypes = [C.c_void_p, C.c_int64]
        L.le_step.restype = C.c_int
        L.le_checkpoint_size.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
        L.le_checkpoint_size.restype = C.c_int
        L.le_checkpoint_save.argtypes = [C.c_void_p, C.c_void_p, C.c_int64]
        L.le_checkpoint_save.restype = C.c_int
        L.le_checkpoint_load.argtypes = [C.c_void_p, C.c_void_p, C.c_int64]
        L.le_checkpoint_load.restype = C.c_int
        L.le_corrector_projection.argtypes = [C.c_void_p, C.c_int32]
        L.le_corrector_projection.restype = C.c_int
        L.le_step_noalloc.argtypes = [C.POINTER(LeParams), C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_int64, C.c_int64]
        L.le_step_noalloc.restype = C.c_int
        L.le_set_scheme.argtypes = [C.c_void_p, C.c_int32]
        L.le_set_scheme.restype = C.c_int
        L.le_set_recovery.argtypes = [C.c_void_p, C.c_int]
        L.le_set_recovery.restype = C.c_int
        L.le_batch_set_scheme.argtypes = [C.c_void_p, C.c_int32]
        L.le_batch_set_scheme.restype = C.c_int
        L.le_observables.argtypes = [C.c_void_p, C.POINTER(LeObs), _DP, C.c_int32]
        L.le_observables.restype = C.c_int
        L.le_destroy.argtypes = [C.c_void_p]
        L.le_destroy.restype = None
        L.le_get_state.argtypes = [C.c_void_p, _DP, _DP, _DP, C.POINTER(C.c_int64),
                                   C.POINTER(C.c_int64)]
        L.le_get_state.restype = C.c_int
        L.le_set_state.argtypes = [C.c_void_p, _DP, _DP, _DP, C.c_int64, C.c_int64]
        L.le_set_state.restype = C.c_int
        L.le_profile.argtypes = [C.c_void_p, C.c_int]
        L.le_profile.restype = C.c_int
        L.le_stage_times.argtypes = [C.c_void_p, _DP, C.POINTER(C.c_int64), C.c_int32]
        L.le_stage_times.restype = C.c_int
        _PP = C.POINTER(_DP)
        L.le_batch_create.argtypes = [C.c_int32, C.POINTER(LeParams), _PP, _PP,
                                      C.POINTER(C.c_void_p)]
        L.le_batch_create.restype = C.c_int
        L.le_batch_step.argtypes = [C.c_void_p, C.c_int64]
        L.le_batch_step.restype = C.c_int
        L.le_batch_observables.argtypes = [C.c_void_p, C.c_int32, C.POINTER(LeObs), _DP,
                                           C.c_int32]
        L.le_batch_observables.restype = C.c_int
        L.le_batch_get_state.argtypes = [C.c_void_p, C.c_int32, _DP, _DP, _DP,
                                         C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.le_batch_get_state.restype = C.c_int
        L.le_batch_profile.argtypes = [C.c_void_p, C.c_int]
        L.le_batch_profile.restype = C.c_int
        L.le_batch_stage_times.argtypes = [C.c_void_p, _DP, C.POINTER(C.c_int64), C.c_int32]
        L.le_batch_stage_times.restype = C.c_int
        L.le_time_stage.argtypes = [C.c_void_p, C.c_int32, C.c_int32, _DP]
        L.le_time_stage.restype = C.c_int
        for f in (L.le_tuning, L.le_batch_tuning):
            f.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.c_int32]
            f.restype = C.c_int
        L.le_batch_destroy.argtypes = [C.c_void_p]
        L.le_batch_destroy.restype = None
        _FP = C.POINTER(C.c_float)
        _U16 = C.POINTER(C.c_uint16)
        L.le_corrector_load.argtypes = [C.c_void_p, _FP, C.c_int32, _FP]
        L.le_corrector_load.restype = C.c_int
        L.le_step_corrected.argtypes = [C.c_void_p, C.c_int64]
        L.le_step_corrected.restype = C.c_int
        L.le_corrector_audit.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_double]
        L.le_corrector_audit.restype = C.c_int
        L.le_corrector_status.argtypes = [C.c_void_p, C.POINTER(C.c_int32),
                                          C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.le_corrector_status.restype = C.c_int
        L.le_restrict.argtypes = [C.c_void_p, C.c_int32, _DP, _DP]
        L.le_restrict.restype = C.c_int
        L.le_set_fields.argtypes = [C.c_void_p, _DP, _DP, C.c_int64]
        L.le_set_fields.restype = C.c_int
        L.le_cnn_nparams.argtypes = []
        L.le_cnn_nparams.restype = C.c_int
        L.le_cnn_create.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_void_p)]
        L.le_cnn_create.restype = C.c_int
        L.le_cnn_destroy.argtypes = [C.c_void_p]
        L.le_cnn_destroy.restype = None
        L.le_cnn_set_params.argtypes = [C.c_void_p, _FP, C.c_int32, _FP]
        L.le_cnn_set_params.restype = C.c_int
        L.le_cnn_get_params.argtypes = [C.c_void_p, _FP, C.c_int32]
        L.le_cnn_get_params.restype = C.c_int
        L.le_cnn_forward.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.le_cnn_forward.restype = C.c_int
        L.le_cnn_grad.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                  C.POINTER(C.c_double), _FP, C.c_void_p]
        L.le_cnn_grad.restype = C.c_int
        L.le_cnn_adam.argtypes = [C.c_void_p, C.c_float, C.c_float, C.c_float, C.c_float,
                                  C.c_void_p]
        L.le_cnn_adam.restype = C.c_int
        L.le_cnn_layer_fwd.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p]
        L.le_cnn_layer_fwd.restype = C.c_int
        L.le_cnn_layer_bwd.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.le_cnn_layer_bwd.restype = C.c_int
        L.le_cnn_mfma_probe.argtypes = [_U16, _U16, _FP]
        L.le_cnn_mfma_probe.restype = C.c_int
        L.le_last_error.argtypes = []
        L.le_last_error.restype = C.c_char_p
        L.le_strerror.argtypes = [C.c_int]
        L.le_strerror.restype = C.c_char_p
        _LIB = L
    return _LIB


def strerror(code: int) -> str:
    return lib().le_strerror(code).decode()


def _dp(a):
    return None if a is None else a.ctypes.data_as(_DP)


def _f64(a, shape):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def make_params(params: dict, precision: str = "fp64", stream=None) -> LeParams:
    p = LeParams()
    for k in ("nx", "ny"):
        setattr(p, k, int(params[k]))
    for k in ("lx", "ly", "gdot", "A", "B", "kappa", "M", "eta", "rho", "dt"):
        setattr(p, k, float(params[k]))
    p.precision = {"fp64": LE_FP64, "fp32": LE_FP32}[precision]
    p.stream = stream
    return p


class Context:
    """One run of the sheared model-H step on the GPU."""

    def __init__(self, params: dict, phi0, omega0=None, precision: str = "fp64",
                 stream=None):
        self.params = dict(params)
        self.precision = precision
        self.shape = (int(params["ny"]), int(params["nx"]))
        self._p = make_params(params, precision, stream)
        phi0 = _f64(phi0, self.shape)
        omega0 = _f64(omega0, self.shape)
        h = C.c_void_p()
        rc = lib().le_create(C.byref(self._p), _dp(phi0), _dp(omega0), C.byref(h))
        if rc != LE_OK:
            raise LeError(rc, "le_create")
        self._h = h

    def _check(self):
        if self._h is None:
            raise ValueError("context is closed")

    def step(self, nsteps: int) -> None:
        self._check()
        rc = lib().le_step(self._h, int(nsteps))
        if rc != LE_OK:
            raise LeError(rc, "le_step")

    def set_recovery(self, enable: bool = True) -> None:
        """Stop at the last finite step when a step call goes non-finite."""
        self._check()
        rc = lib().le_set_recovery(self._h, 1 if enable else 0)
        if rc != LE_OK:
            raise LeError(rc, "le_set_recovery")

    def set_scheme(self, f_half: bool = False, midpoint_s: bool = False,
                   upwind3: bool = False, banded: bool = False) -> None:
        """Scheme variants (le_set_scheme): f of the advected phi, and/or the
        sawtooth at the step's midpoint."""
        self._check()
        flags = ((LE_SCHEME_F_HALF if f_half else 0) | (LE_SCHEME_MIDPOINT_S if midpoint_s else 0)
                 | (LE_SCHEME_UPWIND3 if upwind3 else 0) | (LE_SCHEME_BANDED if banded else 0))
        rc = lib().le_set_scheme(self._h, flags)
        if rc != LE_OK:
            raise LeError(rc, "le_set_scheme")

    def observables(self, sk: bool = True):
        """Return (dict of le_obs fields, S(k) array or None)."""
        self._check()
        o = LeObs()
        nb = self.shape[0] // 2
        Sk = np.zeros(nb) if sk else None
        rc = lib().le_observables(self._h, C.byref(o), _dp(Sk), nb if sk else 0)
        if rc != LE_OK:
            raise LeError(rc, "le_observables")
        d = {name: getattr(o, name) for name, _ in LeObs._fields_}
        return d, Sk

    def get_state(self):
        self._check()
        phi = np.empty(self.shape)
        om = np.empty(self.shape)
        psi = np.empty(self.shape)
        step = C.c_int64()
        wraps = C.c_int64()
        rc = lib().le_get_state(self._h, _dp(phi), _dp(om), _dp(psi), C.byref(step),
                                C.byref(wraps))
        if rc != LE_OK:
            raise LeError(rc, "le_get_state")
        return dict(phi=phi, omega=om, psi=psi, step=step.value, wraps=wraps.value)

    def checkpoint(self) -> bytes:
        """The exact stored state as a blob (le_checkpoint_save)."""
        self._check()
        n = C.c_int64()
        rc = lib().le_checkpoint_size(self._h, C.byref(n))
        if rc != LE_OK:
            raise LeError(rc, "le_checkpoint_size")
        buf = C.create_string_buffer(n.value)
        rc = lib().le_checkpoint_save(self._h, buf, n.value)
        if rc != LE_OK:
            raise LeError(rc, "le_checkpoint_save")
        return buf.raw

    def restore(self, blob: bytes) -> None:
        """Load a blob from checkpoint() (le_checkpoint_load)."""
        self._check()
        rc = lib().le_checkpoint_load(self._h, blob, len(blob))
        if rc != LE_OK:
            raise LeError(rc, "le_checkpoint_load")

    def set_state(self, phi, omega, psi, step: int, wraps: int) -> None:
        self._check()
        phi = _f64(phi, self.shape)
        omega = _f64(omega, self.shape)
        psi = _f64(psi, self.shape)
        rc = lib().le_set_state(self._h, _dp(phi), _dp(omega), _dp(psi), int(step), int(wraps))
        if rc != LE_OK:
            raise LeError(rc, "le_set_state")

    def profile(self, enable: bool) -> None:
        """Enable (and clear) or disable per-stage event timing."""
        self._check()
        rc = lib().le_profile(self._h, 1 if enable else 0)
        if rc != LE_OK:
            raise LeError(rc, "le_profile")

    def stage_times(self):
        """Dict stage -> (accumulated ms, launches)."""
        self._check()
        ms = np.zeros(LE_NSTAGES)
        n = (C.c_int64 * LE_NSTAGES)()
        rc = lib().le_stage_times(self._h, _dp(ms), n, LE_NSTAGES)
        if rc != LE_OK:
            raise LeError(rc, "le_stage_times")
        return {STAGES[k]: (float(ms[k]), int(n[k])) for k in range(LE_NSTAGES)}

    def time_stage(self, stage: str, reps: int = 100) -> float:
        """Average microseconds of one launch of `stage` (back-to-back launches;
        the state is not advanced)."""
        self._check()
        ms = C.c_double()
        rc = lib().le_time_stage(self._h, STAGES.index(stage), reps, C.byref(ms))
        if rc != LE_OK:
            raise LeError(rc, "le_time_stage")
        return ms.value * 1e3

    def tuning(self):
        """Kernel variants the autotuner chose for this run (list of one dict)."""
        self._check()
        return _tuning(lib().le_tuning, self._h, "le_tuning")

    def corrector_load(self, params, scales) -> None:
        """Install the corrector network (FP32 weight vector, 4 scales)."""
        self._check()
        p = np.ascontiguousarray(params, dtype=np.float32)
        sc = np.ascontiguousarray(scales, dtype=np.float32)
        rc = lib().le_corrector_load(self._h, p.ctypes.data_as(C.POINTER(C.c_float)), p.size,
                                     sc.ctypes.data_as(C.POINTER(C.c_float)))
        if rc != LE_OK:
            raise LeError(rc, "le_corrector_load")

    def corrector_projection(self, mode: int) -> None:
        """0: subtract the phi residual's mean; 1: its interpolated tile means."""
        self._check()
        rc = lib().le_corrector_projection(self._h, int(mode))
        if rc != LE_OK:
            raise LeError(rc, "le_corrector_projection")

    def step_corrected(self, ncoarse: int) -> None:
        self._check()
        rc = lib().le_step_corrected(self._h, int(ncoarse))
        if rc != LE_OK:
            raise LeError(rc, "le_step_corrected")

    def corrector_audit(self, every: int, window: int, tol: float) -> None:
        """Audit the corrected run against the plain step (le_corrector_audit)."""
        self._check()
        rc = lib().le_corrector_audit(self._h, int(every), int(window), float(tol))
        if rc != LE_OK:
            raise LeError(rc, "le_corrector_audit")

    def corrector_status(self):
        """(fallback, audits, last relative L_s deviation)."""
        self._check()
        fb, n, dev = C.c_int32(), C.c_int64(), C.c_double()
        rc = lib().le_corrector_status(self._h, C.byref(fb), C.byref(n), C.byref(dev))
        if rc != LE_OK:
            raise LeError(rc, "le_corrector_status")
        return bool(fb.value), n.value, dev.value

    def restrict(self, factor: int):
        """(phi, omega) block means over factor x factor cells."""
        self._check()
        shape = (self.shape[0] // factor, self.shape[1] // factor)
        phi, om = np.empty(shape), np.empty(shape)
        rc = lib().le_restrict(self._h, int(factor), _dp(phi), _dp(om))
        if rc != LE_OK:
            raise LeError(rc, "le_restrict")
        return phi, om

    def set_fields(self, phi, omega, step: int) -> None:
        self._check()
        phi = _f64(phi, self.shape)
        omega = _f64(omega, self.shape)
        rc = lib().le_set_fields(self._h, _dp(phi), _dp(omega), int(step))
        if rc != LE_OK:
            raise LeError(rc, "le_set_fields")

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            lib().le_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass



class Batch:
    """Many independent runs advanced together (one launch per stage and shape)."""

    def __init__(self, params_list, phi0s, omega0s=None, precisions=None, stream=None):
        n = len(params_list)
        if n < 1 or len(phi0s) != n:
            raise ValueError("need one phi0 per run")
        precisions = precisions or ["fp64"] * n
        self.shapes = [(int(p["ny"]), int(p["nx"])) for p in params_list]
        arr = (LeParams * n)()
        for i, p in enumerate(params_list):
            arr[i] = make_params(p, precisions[i], stream)
        self._keep = [_f64(a, self.shapes[i]) for i, a in enumerate(phi0s)]
        phis = (_DP * n)(*[_dp(a) for a in self._keep])
        oms = None
        if omega0s is not None:
            self._keep_om = [None if a is None else _f64(a, self.shapes[i])
                             for i, a in enumerate(omega0s)]
            oms = (_DP * n)(*[_dp(a) if a is not None else None for a in self._keep_om])
        h = C.c_void_p()
        rc = lib().le_batch_create(n, arr, phis, oms, C.byref(h))
        if rc != LE_OK:
            raise LeError(rc, "le_batch_create")
        self._h = h
        self.n = n
        self._keep = None
        self._keep_om = None

    def set_scheme(self, f_half: bool = False, midpoint_s: bool = False,
                   upwind3: bool = False, banded: bool = False) -> None:
        """Scheme variants for every run (le_batch_set_scheme)."""
        flags = ((LE_SCHEME_F_HALF if f_half else 0) | (LE_SCHEME_MIDPOINT_S if midpoint_s else 0)
                 | (LE_SCHEME_UPWIND3 if upwind3 else 0) | (LE_SCHEME_BANDED if banded else 0))
        rc = lib().le_batch_set_scheme(self._h, flags)
        if rc != LE_OK:
            raise LeError(rc, "le_batch_set_scheme")

    def step(self, nsteps: int) -> None:
        rc = lib().le_batch_step(self._h, int(nsteps))
        if rc != LE_OK:
            raise LeError(rc, "le_batch_step")

    def observables(self, run: int, sk: bool = True):
        o = LeObs()
        if not 0 <= run < self.n:
            rc = lib().le_batch_observables(self._h, int(run), C.byref(o), None, 0)
            raise LeError(rc, "le_batch_observables")
        nb = self.shapes[run][0] // 2
        Sk = np.zeros(nb) if sk else None
        rc = lib().le_batch_observables(self._h, int(run), C.byref(o), _dp(Sk), nb if sk else 0)
        if rc != LE_OK:
            raise LeError(rc, "le_batch_observables")
        return {name: getattr(o, name) for name, _ in LeObs._fields_}, Sk

    def get_state(self, run: int):
        if not 0 <= run < self.n:   # let the library reject it
            rc = lib().le_batch_get_state(self._h, int(run), None, None, None, None, None)
            raise LeError(rc, "le_batch_get_state")
        shape = self.shapes[run]
        phi, om, psi = np.empty(shape), np.empty(shape), np.empty(shape)
        step, wraps = C.c_int64(), C.c_int64()
        rc = lib().le_batch_get_state(self._h, int(run), _dp(phi), _dp(om), _dp(psi),
                                      C.byref(step), C.byref(wraps))
        if rc != LE_OK:
            raise LeError(rc, "le_batch_get_state")
        return dict(phi=phi, omega=om, psi=psi, step=step.value, wraps=wraps.value)

    def profile(self, enable: bool) -> None:
        rc = lib().le_batch_profile(self._h, 1 if enable else 0)
        if rc != LE_OK:
            raise LeError(rc, "le_batch_profile")

    def tuning(self):
        """Kernel variants the autotuner chose, one dict per group of runs."""
        return _tuning(lib().le_batch_tuning, self._h, "le_batch_tuning")

    def stage_times(self):
        ms = np.zeros(LE_NSTAGES)
        n = (C.c_int64 * LE_NSTAGES)()
        rc = lib().le_batch_stage_times(self._h, _dp(ms), n, LE_NSTAGES)
        if rc != LE_OK:
            raise LeError(rc, "le_batch_stage_times")
        return {STAGES[k]: (float(ms[k]), int(n[k])) for k in range(LE_NSTAGES)}

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            lib().le_batch_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    return None if t is None else C.c_void_p(t.data_ptr())


def step_noalloc(params: dict, phi, omega, psi, step0: int, nsteps: int, stream=None) -> None:
    """le_step_noalloc on caller device buffers (torch float64 CUDA tensors of
    shape (ny, nx), C-contiguous; omega may be None when rho == 0), advanced in
    place from step step0 by nsteps steps."""
    p = make_params(params, "fp64", stream)
    shape = (int(params["ny"]), int(params["nx"]))
    for t in (phi, omega, psi):
        if t is None:
            continue
        if (tuple(t.shape) != shape or not t.is_cuda or not t.is_contiguous()
                or str(t.dtype) != "torch.float64"):
            raise ValueError("step_noalloc: fields must be contiguous float64 CUDA tensors "
                             f"of shape {shape}")
    rc = lib().le_step_noalloc(C.byref(p), _ptr(phi), _ptr(omega), _ptr(psi), int(step0),
                               int(nsteps))
    if rc != LE_OK:
        raise LeError(rc, "le_step_noalloc")


class Net:
    """The corrector network with training state on the GPU.

    Tensors passed in are torch device tensors (FP32 planes [B][2][H][W], or
    the per-layer BF16 bit patterns as int16); the library reads and writes
    them in place.
    """

    def __init__(self, H: int, W: int):
        h = C.c_void_p()
        rc = lib().le_cnn_create(int(H), int(W), C.byref(h))
        if rc != LE_OK:
            raise LeError(rc, "le_cnn_create")
        self._h = h
        self.H, self.W = H, W

    @staticmethod
    def nparams() -> int:
        return lib().le_cnn_nparams()

    def set_params(self, params, scales) -> None:
        p = np.ascontiguousarray(params, dtype=np.float32)
        sc = np.ascontiguousarray(scales, dtype=np.float32)
        rc = lib().le_cnn_set_params(self._h, p.ctypes.data_as(C.POINTER(C.c_float)), p.size,
                                     sc.ctypes.data_as(C.POINTER(C.c_float)))
        if rc != LE_OK:
            raise LeError(rc, "le_cnn_set_params")

    def get_params(self) -> np.ndarray:
        p = np.empty(self.nparams(), dtype=np.float32)
        rc = lib().le_cnn_get_params(self._h, p.ctypes.data_as(C.POINTER(C.c_float)), p.size)
        if rc != LE_OK:
            raise LeError(rc, "le_cnn_get_params")
        return p

    def forward(self, x, r, stream=None) -> None:
        rc = lib().le_cnn_forward(self._h, _ptr(x), _ptr(r), stream)
        if rc != LE_OK:
            raise LeError(rc, "le_cnn_forward")

    def grad(self, xs, ts, batch: int, want_grad: bool = False, stream=None):
        loss = C.c_double()
        g = np.empty(self.nparams(), dtype=np.float32) if want_grad else None
        rc = lib().le_cnn_grad(self._h, _ptr(xs), _ptr(ts), int(batch), C.byref(loss),
                               None if g is None else g.ctypes.data_as(C.POINTER(C.c_float)),
                               stream)
        if rc != LE_OK:
            raise LeError(rc, "le_cnn_grad")
        return loss.value, g

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
             stream=None) -> None:
        rc = lib().le_cnn_adam(self._h, lr, beta1, beta2, eps, stream)
        if rc != LE_OK:
            raise LeError(rc, "le_cnn_adam")

    def layer_fwd(self, layer, a_in, z_out, a_out=None, stream=None) -> None:
        rc = lib().le_cnn_layer_fwd(self._h, int(layer), _ptr(a_in), _ptr(z_out), _ptr(a_out),
                                    stream)
        if rc != LE_OK:
            raise LeError(rc, "le_cnn_layer_fwd")

    def layer_bwd(self, layer, dz, a_in, zprev=None, dzprev=None, dw=None, stream=None) -> None:
        rc = lib().le_cnn_layer_bwd(self._h, int(layer), _ptr(dz), _ptr(a_in), _ptr(zprev),
                                    _ptr(dzprev), _ptr(dw), stream)
        if rc != LE_OK:
            raise LeError(rc, "le_cnn_layer_bwd")

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            lib().le_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mfma_probe(a_bits: np.ndarray, b_bits: np.ndarray) -> np.ndarray:
    """c = a b on one matrix-core tile (BF16 bit patterns in, FP32 out)."""
    a = np.ascontiguousarray(a_bits, dtype=np.uint16)
    b = np.ascontiguousarray(b_bits, dtype=np.uint16)
    c = np.empty((32, 32), dtype=np.float32)
    rc = lib().le_cnn_mfma_probe(a.ctypes.data_as(C.POINTER(C.c_uint16)),
                                 b.ctypes.data_as(C.POINTER(C.c_uint16)),
                                 c.ctypes.data_as(C.POINTER(C.c_float)))
    if rc != LE_OK:
        raise LeError(rc, "le_cnn_mfma_probe")
    return c
