"""Thin ctypes binding of libahom (argument marshalling only).

Every step of the computation runs in the HIP library; this module only
converts Python/numpy arguments to pointers and sizes.  Importing it fails
loudly if the library has not been built.

Device-resident arguments (MEM_DEVICE) are objects with a ``data_ptr()``
method: ``DeviceArray`` below, which allocates through the HIP runtime that
the library itself links, or any other device allocation of the same
runtime.  PyTorch wheels bundle a HIP runtime of their own; two runtimes in
one process are not supported by this binding.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libahom.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"libahom.so not built at {_LIB_PATH}; run __graft_entry__.build()")
_lib = ct.CDLL(_LIB_PATH)

AHOM_OK = 0
AHOM_W_NOT_CONVERGED = 1
AHOM_E_ARG = -1
AHOM_E_SINGULAR = -2
AHOM_E_OVERFLOW = -3
AHOM_E_UNSUPPORTED_SIZE = -4
AHOM_E_MATERIAL = -5
AHOM_E_DIVERGED = -6
AHOM_E_DEVICE = -7
AHOM_E_NOMEM = -8
FP64 = 0
FP32_MIXED = 1
MEM_HOST = 0
MEM_DEVICE = 1
NYQUIST_HERMITIAN = 0
STOP_RESIDUAL = 0
STOP_CAUCHY = 1
SCHEME_BASIC = 0
SCHEME_CG = 1
ELASTICITY = 0
CONDUCTIVITY = 1

EXPORTS = [
    "ahom_version", "ahom_last_error", "ahom_pattern_create", "ahom_pattern_create_transformed", "ahom_pattern_destroy",
    "ahom_pattern_info",
    "ahom_pattern_points", "ahom_pattern_freqs", "ahom_dft", "ahom_dft_noalloc", "ahom_solver_create", "ahom_solver_destroy",
    "ahom_solver_set_material", "ahom_solver_set_stiffness_field", "ahom_solver_set_reference", "ahom_solve",
    "ahom_solver_set_conductivity", "ahom_solver_set_reference_conductivity", "ahom_solve_conductivity",
    "ahom_effective_conductivity", "ahom_solver_last_starts",
    "ahom_effective_stiffness", "ahom_solver_last_timing", "ahom_solver_last_restarts", "ahom_solver_history",
    "ahom_solver_pass_times", "ahom_solver_cauchy_history", "ahom_batch_create", "ahom_batch_create_transformed",
    "ahom_batch_destroy", "ahom_batch_member_info",
    "ahom_batch_member_points", "ahom_batch_set_material", "ahom_batch_set_reference", "ahom_batch_solve",
    "ahom_batch_strain", "ahom_batch_history", "ahom_batch_cauchy_history", "ahom_batch_last_timing", "ahom_batch_member_variant",
    "ahom_guess_create", "ahom_guess_destroy", "ahom_guess_num_params", "ahom_guess_get_params", "ahom_guess_set_params",
    "ahom_guess_add_sample", "ahom_guess_num_samples", "ahom_guess_clear_samples", "ahom_guess_gradients",
    "ahom_guess_train",
    "ahom_guess_adam_step", "ahom_guess_infer", "ahom_guess_predict_sample", "ahom_guess_save", "ahom_guess_load",
    "ahom_conv3d",
]


class Config(ct.Structure):
    _fields_ = [("precision", ct.c_int), ("tol", ct.c_double), ("max_iter", ct.c_int),
                ("check_period", ct.c_int), ("nyquist", ct.c_int), ("stream", ct.c_void_p),
                ("resid_period", ct.c_int), ("refine", ct.c_double), ("stop_rule", ct.c_int), ("scheme", ct.c_int), ("physics", ct.c_int),
                ("guess_probe", ct.c_int)]


_P = ct.c_void_p
_i64p = ct.POINTER(ct.c_int64)
_dp = ct.POINTER(ct.c_double)
_ip = ct.POINTER(ct.c_int)

_lib.ahom_version.restype = ct.c_int
_lib.ahom_last_error.restype = ct.c_char_p
_lib.ahom_pattern_create.argtypes = [ct.c_int, _i64p, ct.POINTER(_P)]
_lib.ahom_pattern_create_transformed.argtypes = [ct.c_int, _i64p, _dp, ct.POINTER(_P)]
_lib.ahom_pattern_destroy.argtypes = [_P]
_lib.ahom_pattern_destroy.restype = None
_lib.ahom_pattern_info.argtypes = [_P, _i64p, _ip, _i64p, _i64p, _i64p]
_lib.ahom_pattern_points.argtypes = [_P, _i64p]
_lib.ahom_pattern_freqs.argtypes = [_P, _i64p]
_lib.ahom_dft.argtypes = [_P, ct.c_int, ct.c_int, _P, _P, ct.c_int, _P]
_lib.ahom_dft_noalloc.argtypes = [_P, ct.c_int, ct.c_int, _P, _P, _P]
_lib.ahom_solver_create.argtypes = [_P, ct.POINTER(Config), ct.POINTER(_P)]
_lib.ahom_solver_destroy.argtypes = [_P]
_lib.ahom_solver_destroy.restype = None
_lib.ahom_solver_set_material.argtypes = [_P, ct.c_int, _dp, _P, ct.c_int]
_lib.ahom_solver_set_stiffness_field.argtypes = [_P, _P, ct.c_int]
_lib.ahom_solver_set_reference.argtypes = [_P, ct.c_double, ct.c_double]
_lib.ahom_solve.argtypes = [_P, ct.c_int, _dp, _P, _P, _ip, _dp, _dp, ct.c_int]
_lib.ahom_effective_stiffness.argtypes = [_P, _dp, _ip]
_lib.ahom_solver_set_conductivity.argtypes = [_P, ct.c_int, _dp, _P, ct.c_int]
_lib.ahom_solver_set_reference_conductivity.argtypes = [_P, ct.c_double]
_lib.ahom_solve_conductivity.argtypes = [_P, ct.c_int, _dp, _P, _ip, _dp, _dp, ct.c_int]
_lib.ahom_effective_conductivity.argtypes = [_P, _dp, _ip]
_lib.ahom_solver_last_timing.argtypes = [_P, _dp, _ip]
_lib.ahom_solver_last_restarts.argtypes = [_P, _ip]
_lib.ahom_solver_last_starts.argtypes = [_P, _ip, ct.c_int]
_lib.ahom_solver_history.argtypes = [_P, ct.c_int, _dp, ct.c_int, _ip]
_lib.ahom_solver_cauchy_history.argtypes = [_P, ct.c_int, _dp, ct.c_int, _ip]
_lib.ahom_solver_pass_times.argtypes = [_P, ct.c_int, _dp, _dp, ct.c_int, _ip]
_lib.ahom_batch_create.argtypes = [ct.c_int, ct.c_int, _i64p, _P, ct.POINTER(_P)]
_lib.ahom_batch_create_transformed.argtypes = [ct.c_int, ct.c_int, _i64p, _dp, ct.POINTER(Config), ct.POINTER(_P)]
_lib.ahom_batch_destroy.argtypes = [_P]
_lib.ahom_batch_destroy.restype = None
_lib.ahom_batch_member_info.argtypes = [_P, ct.c_int, _i64p, _i64p]
_lib.ahom_batch_member_points.argtypes = [_P, ct.c_int, _i64p]
_lib.ahom_batch_set_material.argtypes = [_P, ct.c_int, ct.c_int, _dp, _P]
_lib.ahom_batch_set_reference.argtypes = [_P, ct.c_int, ct.c_double, ct.c_double]
_lib.ahom_batch_solve.argtypes = [_P, ct.c_int, _dp, _ip, _dp, _dp, _ip, ct.c_int]
_lib.ahom_batch_strain.argtypes = [_P, ct.c_int, ct.c_int, _dp]
_lib.ahom_batch_history.argtypes = [_P, ct.c_int, ct.c_int, _dp, ct.c_int, _ip]
_lib.ahom_batch_cauchy_history.argtypes = [_P, ct.c_int, ct.c_int, _dp, ct.c_int, _ip]
_lib.ahom_batch_last_timing.argtypes = [_P, _dp, _ip]
_lib.ahom_batch_member_variant.argtypes = [_P, ct.c_int, _ip]
_fp = ct.POINTER(ct.c_float)
_lib.ahom_guess_create.argtypes = [ct.c_int, ct.c_int, ct.c_uint64, _P, ct.POINTER(_P)]
_lib.ahom_guess_destroy.argtypes = [_P]
_lib.ahom_guess_destroy.restype = None
_lib.ahom_guess_num_params.argtypes = [_P, _i64p]
_lib.ahom_guess_get_params.argtypes = [_P, _fp]
_lib.ahom_guess_set_params.argtypes = [_P, _fp]
_lib.ahom_guess_add_sample.argtypes = [_P, _P, ct.c_int, _dp, ct.c_double, ct.c_double, _P, ct.c_int]
_lib.ahom_guess_num_samples.argtypes = [_P, _ip]
_lib.ahom_guess_clear_samples.argtypes = [_P]
_lib.ahom_guess_gradients.argtypes = [_P, _ip, ct.c_int, _fp, _dp]
_lib.ahom_guess_train.argtypes = [_P, ct.c_int, ct.c_int, ct.c_double, _dp]
_lib.ahom_guess_adam_step.argtypes = [_P, _fp, ct.c_double]
_lib.ahom_guess_infer.argtypes = [_P, ct.c_int, _dp, ct.c_double, ct.c_double, _P, ct.c_int, _dp, _P, ct.c_int]
_lib.ahom_guess_predict_sample.argtypes = [_P, ct.c_int, _fp]
_lib.ahom_guess_save.argtypes = [_P, ct.c_char_p]
_lib.ahom_guess_load.argtypes = [_P, ct.c_char_p]
_lib.ahom_conv3d.argtypes = [ct.c_int, ct.c_int, ct.c_int, ct.c_int, ct.c_int, ct.c_int, _fp, _fp, _fp, _fp, _fp, _fp]


class AhomError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ahom error {code}: {msg}")
        self.code = code


def _check(rc, allow=(AHOM_OK,)):
    if rc not in allow:
        raise AhomError(rc, _lib.ahom_last_error().decode())
    return rc


def version():
    return _lib.ahom_version()


def _ptr(a, ctype):
    return a.ctypes.data_as(ct.POINTER(ctype))


def _is_device(x):
    return hasattr(x, "data_ptr")


# the HIP runtime the library is linked against (already loaded with it)
_hip = ct.CDLL("libamdhip64.so.7")
_hip.hipMalloc.argtypes = [ct.POINTER(ct.c_void_p), ct.c_size_t]
_hip.hipFree.argtypes = [ct.c_void_p]
_hip.hipMemcpy.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_int]
_hip.hipGetDeviceCount.argtypes = [ct.POINTER(ct.c_int)]
_HIP_H2D, _HIP_D2H, _HIP_D2D = 1, 2, 3


def device_count():
    """Number of HIP devices visible to the library's runtime (0 if none)."""
    n = ct.c_int(0)
    return n.value if _hip.hipGetDeviceCount(ct.byref(n)) == 0 else 0


class DeviceArray:
    """A device allocation of the library's HIP runtime with a numpy shape/dtype."""

    def __init__(self, shape, dtype):
        self.shape = tuple(int(v) for v in np.atleast_1d(shape))
        self.dtype = np.dtype(dtype)
        self.nbytes = int(np.prod(self.shape)) * self.dtype.itemsize
        p = ct.c_void_p()
        rc = _hip.hipMalloc(ct.byref(p), max(self.nbytes, 1))
        if rc != 0:
            raise AhomError(AHOM_E_DEVICE, f"hipMalloc of {self.nbytes} bytes failed ({rc})")
        self._p = p

    @classmethod
    def from_numpy(cls, a):
        a = np.ascontiguousarray(a)
        d = cls(a.shape, a.dtype)
        if d.nbytes and _hip.hipMemcpy(d._p, a.ctypes.data, d.nbytes, _HIP_H2D) != 0:
            raise AhomError(AHOM_E_DEVICE, "hipMemcpy to device failed")
        return d

    def numpy(self):
        out = np.empty(self.shape, self.dtype)
        if self.nbytes and _hip.hipMemcpy(out.ctypes.data, self._p, self.nbytes, _HIP_D2H) != 0:
            raise AhomError(AHOM_E_DEVICE, "hipMemcpy to host failed")
        return out

    def copy_from(self, other):
        """Device-to-device copy of another DeviceArray of the same size."""
        if other.nbytes != self.nbytes:
            raise ValueError("size mismatch")
        if self.nbytes and _hip.hipMemcpy(self._p, other._p, self.nbytes, _HIP_D2D) != 0:
            raise AhomError(AHOM_E_DEVICE, "hipMemcpy device to device failed")

    def data_ptr(self):
        return self._p.value

    def __del__(self):
        if getattr(self, "_p", None) and self._p.value:
            _hip.hipFree(self._p)
            self._p = ct.c_void_p()


class Pattern:
    """P(M) with the library's Smith-normal-form addressing (host only).

    L: optional real d x d cell matrix of the transformed pattern P_L(M)
    (Def. 3.3); points sit at L y, frequencies at L^{-T} h.
    """

    def __init__(self, M, L=None):
        M = np.ascontiguousarray(np.asarray(M, dtype=np.int64))
        if M.ndim != 2 or M.shape[0] != M.shape[1]:
            raise ValueError("M must be square")
        self.d = M.shape[0]
        self.M = M
        h = _P()
        if L is None:
            self.L = None
            _check(_lib.ahom_pattern_create(self.d, _ptr(M, ct.c_int64), ct.byref(h)))
        else:
            Lm = np.ascontiguousarray(np.asarray(L, dtype=np.float64))
            if Lm.shape != (self.d, self.d):
                raise ValueError("L must be d x d")
            self.L = Lm
            _check(_lib.ahom_pattern_create_transformed(self.d, _ptr(M, ct.c_int64), _ptr(Lm, ct.c_double), ct.byref(h)))
        self._h = h
        m = ct.c_int64()
        dM = ct.c_int()
        e = np.zeros(self.d, np.int64)
        Q = np.zeros(self.d * self.d, np.int64)
        R = np.zeros(self.d * self.d, np.int64)
        _check(_lib.ahom_pattern_info(h, ct.byref(m), ct.byref(dM), _ptr(e, ct.c_int64), _ptr(Q, ct.c_int64), _ptr(R, ct.c_int64)))
        self.m, self.dM, self.e = int(m.value), int(dM.value), e
        self.Q, self.R = Q.reshape(self.d, self.d), R.reshape(self.d, self.d)

    def points(self):
        out = np.zeros((self.m, self.d), np.int64)
        _check(_lib.ahom_pattern_points(self._h, _ptr(out, ct.c_int64)))
        return out

    def freqs(self):
        out = np.zeros((self.m, self.d), np.int64)
        _check(_lib.ahom_pattern_freqs(self._h, _ptr(out, ct.c_int64)))
        return out

    def dft(self, a, sign=-1, precision=FP64, stream=None, out=None):
        """Pattern DFT of m complex values (numpy: host path; DeviceArray: device path)."""
        if _is_device(a):
            if out is None:
                out = DeviceArray(a.shape, a.dtype)
            _check(_lib.ahom_dft(self._h, sign, precision, a.data_ptr(), out.data_ptr(), MEM_DEVICE, stream))
            return out
        dt = np.complex128 if precision == FP64 else np.complex64
        a = np.ascontiguousarray(np.asarray(a, dtype=dt))
        if a.size != self.m:
            raise ValueError("need m values")
        out = np.empty_like(a)
        _check(_lib.ahom_dft(self._h, sign, precision, a.ctypes.data, out.ctypes.data, MEM_HOST, None))
        return out

    def dft_noalloc(self, a, out, sign=-1, precision=FP64, stream=None):
        """The pattern DFT through the library's static scratch (no device allocation); a, out: DeviceArray."""
        _check(_lib.ahom_dft_noalloc(self._h, sign, precision, a.data_ptr(), out.data_ptr(), stream))
        return out

    def __del__(self):
        if getattr(self, "_h", None):
            _lib.ahom_pattern_destroy(self._h)
            self._h = None


class Solver:
    """Algorithm 1 on a pattern (device buffers owned by the library)."""

    def __init__(self, pattern, precision=FP64, tol=1e-8, max_iter=1000, check_period=8, stream=None, resid_period=1,
                 refine=0.0, stop_rule=0, scheme=SCHEME_BASIC, physics=ELASTICITY, guess_probe=0):
        """stop_rule: STOP_RESIDUAL (r(n) <= tol) or STOP_CAUCHY (the Sec. 5.2 criterion);
        scheme: SCHEME_BASIC (Algorithm 1) or SCHEME_CG (conjugate gradients);
        physics: ELASTICITY or CONDUCTIVITY; guess_probe: updates run from both the
        initial guess and the plain start before keeping the better one (0: off)."""
        self.pattern = pattern
        self.physics = physics
        self.ncomp = (6 if pattern.d == 3 else 3) if physics == ELASTICITY else pattern.d
        self.cfg = Config(precision, tol, max_iter, check_period, NYQUIST_HERMITIAN, stream, resid_period, refine,
                          stop_rule, scheme, physics, guess_probe)
        h = _P()
        _check(_lib.ahom_solver_create(pattern._h, ct.byref(self.cfg), ct.byref(h)))
        self._h = h

    def set_material(self, lame, phase):
        lame = np.ascontiguousarray(np.asarray(lame, dtype=np.float64).reshape(-1, 2))
        if _is_device(phase):
            _check(_lib.ahom_solver_set_material(self._h, lame.shape[0], _ptr(lame, ct.c_double), phase.data_ptr(), MEM_DEVICE))
        else:
            ph = np.ascontiguousarray(np.asarray(phase, dtype=np.uint8))
            _check(_lib.ahom_solver_set_material(self._h, lame.shape[0], _ptr(lame, ct.c_double), ph.ctypes.data, MEM_HOST))

    def set_stiffness_field(self, lame_pts):
        lp = np.ascontiguousarray(np.asarray(lame_pts, dtype=np.float64).reshape(-1, 2))
        _check(_lib.ahom_solver_set_stiffness_field(self._h, lp.ctypes.data, MEM_HOST))

    def set_reference(self, lam0, mu0):
        _check(_lib.ahom_solver_set_reference(self._h, float(lam0), float(mu0)))

    def solve(self, eps_bar, init=None, want_strain=False, allow=(AHOM_OK, AHOM_W_NOT_CONVERGED)):
        """eps_bar: (n_load, 3, 3).  Returns dict(status, iters, resid, mean_stress, strain)."""
        eb = np.ascontiguousarray(np.asarray(eps_bar, dtype=np.float64).reshape(-1, 9))
        n = eb.shape[0]
        iters = np.zeros(n, np.int32)
        resid = np.zeros(n, np.float64)
        mean = np.zeros((n, 9), np.float64)
        strain = np.empty((n, self.ncomp, self.pattern.m), np.float64) if want_strain else None
        init_arr = None
        if init is not None:
            init_arr = np.ascontiguousarray(np.asarray(init, dtype=np.float64).reshape(n, self.ncomp, self.pattern.m))
        rc = _lib.ahom_solve(self._h, n, _ptr(eb, ct.c_double),
                             init_arr.ctypes.data if init_arr is not None else None,
                             strain.ctypes.data if strain is not None else None,
                             _ptr(iters, ct.c_int), _ptr(resid, ct.c_double), _ptr(mean, ct.c_double), MEM_HOST)
        _check(rc, allow)
        return dict(status=rc, iters=iters, resid=resid, mean_stress=mean.reshape(n, 3, 3), strain=strain)

    def solve_device(self, eps_bar, strain_out=None, init=None, allow=(AHOM_OK, AHOM_W_NOT_CONVERGED)):
        """Like solve() with device-resident field arrays (DeviceArray, float64)."""
        eb = np.ascontiguousarray(np.asarray(eps_bar, dtype=np.float64).reshape(-1, 9))
        n = eb.shape[0]
        iters = np.zeros(n, np.int32)
        resid = np.zeros(n, np.float64)
        mean = np.zeros((n, 9), np.float64)
        rc = _lib.ahom_solve(self._h, n, _ptr(eb, ct.c_double),
                             init.data_ptr() if init is not None else None,
                             strain_out.data_ptr() if strain_out is not None else None,
                             _ptr(iters, ct.c_int), _ptr(resid, ct.c_double), _ptr(mean, ct.c_double), MEM_DEVICE)
        _check(rc, allow)
        return dict(status=rc, iters=iters, resid=resid, mean_stress=mean.reshape(n, 3, 3))

    def effective_stiffness(self, allow=(AHOM_OK, AHOM_W_NOT_CONVERGED)):
        k = self.ncomp
        C = np.zeros(k * k, np.float64)
        iters = np.zeros(k, np.int32)
        rc = _lib.ahom_effective_stiffness(self._h, _ptr(C, ct.c_double), _ptr(iters, ct.c_int))
        _check(rc, allow)
        return C.reshape(k, k), iters

    def set_conductivity(self, k, phase):
        k = np.ascontiguousarray(np.asarray(k, dtype=np.float64).reshape(-1))
        if _is_device(phase):
            _check(_lib.ahom_solver_set_conductivity(self._h, k.size, _ptr(k, ct.c_double), phase.data_ptr(), MEM_DEVICE))
        else:
            ph = np.ascontiguousarray(np.asarray(phase, dtype=np.uint8))
            _check(_lib.ahom_solver_set_conductivity(self._h, k.size, _ptr(k, ct.c_double), ph.ctypes.data, MEM_HOST))

    def set_reference_conductivity(self, k0):
        _check(_lib.ahom_solver_set_reference_conductivity(self._h, float(k0)))

    def solve_conductivity(self, grad_bar, want_field=False, allow=(AHOM_OK, AHOM_W_NOT_CONVERGED)):
        """grad_bar: (n_load, 3).  Returns dict(status, iters, resid, mean_flux (n_load, 3), field (n_load, d, m))."""
        g = np.ascontiguousarray(np.asarray(grad_bar, dtype=np.float64).reshape(-1, 3))
        n = g.shape[0]
        iters = np.zeros(n, np.int32)
        resid = np.zeros(n, np.float64)
        mean = np.zeros((n, 3), np.float64)
        field = np.empty((n, self.pattern.d, self.pattern.m), np.float64) if want_field else None
        rc = _lib.ahom_solve_conductivity(self._h, n, _ptr(g, ct.c_double), field.ctypes.data if field is not None else None,
                                          _ptr(iters, ct.c_int), _ptr(resid, ct.c_double), _ptr(mean, ct.c_double), MEM_HOST)
        _check(rc, allow)
        return dict(status=rc, iters=iters, resid=resid, mean_flux=mean, field=field)

    def effective_conductivity(self, allow=(AHOM_OK, AHOM_W_NOT_CONVERGED)):
        d = self.pattern.d
        K = np.zeros(d * d, np.float64)
        iters = np.zeros(d, np.int32)
        rc = _lib.ahom_effective_conductivity(self._h, _ptr(K, ct.c_double), _ptr(iters, ct.c_int))
        _check(rc, allow)
        return K.reshape(d, d), iters

    def last_timing(self):
        ms = ct.c_double()
        enq = ct.c_int()
        _check(_lib.ahom_solver_last_timing(self._h, ct.byref(ms), ct.byref(enq)))
        return ms.value, enq.value

    def last_starts(self, n):
        """Per load of the last solve: 1 if the initial guess was kept, 0 for the plain start."""
        w = np.zeros(n, np.int32)
        _check(_lib.ahom_solver_last_starts(self._h, _ptr(w, ct.c_int), n))
        return w

    def last_restarts(self):
        """FP64 defect-correction restarts of the last solve."""
        n = ct.c_int()
        _check(_lib.ahom_solver_last_restarts(self._h, ct.byref(n)))
        return n.value

    def pass_times(self, n_iter=10):
        """Mean ms per pass and algorithmic bytes per launch (profiling mode)."""
        ms = np.zeros(32, np.float64)
        by = np.zeros(32, np.float64)
        n = ct.c_int()
        _check(_lib.ahom_solver_pass_times(self._h, n_iter, _ptr(ms, ct.c_double), _ptr(by, ct.c_double), 32, ct.byref(n)))
        return ms[: n.value], by[: n.value]

    def history(self, load=0, cap=100000):
        out = np.zeros(cap, np.float64)
        cnt = ct.c_int()
        _check(_lib.ahom_solver_history(self._h, load, _ptr(out, ct.c_double), cap, ct.byref(cnt)))
        return out[:cnt.value]

    def cauchy_history(self, load=0, cap=100000):
        """|eps(n+1) - eps(n)| / |eps(0)| per iteration (-1 where not evaluated)."""
        out = np.zeros(cap, np.float64)
        cnt = ct.c_int()
        _check(_lib.ahom_solver_cauchy_history(self._h, load, _ptr(out, ct.c_double), cap, ct.byref(cnt)))
        return out[:cnt.value]

    def __del__(self):
        if getattr(self, "_h", None):
            _lib.ahom_solver_destroy(self._h)
            self._h = None


class Batch:
    """Many patterns (same dimension) solved in one persistent device launch."""

    def __init__(self, Ms, precision=FP64, tol=1e-8, max_iter=1000, resid_period=1, refine=0.0, stream=None, cells=None):
        Ms = [np.asarray(M, dtype=np.int64) for M in Ms]
        self.d = Ms[0].shape[0]
        if any(M.shape != (self.d, self.d) for M in Ms):
            raise ValueError("all members need d x d matrices of one d")
        self.n = len(Ms)
        self.ncomp = 6 if self.d == 3 else 3
        flat = np.ascontiguousarray(np.stack(Ms).reshape(-1))
        self.cfg = Config(precision, tol, max_iter, 1, NYQUIST_HERMITIAN, stream, resid_period, refine)
        h = _P()
        if cells is None:
            _check(_lib.ahom_batch_create(self.d, self.n, _ptr(flat, ct.c_int64), ct.byref(self.cfg), ct.byref(h)))
        else:
            Ls = np.ascontiguousarray(np.asarray(cells, dtype=np.float64).reshape(self.n, self.d, self.d))
            _check(_lib.ahom_batch_create_transformed(self.d, self.n, _ptr(flat, ct.c_int64), _ptr(Ls, ct.c_double),
                                                      ct.byref(self.cfg), ct.byref(h)))
        self._h = h
        self.nload = 0

    def info(self, i):
        m = ct.c_int64()
        e = np.zeros(self.d, np.int64)
        _check(_lib.ahom_batch_member_info(self._h, i, ct.byref(m), _ptr(e, ct.c_int64)))
        return int(m.value), e

    def points(self, i):
        m, _ = self.info(i)
        out = np.zeros((m, self.d), np.int64)
        _check(_lib.ahom_batch_member_points(self._h, i, _ptr(out, ct.c_int64)))
        return out

    def set_material(self, i, lame, phase):
        lame = np.ascontiguousarray(np.asarray(lame, dtype=np.float64).reshape(-1, 2))
        ph = np.ascontiguousarray(np.asarray(phase, dtype=np.uint8))
        _check(_lib.ahom_batch_set_material(self._h, i, lame.shape[0], _ptr(lame, ct.c_double), ph.ctypes.data))

    def set_reference(self, i, lam0, mu0):
        _check(_lib.ahom_batch_set_reference(self._h, i, float(lam0), float(mu0)))

    def solve(self, eps_bar, use_graph=False, allow=(AHOM_OK, AHOM_W_NOT_CONVERGED)):
        """eps_bar: (n_load, 3, 3).  Arrays indexed [member, load]."""
        eb = np.ascontiguousarray(np.asarray(eps_bar, dtype=np.float64).reshape(-1, 9))
        nl = eb.shape[0]
        iters = np.zeros(self.n * nl, np.int32)
        resid = np.zeros(self.n * nl, np.float64)
        mean = np.zeros((self.n * nl, 9), np.float64)
        status = np.zeros(self.n * nl, np.int32)
        rc = _lib.ahom_batch_solve(self._h, nl, _ptr(eb, ct.c_double), _ptr(iters, ct.c_int), _ptr(resid, ct.c_double),
                                   _ptr(mean, ct.c_double), _ptr(status, ct.c_int), 1 if use_graph else 0)
        _check(rc, allow)
        self.nload = nl
        return dict(status=rc, iters=iters.reshape(self.n, nl), resid=resid.reshape(self.n, nl),
                    mean_stress=mean.reshape(self.n, nl, 3, 3), item_status=status.reshape(self.n, nl))

    def strain(self, i, load):
        m, _ = self.info(i)
        out = np.zeros((self.ncomp, m), np.float64)
        _check(_lib.ahom_batch_strain(self._h, i, load, _ptr(out, ct.c_double)))
        return out

    def history(self, i, load, cap=100000):
        h = np.zeros(cap, np.float64)
        n = ct.c_int()
        _check(_lib.ahom_batch_history(self._h, i, load, _ptr(h, ct.c_double), cap, ct.byref(n)))
        return h[: n.value]

    def cauchy_history(self, i, load, cap=100000):
        h = np.zeros(cap, np.float64)
        n = ct.c_int()
        _check(_lib.ahom_batch_cauchy_history(self._h, i, load, _ptr(h, ct.c_double), cap, ct.byref(n)))
        return h[: n.value]

    def last_timing(self):
        ms = ct.c_double()
        r = ct.c_int()
        _check(_lib.ahom_batch_last_timing(self._h, ct.byref(ms), ct.byref(r)))
        return ms.value, r.value

    def variant(self, i):
        v = ct.c_int()
        _check(_lib.ahom_batch_member_variant(self._h, i, ct.byref(v)))
        return v.value

    def __del__(self):
        if getattr(self, "_h", None):
            _lib.ahom_batch_destroy(self._h)
            self._h = None


def _f32(a):
    return None if a is None else np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def conv3d(n, cin, cout, mode, x=None, w=None, b=None, dy=None, relu=False, batch=1):
    """One periodic 3x3x3 convolution through the network kernels (mode 0 fwd, 1 adjoint, 2 weight gradient)."""
    x, w, b, dy = _f32(x), _f32(w), _f32(b), _f32(dy)
    P = n ** 3
    if mode == 0:
        out = np.zeros((batch, P, cout), np.float32)
    elif mode == 1:
        out = np.zeros((batch, P, cin), np.float32)
    else:
        out = np.zeros((cout, 27, cin), np.float32)
    db = np.zeros(cout, np.float32) if mode == 2 else None
    p = lambda a: None if a is None else a.ctypes.data_as(_fp)  # noqa: E731
    _check(_lib.ahom_conv3d(n, batch, cin, cout, mode, 1 if relu else 0, p(x), p(w), p(b), p(dy), p(out), p(db)))
    return (out, db) if mode == 2 else out


class Guess:
    """Learned initial guess (BF16 matrix-core network) on diag(n, n, n) grids."""

    def __init__(self, n, batch=4, seed=0, stream=None):
        h = _P()
        _check(_lib.ahom_guess_create(n, batch, seed, stream, ct.byref(h)))
        self._h = h
        self.n = n
        self.P = n ** 3
        k = ct.c_int64()
        _check(_lib.ahom_guess_num_params(h, ct.byref(k)))
        self.nparam = int(k.value)

    def params(self):
        out = np.zeros(self.nparam, np.float32)
        _check(_lib.ahom_guess_get_params(self._h, out.ctypes.data_as(_fp)))
        return out

    def set_params(self, w):
        w = np.ascontiguousarray(np.asarray(w, dtype=np.float32))
        assert w.size == self.nparam
        _check(_lib.ahom_guess_set_params(self._h, w.ctypes.data_as(_fp)))

    def add_sample(self, phase, lame, lam0, mu0, strain):
        """strain: solved strain of the 6 Mandel unit loads, (6, 6, n^3) host array or DeviceArray."""
        lame = np.ascontiguousarray(np.asarray(lame, dtype=np.float64).reshape(-1, 2))
        if _is_device(phase):
            ph_ptr, flags = phase.data_ptr(), MEM_DEVICE
            assert _is_device(strain)
            st_ptr = strain.data_ptr()
        else:
            ph = np.ascontiguousarray(np.asarray(phase, dtype=np.uint8))
            st = np.ascontiguousarray(np.asarray(strain, dtype=np.float64))
            ph_ptr, st_ptr, flags = ph.ctypes.data, st.ctypes.data, MEM_HOST
        _check(_lib.ahom_guess_add_sample(self._h, ph_ptr, lame.shape[0], _ptr(lame, ct.c_double), float(lam0), float(mu0),
                                          st_ptr, flags))

    def num_samples(self):
        n = ct.c_int()
        _check(_lib.ahom_guess_num_samples(self._h, ct.byref(n)))
        return n.value

    def clear_samples(self):
        _check(_lib.ahom_guess_clear_samples(self._h))

    def gradients(self, samples):
        idx = np.ascontiguousarray(np.asarray(samples, dtype=np.int32))
        g = np.zeros(self.nparam, np.float32)
        loss = ct.c_double()
        _check(_lib.ahom_guess_gradients(self._h, _ptr(idx, ct.c_int), idx.size, g.ctypes.data_as(_fp), ct.byref(loss)))
        return loss.value, g

    def train(self, steps, batch, lr):
        losses = np.zeros(max(steps, 1), np.float64)
        _check(_lib.ahom_guess_train(self._h, steps, batch, float(lr), _ptr(losses, ct.c_double)))
        return losses[:steps]

    def adam_step(self, grad, lr):
        g = np.ascontiguousarray(np.asarray(grad, dtype=np.float32))
        _check(_lib.ahom_guess_adam_step(self._h, g.ctypes.data_as(_fp), float(lr)))

    def infer(self, phase, lame, lam0, mu0, eps_bar, out=None):
        """Initial fluctuation (n_load, 6, n^3) for strains eps_bar (n_load, 3, 3); out: DeviceArray or None (host)."""
        lame = np.ascontiguousarray(np.asarray(lame, dtype=np.float64).reshape(-1, 2))
        ph = np.ascontiguousarray(np.asarray(phase, dtype=np.uint8))
        eb = np.ascontiguousarray(np.asarray(eps_bar, dtype=np.float64).reshape(-1, 9))
        nl = eb.shape[0]
        if out is None:
            host = np.zeros((nl, 6, self.P), np.float64)
            _check(_lib.ahom_guess_infer(self._h, lame.shape[0], _ptr(lame, ct.c_double), float(lam0), float(mu0), ph.ctypes.data,
                                         nl, _ptr(eb, ct.c_double), host.ctypes.data, MEM_HOST))
            return host
        _check(_lib.ahom_guess_infer(self._h, lame.shape[0], _ptr(lame, ct.c_double), float(lam0), float(mu0), ph.ctypes.data,
                                     nl, _ptr(eb, ct.c_double), out.data_ptr(), MEM_DEVICE))
        return out

    def predict_sample(self, i):
        out = np.zeros((self.P, 36), np.float32)
        _check(_lib.ahom_guess_predict_sample(self._h, i, out.ctypes.data_as(_fp)))
        return out

    def save(self, path):
        _check(_lib.ahom_guess_save(self._h, str(path).encode()))

    def load(self, path):
        _check(_lib.ahom_guess_load(self._h, str(path).encode()))

    def __del__(self):
        if getattr(self, "_h", None):
            _lib.ahom_guess_destroy(self._h)
            self._h = None
