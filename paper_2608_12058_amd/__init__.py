"""qwexp: exp(-i t H) psi on the n-qubit hypercube, MI355X (gfx950) HIP kernels.

Thin ctypes binding over ``libqwexp.so`` (C-ABI declared in include/qwexp.h).
Every step of the computation runs in the library; this module only marshals
arguments: torch tensors supply device memory and the current HIP stream.

H = diag(E) + gamma * sum_j X_j with E(z) the Ising energies (given as a device
vector, or generated on the device from the SK couplings h, J).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqwexp.so")

QW_OK, QW_EINVAL, QW_ENOMEM, QW_EHIP, QW_EDIVERGE, QW_ENOCONV = 0, -1, -2, -3, -4, -5
QW_CHEB, QW_CF = 0, 1
_METHODS = {"cheb": QW_CHEB, "chebyshev": QW_CHEB, "cf": QW_CF}
_STATUS = {0: "QW_OK", -1: "QW_EINVAL", -2: "QW_ENOMEM", -3: "QW_EHIP", -4: "QW_EDIVERGE", -5: "QW_ENOCONV"}


class QwError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class QwInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("K", ctypes.c_int), ("passes", ctypes.c_int), ("method", ctypes.c_int),
                ("shift_c", ctypes.c_double), ("radius_r", ctypes.c_double), ("a", ctypes.c_double),
                ("trunc_bound", ctypes.c_double), ("eval_bound", ctypes.c_double),
                ("timing", ctypes.c_int), ("setup_ms", ctypes.c_float), ("loop_ms", ctypes.c_float),
                ("pass_ms", ctypes.c_float * 4), ("monitor", ctypes.c_int), ("growth", ctypes.c_double),
                ("out_norm", ctypes.c_double), ("otf_mask", ctypes.c_int)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["pass_ms"] = list(self.pass_ms)
        return d


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
_sz = ctypes.c_size_t


def _declare(lib):
    lib.qw_last_error.restype = ctypes.c_char_p
    lib.qw_version.restype = ctypes.c_char_p
    lib.qw_workspace_bytes.restype = _sz
    lib.qw_workspace_bytes.argtypes = [_i, _i, _i]
    lib.qw_bessel_j.argtypes = [_d, _i, _dp]
    lib.qw_cheb_coeffs.argtypes = [_d, _d, _i, _i, _dp, ctypes.POINTER(_i), _dp]
    for name in ("qw_spectral_bound_f32", "qw_spectral_bound_f64"):
        f = getattr(lib, name)
        f.argtypes = [_i, _vp, _dp, _dp, _d, _dp, _dp, _vp, _sz, _vp]
    for name in ("qw_expm_action_c64", "qw_expm_action_c128"):
        f = getattr(lib, name)
        f.argtypes = [_i, _vp, _dp, _dp, _d, _d, _vp, _vp, _d, _i, _vp, _sz, _vp, ctypes.POINTER(QwInfo)]
    lib.qw_expm_action_c64_noalloc.argtypes = [_i, _vp, _dp, _dp, _d, _d, _vp, _vp, _d, _i, _vp,
                                               ctypes.POINTER(QwInfo)]
    for name in ("qw_expm_action_c64_bounded", "qw_expm_action_c128_bounded"):
        f = getattr(lib, name)
        f.argtypes = [_i, _vp, _dp, _dp, _d, _d, _d, _d, _vp, _vp, _d, _i, _vp, _sz, _vp, ctypes.POINTER(QwInfo)]
    for name in ("qw_poly_action_c64", "qw_poly_action_c128"):
        f = getattr(lib, name)
        f.argtypes = [_i, _vp, _dp, _dp, _d, _d, _d, _dp, _i, _i, _vp, _vp, _vp, _sz, _vp, ctypes.POINTER(QwInfo)]
    for name in ("qw_anneal_cfet4_c64", "qw_anneal_cfet4_c128"):
        f = getattr(lib, name)
        f.argtypes = [_i, _dp, _dp, _dp, _i, _dp, _i, _d, _i, _d, _vp, _vp, _dp, _i, _vp, _sz, _vp,
                      ctypes.POINTER(CfetInfo)]
    lib.qw_cfet4_step_bound.argtypes = [_i, _dp, _dp, _dp, _i, _dp, _i, _d, _d, _d, _d, _dp]
    lib.qw_debug_check_plan.argtypes = [_i, _i]
    lib.qw_debug_check_plan.restype = _i
    return lib


def lib():
    """Load libqwexp.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2608_12058_amd.build` "
                              "(there is no CPU fallback)")
        _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


def _check(status: int):
    if status != QW_OK:
        raise QwError(status, lib().qw_last_error().decode())


def version() -> str:
    return lib().qw_version().decode()


# ------------------------------------------------------------------ host calls

def bessel_j(a: float, mmax: int) -> np.ndarray:
    out = np.empty(mmax + 1, dtype=np.float64)
    _check(lib().qw_bessel_j(float(a), int(mmax), out.ctypes.data_as(_dp)))
    return out


def cheb_coeffs(a: float, tol: float, method: str = "cheb", kmax: int = 1 << 20) -> tuple[np.ndarray, float]:
    """alpha_0..alpha_K with c_m = (-i)^m alpha_m, and the truncation bound."""
    buf = np.empty(kmax + 1, dtype=np.float64)
    K = _i(0)
    err = _d(0.0)
    _check(lib().qw_cheb_coeffs(float(a), float(tol), _METHODS[method], int(kmax), buf.ctypes.data_as(_dp),
                                ctypes.byref(K), ctypes.byref(err)))
    return buf[:K.value + 1].copy(), err.value


def workspace_bytes(n: int, precision: int = 64, on_the_fly: bool = False) -> int:
    return int(lib().qw_workspace_bytes(int(n), int(precision), 1 if on_the_fly else 0))


# ------------------------------------------------------------------ device calls

def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _host_f64(x, count):
    if x is None:
        return None, None
    arr = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if arr.shape != (count,):
        raise ValueError(f"expected {count} values, got shape {arr.shape}")
    return arr, arr.ctypes.data_as(_dp)


@dataclass
class Workspace:
    """Device scratch for one action call, owned by the caller (torch uint8)."""
    tensor: object
    nbytes: int

    @staticmethod
    def for_problem(n: int, precision: int = 64, on_the_fly: bool = False, device="cuda"):
        torch = _torch()
        nb = workspace_bytes(n, precision, on_the_fly)
        t = torch.empty(nb + 256, dtype=torch.uint8, device=device)
        return Workspace(t, nb)

    def ptr(self) -> int:
        p = self.tensor.data_ptr()
        return (p + 255) & ~255


def _prec_of(psi) -> int:
    torch = _torch()
    if psi.dtype == torch.complex64:
        return 64
    if psi.dtype == torch.complex128:
        return 128
    raise TypeError("psi must be complex64 or complex128")


def spectral_bound(n: int, gamma: float, diag=None, h=None, J=None, precision: int = 64,
                   workspace: Workspace | None = None, stream=None) -> tuple[float, float]:
    """(c, r): shift and induced 1-norm bound of H - cI."""
    torch = _torch()
    if workspace is None:
        workspace = Workspace.for_problem(n, precision, diag is None and n >= 31 and precision == 64)
    _, hp = _host_f64(h, n) if diag is None else (None, None)
    _, Jp = _host_f64(J, n * (n - 1) // 2) if diag is None else (None, None)
    if diag is not None:
        want = torch.float32 if precision == 64 else torch.float64
        if diag.dtype != want or not diag.is_contiguous() or diag.numel() != (1 << n):
            raise ValueError("diag must be a contiguous vector of 2^n energies in the state's real precision")
    c, r = _d(0.0), _d(0.0)
    fn = lib().qw_spectral_bound_f32 if precision == 64 else lib().qw_spectral_bound_f64
    _check(fn(int(n), _vp(diag.data_ptr()) if diag is not None else None, hp, Jp, float(gamma),
              ctypes.byref(c), ctypes.byref(r), _vp(workspace.ptr()), workspace.nbytes, _stream_ptr(stream)))
    return c.value, r.value


def expm_action(psi, gamma: float, t: float, *, diag=None, h=None, J=None, tol: float = 2.0 ** -23,
                method: str = "cheb", out=None, workspace: Workspace | None = None, stream=None,
                timing: int = 0, monitor: bool = False, bound: tuple | None = None):
    """psi(t) = exp(-i t (diag(E) + gamma sum_j X_j)) psi on the GPU.

    psi: contiguous complex64 or complex128 CUDA tensor of length 2^n.
    diag: CUDA tensor of 2^n energies (float32 for complex64, float64 for
    complex128) or None with h (n values) and J (n(n-1)/2 values, packed upper
    triangle) given as host arrays.  timing=1 records HIP events around the
    setup and the Clenshaw loop (info["setup_ms"], info["loop_ms"]) and makes the
    call synchronous; timing=2 also times every pass (info["pass_ms"]).
    monitor=True measures every ||b_k|| and fills info["eval_bound"] (the
    evaluation-error bound of section II.B.3).  bound=(c, r) skips the spectral
    bound read-back and uses the caller's shift and radius, with the monitor on;
    a radius too small to bound the spectrum raises QwError(QW_EDIVERGE).  Returns (psi_out, info dict)."""
    torch = _torch()
    if not (psi.is_cuda and psi.is_contiguous() and psi.dim() == 1):
        raise ValueError("psi must be a contiguous 1-D CUDA tensor")
    N = psi.numel()
    n = N.bit_length() - 1
    if N != (1 << n):
        raise ValueError("len(psi) must be a power of two")
    prec = _prec_of(psi)
    if out is None:
        out = torch.empty_like(psi)
    elif out.dtype != psi.dtype or out.numel() != N or not out.is_contiguous():
        raise ValueError("out must match psi")
    if diag is not None:
        want = torch.float32 if prec == 64 else torch.float64
        if diag.dtype != want or not diag.is_contiguous() or diag.numel() != N or not diag.is_cuda:
            raise ValueError("diag must be a contiguous CUDA vector of 2^n energies in the state's real precision")
        hp = Jp = None
    else:
        if h is None or J is None:
            raise ValueError("give diag, or h and J")
        _h, hp = _host_f64(h, n)
        _J, Jp = _host_f64(J, n * (n - 1) // 2)
    otf = diag is None and n >= 31 and prec == 64
    if workspace is None:
        workspace = Workspace.for_problem(n, prec, otf, device=psi.device)
    info = QwInfo()
    info.timing = int(timing)
    info.monitor = 1 if monitor else 0
    dptr = _vp(diag.data_ptr()) if diag is not None else None
    if bound is None:
        fn = lib().qw_expm_action_c64 if prec == 64 else lib().qw_expm_action_c128
        _check(fn(int(n), dptr, hp, Jp, float(gamma), float(t), _vp(psi.data_ptr()), _vp(out.data_ptr()),
                  float(tol), _METHODS[method], _vp(workspace.ptr()), workspace.nbytes, _stream_ptr(stream),
                  ctypes.byref(info)))
    else:
        fn = lib().qw_expm_action_c64_bounded if prec == 64 else lib().qw_expm_action_c128_bounded
        _check(fn(int(n), dptr, hp, Jp, float(gamma), float(t), float(bound[0]), float(bound[1]),
                  _vp(psi.data_ptr()), _vp(out.data_ptr()), float(tol), _METHODS[method], _vp(workspace.ptr()),
                  workspace.nbytes, _stream_ptr(stream), ctypes.byref(info)))
    return out, info.as_dict()


def expm_action_noalloc(psi, gamma: float, t: float, out, *, diag=None, h=None, J=None,
                        tol: float = 2.0 ** -23, method: str = "cheb", stream=None, timing: int = 0):
    """exp(-i t H) psi in complex64 through qw_expm_action_c64_noalloc: no
    workspace (the library's fixed device scratch, n <= 20) and a caller-given
    out, so nothing is allocated on the device.  Returns the info dict."""
    torch = _torch()
    if not (psi.is_cuda and psi.is_contiguous() and psi.dim() == 1 and psi.dtype == torch.complex64):
        raise ValueError("psi must be a contiguous 1-D complex64 CUDA tensor")
    N = psi.numel()
    n = N.bit_length() - 1
    if N != (1 << n):
        raise ValueError("len(psi) must be a power of two")
    if out.dtype != psi.dtype or out.numel() != N or not out.is_contiguous():
        raise ValueError("out must match psi")
    if diag is not None:
        if diag.dtype != torch.float32 or not diag.is_contiguous() or diag.numel() != N or not diag.is_cuda:
            raise ValueError("diag must be a contiguous float32 CUDA vector of 2^n energies")
        hp = Jp = None
    else:
        if h is None or J is None:
            raise ValueError("give diag, or h and J")
        _h, hp = _host_f64(h, n)
        _J, Jp = _host_f64(J, n * (n - 1) // 2)
    info = QwInfo()
    info.timing = int(timing)
    _check(lib().qw_expm_action_c64_noalloc(int(n), _vp(diag.data_ptr()) if diag is not None else None, hp, Jp,
                                            float(gamma), float(t), _vp(psi.data_ptr()), _vp(out.data_ptr()),
                                            float(tol), _METHODS[method], _stream_ptr(stream), ctypes.byref(info)))
    return info.as_dict()


QW_BASIS_CHEB, QW_BASIS_MONO = 0, 1
_BASES = {"cheb": QW_BASIS_CHEB, "chebyshev": QW_BASIS_CHEB, "mono": QW_BASIS_MONO, "monomial": QW_BASIS_MONO}


def poly_action(psi, coef, gamma: float, *, basis: str = "cheb", diag=None, h=None, J=None,
                shift: float | None = None, radius: float | None = None, out=None,
                workspace: Workspace | None = None, stream=None, timing: int = 0):
    """psi_out = p(H~) psi with H~ = (H - shift) / radius, H = diag(E) + gamma sum_j X_j.

    coef: K + 1 (complex) coefficients, of T_k (basis "cheb": Clenshaw, Alg. 2)
    or of x^k (basis "mono": Horner's rule, Alg. 1).  shift and radius default
    to the spectral bound (spectrum of H~ in [-1, 1]); info["shift_c"] and
    info["radius_r"] report the pair used.  Same state/diagonal conventions as
    expm_action.  Returns (psi_out, info dict)."""
    torch = _torch()
    if not (psi.is_cuda and psi.is_contiguous() and psi.dim() == 1):
        raise ValueError("psi must be a contiguous 1-D CUDA tensor")
    N = psi.numel()
    n = N.bit_length() - 1
    if N != (1 << n):
        raise ValueError("len(psi) must be a power of two")
    prec = _prec_of(psi)
    cf = np.asarray(coef, dtype=np.complex128).ravel()
    if cf.size < 1:
        raise ValueError("need at least one coefficient")
    cpair = np.ascontiguousarray(np.stack([cf.real, cf.imag], axis=1).ravel())
    if out is None:
        out = torch.empty_like(psi)
    elif out.dtype != psi.dtype or out.numel() != N or not out.is_contiguous():
        raise ValueError("out must match psi")
    if diag is not None:
        want = torch.float32 if prec == 64 else torch.float64
        if diag.dtype != want or not diag.is_contiguous() or diag.numel() != N or not diag.is_cuda:
            raise ValueError("diag must be a contiguous CUDA vector of 2^n energies in the state's real precision")
        hp = Jp = None
    else:
        if h is None or J is None:
            raise ValueError("give diag, or h and J")
        _h, hp = _host_f64(h, n)
        _J, Jp = _host_f64(J, n * (n - 1) // 2)
    otf = diag is None and n >= 31 and prec == 64
    if workspace is None:
        workspace = Workspace.for_problem(n, prec, otf, device=psi.device)
    c = 0.0 if shift is None else float(shift)
    r = 0.0 if radius is None else float(radius)
    if (shift is None) != (radius is None):
        raise ValueError("give both shift and radius, or neither")
    info = QwInfo()
    info.timing = int(timing)
    dptr = _vp(diag.data_ptr()) if diag is not None else None
    fn = lib().qw_poly_action_c64 if prec == 64 else lib().qw_poly_action_c128
    _check(fn(int(n), dptr, hp, Jp, float(gamma), c, r, cpair.ctypes.data_as(_dp), int(cf.size - 1),
              _BASES[basis], _vp(psi.data_ptr()), _vp(out.data_ptr()), _vp(workspace.ptr()), workspace.nbytes,
              _stream_ptr(stream), ctypes.byref(info)))
    return out, info.as_dict()


class CfetInfo(ctypes.Structure):
    _fields_ = [("timing", ctypes.c_int), ("steps", ctypes.c_int), ("exponentials", ctypes.c_int),
                ("terms", ctypes.c_longlong), ("err_bound", ctypes.c_double), ("h_min", ctypes.c_double),
                ("h_max", ctypes.c_double), ("comm_bound", ctypes.c_double), ("total_ms", ctypes.c_float)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


def anneal_cfet4(psi, h, J, A, B, T: float, *, steps: int = 0, tol: float = 1e-6, out=None,
                 workspace: Workspace | None = None, stream=None, timing: int = 0, max_record: int = 1 << 16):
    """psi(T) for H(t) = A(t) H_P + B(t) sum_j X_j by fourth-order commutator-free
    Magnus steps (sec. III.B).  A, B: monomial coefficients in s = t / T (e.g.
    A = [0, 1], B = [1, -1] for a linear anneal).  steps > 0: equal steps; 0:
    adaptive steps from the library's bound on the leading local error, with
    tol the total error target.  Returns (psi_out, info dict, step sizes)."""
    torch = _torch()
    if not (psi.is_cuda and psi.is_contiguous() and psi.dim() == 1):
        raise ValueError("psi must be a contiguous 1-D CUDA tensor")
    N = psi.numel()
    n = N.bit_length() - 1
    if N != (1 << n):
        raise ValueError("len(psi) must be a power of two")
    prec = _prec_of(psi)
    _h, hp = _host_f64(h, n)
    _J, Jp = _host_f64(J, n * (n - 1) // 2)
    a = np.ascontiguousarray(np.asarray(A, dtype=np.float64).ravel())
    b = np.ascontiguousarray(np.asarray(B, dtype=np.float64).ravel())
    if out is None:
        out = torch.empty_like(psi)
    elif out.dtype != psi.dtype or out.numel() != N or not out.is_contiguous():
        raise ValueError("out must match psi")
    if workspace is None:
        workspace = Workspace.for_problem(n, prec, n >= 31 and prec == 64, device=psi.device)
    rec = np.zeros(max(1, int(max_record)), dtype=np.float64)
    info = CfetInfo()
    info.timing = int(timing)
    fn = lib().qw_anneal_cfet4_c64 if prec == 64 else lib().qw_anneal_cfet4_c128
    _check(fn(int(n), hp, Jp, a.ctypes.data_as(_dp), int(a.size - 1), b.ctypes.data_as(_dp), int(b.size - 1),
              float(T), int(steps), float(tol), _vp(psi.data_ptr()), _vp(out.data_ptr()), rec.ctypes.data_as(_dp),
              int(rec.size), _vp(workspace.ptr()), workspace.nbytes, _stream_ptr(stream), ctypes.byref(info)))
    d = info.as_dict()
    return out, d, rec[:min(d["steps"], rec.size)].copy()


def cfet4_step_bound(n: int, h, J, A, B, T: float, emin: float, emax: float, t: float) -> float:
    """Host-only: the library's bound on ||E5|| at time t (leading local error per h^5)."""
    _h, hp = _host_f64(h, n)
    _J, Jp = _host_f64(J, n * (n - 1) // 2)
    a = np.ascontiguousarray(np.asarray(A, dtype=np.float64).ravel())
    b = np.ascontiguousarray(np.asarray(B, dtype=np.float64).ravel())
    out = _d(0.0)
    _check(lib().qw_cfet4_step_bound(int(n), hp, Jp, a.ctypes.data_as(_dp), int(a.size - 1), b.ctypes.data_as(_dp),
                                     int(b.size - 1), float(T), float(emin), float(emax), float(t),
                                     ctypes.byref(out)))
    return float(out.value)


def debug_check_plan(n: int, precision: int) -> int:
    """Host-only check of the pass index maps (number of passes, or < 0)."""
    return int(lib().qw_debug_check_plan(int(n), int(precision)))


# ------------------------------------------------------------------ batched form

class BatchItem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("reserved", ctypes.c_int), ("gamma", ctypes.c_double),
                ("t", ctypes.c_double), ("tol", ctypes.c_double), ("off_hJ", ctypes.c_int64),
                ("off_psi", ctypes.c_int64), ("off_out", ctypes.c_int64)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("timing", ctypes.c_int), ("count", ctypes.c_int), ("small_count", ctypes.c_int),
                ("large_count", ctypes.c_int), ("max_K", ctypes.c_int), ("launches", ctypes.c_int),
                ("waves", ctypes.c_int), ("amp_terms", ctypes.c_longlong), ("wave_bytes", ctypes.c_longlong),
                ("setup_ms", ctypes.c_float), ("loop_ms", ctypes.c_float), ("onchip_nmax", ctypes.c_int),
                ("concurrent", ctypes.c_int), ("graph_cached", ctypes.c_int), ("graph_ms", ctypes.c_float),
                ("class_count", ctypes.c_int * 3), ("tile_class", ctypes.c_byte * 23)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["class_count"] = list(self.class_count)
        d["tile_class"] = {n: int(self.tile_class[n]) for n in range(23) if self.tile_class[n] >= 0}
        return d


class BatchSched(ctypes.Structure):
    """Schedule of a batched call (qw_batch_sched): wave_bytes, onchip_nmax,
    concurrent and a tile class per size (-1 = default)."""
    _fields_ = [("wave_bytes", ctypes.c_longlong), ("onchip_nmax", ctypes.c_int), ("concurrent", ctypes.c_int),
                ("tile_class", ctypes.c_byte * 23)]

    @staticmethod
    def make(wave_bytes: int = 0, onchip_nmax: int = 13, concurrent: bool = False, tile_class: dict | None = None):
        S = BatchSched()
        S.wave_bytes, S.onchip_nmax, S.concurrent = int(wave_bytes), int(onchip_nmax), 1 if concurrent else 0
        for n in range(23):
            S.tile_class[n] = -1
        for n, c in (tile_class or {}).items():
            S.tile_class[int(n)] = int(c)
        return S

    def as_dict(self) -> dict:
        return {"wave_bytes": self.wave_bytes, "onchip_nmax": self.onchip_nmax, "concurrent": self.concurrent,
                "tile_class": {n: int(self.tile_class[n]) for n in range(23) if self.tile_class[n] >= 0}}


def _declare_batched(lib):
    if getattr(lib, "_qw_batched_declared", False):
        return
    lib.qw_batched_workspace_bytes_c64.restype = _sz
    lib.qw_batched_workspace_bytes_c64.argtypes = [ctypes.POINTER(BatchItem), _i, _dp]
    lib.qw_expm_action_batched_c64.argtypes = [ctypes.POINTER(BatchItem), _i, _dp, _vp, _vp, _i, _vp, _sz,
                                               ctypes.c_char_p, _vp, ctypes.POINTER(BatchInfo)]
    lib.qw_expm_action_batched_c64_sched.argtypes = [ctypes.POINTER(BatchItem), _i, _dp, _vp, _vp, _i, _vp, _sz,
                                                     ctypes.POINTER(BatchSched), _i, _vp, ctypes.POINTER(BatchInfo)]
    lib.qw_batched_tune_c64.argtypes = [ctypes.POINTER(BatchItem), _i, _dp, _vp, _vp, _vp, _sz,
                                        ctypes.c_char_p, _vp, ctypes.POINTER(BatchSched)]
    lib._qw_batched_declared = True


class Batch:
    """Independent complex64 instances packed for qw_expm_action_batched_c64.

    instances: dicts with n, gamma, t, tol, h, J.  The input states live in one
    device pool (``state(i)`` views), outputs in another (``output(i)``)."""

    def __init__(self, instances, device="cuda"):
        torch = _torch()
        _declare_batched(lib())
        self.count = len(instances)
        self.items = (BatchItem * self.count)()
        hj, off_hj, off = [], 0, 0
        self.offsets = []
        for i, ins in enumerate(instances):
            n = int(ins["n"])
            N = 1 << n
            h = np.asarray(ins["h"], dtype=np.float64).reshape(n)
            J = np.asarray(ins["J"], dtype=np.float64).reshape(n * (n - 1) // 2)
            it = self.items[i]
            it.n, it.gamma, it.t, it.tol = n, float(ins["gamma"]), float(ins["t"]), float(ins.get("tol", 1e-6))
            it.off_hJ, it.off_psi, it.off_out = off_hj, off, off
            hj += [h, J]
            off_hj += n + J.size
            self.offsets.append((off, N))
            off += N + (N & 1)          # keep every state 16-byte aligned
        self.hJ = np.ascontiguousarray(np.concatenate(hj)) if hj else np.zeros(0)
        self.total = off
        self.psi_pool = torch.zeros(max(off, 2), dtype=torch.complex64, device=device)
        self.out_pool = torch.zeros_like(self.psi_pool)
        self.ws_bytes = int(lib().qw_batched_workspace_bytes_c64(self.items, self.count, self.hJ.ctypes.data_as(_dp)))
        if self.ws_bytes == 0:
            raise QwError(QW_EINVAL, lib().qw_last_error().decode())
        self._ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)

    def state(self, i):
        o, N = self.offsets[i]
        return self.psi_pool[o:o + N]

    def output(self, i):
        o, N = self.offsets[i]
        return self.out_pool[o:o + N]

    def ws_ptr(self) -> int:
        return (self._ws.data_ptr() + 255) & ~255


def expm_action_batched(batch: Batch, method: str = "cheb", tune_cache: str | None = None, stream=None,
                        timing: int = 0, wave_bytes: int | None = None, use_graph: bool = True,
                        sched: BatchSched | dict | None = None) -> dict:
    """Run every instance of the batch; outputs land in batch.out_pool.  With
    sched (a BatchSched or the keyword dict of BatchSched.make), wave_bytes or
    use_graph=False the schedule is explicit, otherwise it comes from the tune
    file (or the default)."""
    L = lib()
    _declare_batched(L)
    info = BatchInfo()
    info.timing = int(timing)
    args = (batch.items, batch.count, batch.hJ.ctypes.data_as(_dp), _vp(batch.psi_pool.data_ptr()),
            _vp(batch.out_pool.data_ptr()), _METHODS[method], _vp(batch.ws_ptr()), batch.ws_bytes)
    if sched is None and wave_bytes is None and use_graph:
        st = L.qw_expm_action_batched_c64(*args, tune_cache.encode() if tune_cache else None, _stream_ptr(stream),
                                          ctypes.byref(info))
    else:
        if isinstance(sched, dict):
            sched = BatchSched.make(**sched)
        if sched is None:
            sched = BatchSched.make(wave_bytes=int(wave_bytes or 0))
        elif wave_bytes is not None:
            sched.wave_bytes = int(wave_bytes)
        st = L.qw_expm_action_batched_c64_sched(*args, ctypes.byref(sched), 1 if use_graph else 0,
                                                _stream_ptr(stream), ctypes.byref(info))
    _check(st)
    return info.as_dict()


def batched_tune(batch: Batch, tune_cache: str | None, stream=None) -> dict:
    """Search the schedule of this batch (tile class per size bucket, the
    one-workgroup limit, the side-stream launch, the wave size), append the
    best to tune_cache and return it as a dict."""
    L = lib()
    _declare_batched(L)
    best = BatchSched()
    _check(L.qw_batched_tune_c64(batch.items, batch.count, batch.hJ.ctypes.data_as(_dp),
                                 _vp(batch.psi_pool.data_ptr()), _vp(batch.out_pool.data_ptr()),
                                 _vp(batch.ws_ptr()), batch.ws_bytes, tune_cache.encode() if tune_cache else None,
                                 _stream_ptr(stream), ctypes.byref(best)))
    return best.as_dict()


# ------------------------------------------------------------------ anneal gradient

class GradInfo(ctypes.Structure):
    _fields_ = [("timing", ctypes.c_int), ("passes", ctypes.c_int), ("sum_K", ctypes.c_int),
                ("amp_terms", ctypes.c_longlong), ("total_ms", ctypes.c_float)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


def _declare_grad(lib):
    if getattr(lib, "_qw_grad_declared", False):
        return
    lib.qw_anneal_workspace_bytes_c64.restype = _sz
    lib.qw_anneal_workspace_bytes_c64.argtypes = [_i, _dp, _dp, _i, _dp, _dp, _i]
    lib.qw_anneal_energy_grad_c64.argtypes = [_i, _dp, _dp, _i, _dp, _dp, _vp, _d, _i, _dp, _dp, _dp, _dp, _dp,
                                              _vp, _sz, _vp, _vp, ctypes.POINTER(GradInfo)]
    lib._qw_grad_declared = True


def anneal_energy_grad(h, J, gammas, ts, psi0, tol: float = 2.0 ** -23, ckpt_every: int = 0, stream=None,
                       timing: int = 0, psiT_out=None):
    """E = <psi_S|H_P|psi_S> after the piecewise-constant anneal (gammas, ts) from
    psi0 (complex64 CUDA tensor), and dE/d(gamma, t, h, J).  Returns
    (E, {"gamma", "t", "h", "J"}, info)."""
    torch = _torch()
    L = lib()
    _declare_grad(L)
    if psi0.dtype != torch.complex64 or not psi0.is_cuda or not psi0.is_contiguous():
        raise ValueError("psi0 must be a contiguous complex64 CUDA tensor")
    n = psi0.numel().bit_length() - 1
    S = len(gammas)
    h_, hp = _host_f64(h, n)
    J_, Jp = _host_f64(J, n * (n - 1) // 2)
    g_, gp = _host_f64(gammas, S)
    t_, tp = _host_f64(ts, S)
    nb = int(L.qw_anneal_workspace_bytes_c64(n, hp, Jp, S, gp, tp, int(ckpt_every)))
    if nb == 0:
        raise QwError(QW_EINVAL, L.qw_last_error().decode())
    ws = torch.empty(nb + 256, dtype=torch.uint8, device=psi0.device)
    wsp = (ws.data_ptr() + 255) & ~255
    E = ctypes.c_double(0.0)
    dg, dt = np.zeros(S), np.zeros(S)
    dh, dJ = np.zeros(n), np.zeros(max(n * (n - 1) // 2, 1))
    info = GradInfo()
    info.timing = int(timing)
    _check(L.qw_anneal_energy_grad_c64(n, hp, Jp, S, gp, tp, _vp(psi0.data_ptr()), float(tol), int(ckpt_every),
                                       ctypes.byref(E), dg.ctypes.data_as(_dp), dt.ctypes.data_as(_dp),
                                       dh.ctypes.data_as(_dp), dJ.ctypes.data_as(_dp), _vp(wsp), nb,
                                       _stream_ptr(stream), _vp(psiT_out.data_ptr()) if psiT_out is not None else None,
                                       ctypes.byref(info)))
    return E.value, {"gamma": dg, "t": dt, "h": dh, "J": dJ[:n * (n - 1) // 2]}, info.as_dict()


def _make_anneal_function():
    torch = _torch()

    class AnnealEnergy(torch.autograd.Function):
        """E(gamma, t, h, J) = <psi_S|H_P|psi_S> with the gradient from the
        library's adjoint Clenshaw sweep (one library call computes both)."""

        @staticmethod
        def forward(ctx, gammas, ts, h, J, psi0, tol=2.0 ** -23, ckpt_every=0):
            E, g, _ = anneal_energy_grad(h.detach().cpu().numpy(), J.detach().cpu().numpy(),
                                         gammas.detach().cpu().numpy(), ts.detach().cpu().numpy(), psi0,
                                         tol=tol, ckpt_every=ckpt_every)
            grads = [torch.as_tensor(g[k], dtype=x.dtype, device=x.device)
                     for k, x in (("gamma", gammas), ("t", ts), ("h", h), ("J", J))]
            ctx.save_for_backward(*grads)
            return torch.tensor(E, dtype=torch.float64, device=gammas.device)

        @staticmethod
        def backward(ctx, gE):
            gg, gt, gh, gJ = ctx.saved_tensors
            return gE * gg, gE * gt, gE * gh, gE * gJ, None, None, None

    return AnnealEnergy


_AnnealEnergy = None


def anneal_energy(gammas, ts, h, J, psi0, tol: float = 2.0 ** -23, ckpt_every: int = 0):
    """Differentiable anneal energy: gammas, ts, h, J are float64 tensors
    (requires_grad as needed); psi0 is a complex64 CUDA tensor."""
    global _AnnealEnergy
    if _AnnealEnergy is None:
        _AnnealEnergy = _make_anneal_function()
    return _AnnealEnergy.apply(gammas, ts, h, J, psi0, tol, ckpt_every)
