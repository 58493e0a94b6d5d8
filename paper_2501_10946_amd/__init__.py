"""MI355X (gfx950) library for the random batch sum-of-Gaussians (RBSOG)
force evaluation and velocity-Verlet step of 3-D periodic Yukawa systems.

This module is the Python binding of the C-ABI in ``include/rbsog.h``: each
function has the C name and only marshals arguments (torch tensors become
device pointers, the current torch stream becomes the HIP stream).  Every step
of the computation runs in the HIP kernels of ``librbsog.so``; there is no
Python or CPU fallback.  Loading fails loudly if the library is not built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librbsog.so")

RBSOG_OK = 0
RBSOG_EINVAL, RBSOG_ENOROOT, RBSOG_EWORKSPACE, RBSOG_EAGAIN, RBSOG_ENONFINITE, RBSOG_EHIP, RBSOG_ENOMEM = range(-1, -8, -1)
RBSOG_FP64, RBSOG_MIXED = 0, 1
RBSOG_ADAPTIVE, RBSOG_FLAT, RBSOG_K2, RBSOG_DH4PI = 0, 1, 2, 3
# doubles per energy row: U_N, U*_F, U_k0, U_self, U_bg, KE, W_N, W*_F
ENERGY_COLS = 8
RBSOG_SAMPLER_IID, RBSOG_SAMPLER_MH = 0, 1
RBSOG_BATH_NONE, RBSOG_BATH_LANGEVIN, RBSOG_BATH_NOSE_HOOVER, RBSOG_BATH_BERENDSEN = 0, 1, 2, 3
RBSOG_AUTO = -999
RBSOG_MAX_GAUSS = 32


class RbsogError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"rbsog error {code}: {msg}")
        self.code = code


class rbsog_sog(C.Structure):
    _fields_ = [("lambda_", C.c_double), ("r_c", C.c_double), ("eps", C.c_double),
                ("h", C.c_double), ("t0", C.c_double), ("w", C.c_double),
                ("M1", C.c_int), ("M2", C.c_int), ("n", C.c_int),
                ("c", C.c_double * RBSOG_MAX_GAUSS), ("s", C.c_double * RBSOG_MAX_GAUSS),
                ("A", C.c_double * RBSOG_MAX_GAUSS), ("B", C.c_double * RBSOG_MAX_GAUSS),
                ("F0", C.c_double), ("Fhat0", C.c_double), ("max_err", C.c_double),
                ("smooth", C.c_int), ("sigma", C.c_double),
                ("nyuk", C.c_int), ("nu", C.c_double), ("ya", C.c_double * 2), ("yl", C.c_double * 2)]


class rbsog_params(C.Structure):
    _fields_ = [("N", C.c_int64), ("L", C.c_double), ("kT", C.c_double), ("P", C.c_int), ("mmax", C.c_int),
                ("seed", C.c_uint64), ("replica", C.c_uint32), ("precision", C.c_int), ("density", C.c_int),
                ("skin", C.c_double), ("full_k", C.c_int), ("sampler", C.c_int), ("Ly", C.c_double),
                ("Lz", C.c_double)]


RBSOG_NUM_KERNEL_CLASSES = 9
KERNEL_CLASSES = ("cells", "kick_drift", "sample", "rho_partial", "rho_reduce", "near", "far", "energy", "nlist")


class rbsog_timing(C.Structure):
    _fields_ = [("ms", C.c_double * RBSOG_NUM_KERNEL_CLASSES), ("launches", C.c_int64 * RBSOG_NUM_KERNEL_CLASSES)]


class rbsog_info(C.Structure):
    _fields_ = [("N", C.c_int64), ("nc", C.c_int), ("mmax", C.c_int), ("nshell", C.c_int), ("nlat", C.c_int64),
                ("S", C.c_double), ("Q1", C.c_double), ("Q2", C.c_double), ("ws_bytes", C.c_size_t),
                ("skin", C.c_double), ("nf", C.c_int), ("near_capacity", C.c_int), ("near_poly", C.c_int),
                ("nc_y", C.c_int), ("nc_z", C.c_int)]


_lib = None
_p = C.c_void_p
_sizes = {}  # handle address -> (N, P, ncell) for argument-size checks


def lib() -> C.CDLL:
    """The loaded librbsog.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        sig = {
            "rbsog_sog_init_egs": (C.c_int, [C.c_double, C.c_double, C.c_double, C.c_double, C.c_int,
                                             C.POINTER(rbsog_sog)]),
            "rbsog_sog_init": (C.c_int, [C.c_double, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int,
                                         C.POINTER(rbsog_sog)]),
            "rbsog_sog_expand": (C.c_int, [C.POINTER(rbsog_sog)]),
            "rbsog_sog_near_poly": (C.c_int, [C.POINTER(rbsog_sog), _p, _p]),
            "rbsog_workspace_size": (C.c_int, [C.POINTER(rbsog_params), C.POINTER(rbsog_sog), C.POINTER(C.c_size_t)]),
            "rbsog_create": (C.c_int, [C.POINTER(rbsog_params), C.POINTER(rbsog_sog), _p, _p, _p, C.c_size_t, _p,
                                       C.POINTER(_p)]),
            "rbsog_get_info": (C.c_int, [_p, C.POINTER(rbsog_info)]),
            "rbsog_build_cells": (C.c_int, [_p, _p, _p, _p]),
            "rbsog_sample_k": (C.c_int, [_p, C.c_uint64, _p, _p]),
            "rbsog_compute_rho": (C.c_int, [_p, C.c_uint64, _p, _p]),
            "rbsog_compute_forces": (C.c_int, [_p, C.c_uint64, _p, _p, _p, _p]),
            "rbsog_step": (C.c_int, [_p, _p, _p, _p, C.c_uint64, C.c_int, C.c_double, _p]),
            "rbsog_check": (C.c_int, [_p]),
            "rbsog_set_kT": (C.c_int, [_p, C.c_double]),
            "rbsog_set_thermostat": (C.c_int, [_p, C.c_double, C.c_double]),
            "rbsog_timing_enable": (C.c_int, [_p, C.c_int]),
            "rbsog_timing_read": (C.c_int, [_p, C.POINTER(rbsog_timing)]),
            "rbsog_destroy": (None, [_p]),
            "rbsog_ens_create": (C.c_int, [C.c_size_t, C.c_int, _p, C.POINTER(_p)]),
            "rbsog_ens_bytes": (C.c_int, [C.POINTER(rbsog_params), C.POINTER(rbsog_sog), C.c_int,
                                          C.POINTER(C.c_size_t)]),
            "rbsog_ens_admit": (C.c_int, [_p, C.POINTER(rbsog_params), C.POINTER(rbsog_sog), _p, _p, _p, _p, C.c_int,
                                          C.c_double, C.POINTER(C.c_int)]),
            "rbsog_ens_step": (C.c_int, [_p]),
            "rbsog_ens_poll": (C.c_int, [_p, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
            "rbsog_ens_retire": (C.c_int, [_p, C.c_int, _p, _p, _p]),
            "rbsog_ens_status": (C.c_int, [_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_uint64),
                                           C.POINTER(C.c_size_t)]),
            "rbsog_ens_step_time": (C.c_int, [_p, C.c_uint64, C.POINTER(C.c_double)]),
            "rbsog_ens_destroy": (None, [_p]),
            "rbsog_rho_noalloc": (C.c_int, [C.c_int64, C.c_double, _p, _p, C.c_int, _p, C.c_int, _p, _p]),
            "rbsog_ssf_scratch_size": (C.c_int, [C.c_int64, C.c_int, C.POINTER(C.c_size_t)]),
            "rbsog_ssf": (C.c_int, [C.c_int64, C.c_double, _p, _p, C.c_int, _p, C.c_size_t, _p, _p]),
            "rbsog_rdf": (C.c_int, [_p, _p, C.c_double, C.c_int, _p]),
            "rbsog_set_bath": (C.c_int, [_p, C.c_int, C.c_double, C.c_double]),
            "rbsog_bath_state": (C.c_int, [_p, C.POINTER(C.c_double)]),
            "rbsog_track": (C.c_int, [C.c_int64, C.c_double, _p, _p, _p, _p]),
            "rbsog_track_box": (C.c_int, [C.c_int64, C.c_double, C.c_double, C.c_double, _p, _p, _p, _p]),
            "rbsog_msd_scratch_size": (C.c_int, [C.POINTER(C.c_size_t)]),
            "rbsog_msd_vacf": (C.c_int, [C.c_int64, _p, _p, _p, _p, C.c_size_t, _p, _p]),
            "rbsog_last_error": (C.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(code: int) -> int:
    if code != RBSOG_OK:
        raise RbsogError(code, lib().rbsog_last_error().decode())
    return code


def _dptr(t, dtype=None, numel: Optional[int] = None):
    """Device pointer of a contiguous torch tensor (None passes through)."""
    if t is None:
        return None
    import torch
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected dtype {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"expected at least {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _stream(device=None) -> C.c_void_p:
    import torch
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


# --- host functions ---------------------------------------------------------------

def rbsog_sog_init(lambda_: float, r_c: float, eps: float, M1: int = RBSOG_AUTO, M2: int = RBSOG_AUTO,
                   smooth: int = 1) -> rbsog_sog:
    out = rbsog_sog()
    _check(lib().rbsog_sog_init(lambda_, r_c, eps, smooth, M1, M2, C.byref(out)))
    return out


def rbsog_sog_init_egs(lambda_: float, nu: float, r_c: float, eps: float, smooth: int = 1) -> rbsog_sog:
    out = rbsog_sog()
    _check(lib().rbsog_sog_init_egs(lambda_, nu, r_c, eps, smooth, C.byref(out)))
    return out


def rbsog_sog_expand(sog: rbsog_sog) -> rbsog_sog:
    _check(lib().rbsog_sog_expand(C.byref(sog)))
    return sog


def rbsog_sog_near_poly(sog: rbsog_sog):
    """(degree, h[29], k[29]): the FP64 pair kernel's polynomials H(r) = r^3 (F_N1 + F_N2)
    and K(r) = r (Y - F) in y = 2 r / r_c - 1 (degree 0: declined)."""
    import numpy as np
    h = np.zeros(29)
    k = np.zeros(29)
    r = lib().rbsog_sog_near_poly(C.byref(sog), C.c_void_p(h.ctypes.data), C.c_void_p(k.ctypes.data))
    if r < 0:
        _check(r)
    return int(r), h, k


def sog_from_parameters(lambda_: float, r_c: float, h: float, t0: float, w: float, M1: int, M2: int,
                        eps: float = 0.0, sigma: float = None) -> rbsog_sog:
    """A decomposition given by its parameters (h, t0, w, M1, M2, and sigma for
    the C2 form), expanded by the library."""
    s = rbsog_sog()
    s.lambda_, s.r_c, s.eps, s.h, s.t0, s.w, s.M1, s.M2 = lambda_, r_c, eps, h, t0, w, M1, M2
    s.n = M1 + M2 + 1
    s.smooth, s.sigma = (1, 1.0) if sigma is None else (2, sigma)
    return rbsog_sog_expand(s)


def sog_from_gaussians(lambda_: float, r_c: float, c, s, A, B, ya=None, yl=None, nu: float = 0.0,
                       eps: float = 0.0, smooth: int = 1) -> rbsog_sog:
    """A decomposition given by its Gaussians (F = sum c exp(-s r^2), Fhat =
    sum A exp(-B k^2)) and, for the EGS kernel, its two Yukawa terms (weights
    ya, lengths yl).  F(0) and Fhat(0) are summed in list order."""
    n = len(c)
    if not 1 <= n <= RBSOG_MAX_GAUSS or not len(s) == len(A) == len(B) == n:
        raise ValueError(f"need 1..{RBSOG_MAX_GAUSS} Gaussians with matching c, s, A, B")
    out = rbsog_sog()
    out.lambda_, out.r_c, out.eps, out.smooth = lambda_, r_c, eps, smooth
    out.M1, out.M2, out.n = n - 1, 0, n
    out.sigma = 1.0
    for j in range(n):
        out.c[j], out.s[j], out.A[j], out.B[j] = float(c[j]), float(s[j]), float(A[j]), float(B[j])
    out.F0 = sum(float(v) for v in c)
    out.Fhat0 = sum(float(v) for v in A)
    if yl is not None:
        out.nyuk, out.nu = 2, nu
        out.ya[0], out.ya[1] = float(ya[0]), float(ya[1])
        out.yl[0], out.yl[1] = float(yl[0]), float(yl[1])
    return out


def make_params(N: int, L, kT: float, P: int, seed: int, replica: int = 0, mmax: int = 0,
                precision: int = RBSOG_FP64, density: int = RBSOG_ADAPTIVE, skin: float = -1.0,
                full_k: bool = False, sampler: int = 0) -> rbsog_params:
    """L: one edge (a cube) or the three edges (L_x, L_y, L_z) of a cuboid."""
    if isinstance(L, (tuple, list)):
        Lx, Ly, Lz = (float(v) for v in L)
    else:
        Lx, Ly, Lz = float(L), 0.0, 0.0
    return rbsog_params(N=N, L=Lx, kT=kT, P=P, mmax=mmax, seed=seed, replica=replica, precision=precision,
                        density=density, skin=skin, full_k=1 if full_k else 0, sampler=sampler, Ly=Ly, Lz=Lz)


def rbsog_workspace_size(params: rbsog_params, sog: rbsog_sog) -> int:
    n = C.c_size_t()
    _check(lib().rbsog_workspace_size(C.byref(params), C.byref(sog), C.byref(n)))
    return n.value


# --- device functions -------------------------------------------------------------

def rbsog_create(params: rbsog_params, sog: rbsog_sog, q, m, ws, stream=None) -> C.c_void_p:
    import torch
    N = params.N
    h = C.c_void_p()
    _check(lib().rbsog_create(C.byref(params), C.byref(sog), _dptr(q, torch.float64, N), _dptr(m, torch.float64, N),
                              _dptr(ws), ws.numel() * ws.element_size(), stream or _stream(q.device), C.byref(h)))
    info = rbsog_get_info(h)
    _sizes[h.value] = (info.N, params.P, info.nc * info.nc_y * info.nc_z)
    return h


def _n(h):
    return _sizes.get(h.value if isinstance(h, C.c_void_p) else h, (None, None, None))


def rbsog_get_info(h) -> rbsog_info:
    out = rbsog_info()
    _check(lib().rbsog_get_info(h, C.byref(out)))
    return out


def rbsog_build_cells(h, x, cell_start=None, order=None):
    import torch
    N, P, nce = _n(h)
    _check(lib().rbsog_build_cells(h, _dptr(x, torch.float64, 3 * N), _dptr(cell_start, torch.int32, nce + 1),
                                   _dptr(order, torch.int32, N)))


def rbsog_sample_k(h, step: int, n=None, coef=None):
    import torch
    N, P, _ = _n(h)
    _check(lib().rbsog_sample_k(h, step, _dptr(n, torch.int32, 3 * P), _dptr(coef, torch.float64, P)))


def rbsog_compute_rho(h, step: int, x, rho):
    import torch
    N, P, _ = _n(h)
    _check(lib().rbsog_compute_rho(h, step, _dptr(x, torch.float64, 3 * N), _dptr(rho, torch.float64, 2 * P)))


def rbsog_compute_forces(h, step: int, x, f, f_near=None, energy=None):
    import torch
    N, P, _ = _n(h)
    _check(lib().rbsog_compute_forces(h, step, _dptr(x, torch.float64, 3 * N), _dptr(f, torch.float64, 3 * N),
                                      _dptr(f_near, torch.float64, 3 * N), _dptr(energy, torch.float64, ENERGY_COLS)))


def rbsog_step(h, x, v, f, step0: int, nsteps: int, dt: float, energy_hist=None):
    import torch
    N, P, _ = _n(h)
    _check(lib().rbsog_step(h, _dptr(x, torch.float64, 3 * N), _dptr(v, torch.float64, 3 * N),
                            _dptr(f, torch.float64, 3 * N), step0, nsteps, dt,
                            _dptr(energy_hist, torch.float64, ENERGY_COLS * nsteps)))


def rbsog_rho_noalloc(x, q, L: float, n, rho, precision: int = RBSOG_FP64, stream=None) -> None:
    """Structure factors of the modes n [P, 3] (int32) into rho [P, 2], with no
    allocation (the library's static scratch array)."""
    import torch
    N = q.numel()
    P = n.shape[0]
    _check(lib().rbsog_rho_noalloc(N, L, _dptr(x, torch.float64, 3 * N), _dptr(q, torch.float64, N), P,
                                   _dptr(n, torch.int32, 3 * P), precision, stream or _stream(x.device),
                                   _dptr(rho, torch.float64, 2 * P)))


def rbsog_set_thermostat(h, friction: float, kT: float) -> None:
    """Langevin bath (BAOAB) for rbsog_step; friction 0 turns it off."""
    _check(lib().rbsog_set_thermostat(h, friction, kT))


def rbsog_ssf_scratch_size(N: int, m_s: int) -> int:
    b = C.c_size_t(0)
    _check(lib().rbsog_ssf_scratch_size(N, m_s, C.byref(b)))
    return b.value


def rbsog_ssf(x, w, L: float, m_s: int, scratch, s, stream=None) -> None:
    """Shell means of |sum_j w_j exp(i k.r_j)|^2 for |n|^2 = 0..m_s into s
    [m_s + 1] (S(k) = s / N with unit weights)."""
    import torch
    N = w.numel()
    _check(lib().rbsog_ssf(N, L, _dptr(x, torch.float64, 3 * N), _dptr(w, torch.float64, N), m_s,
                           _dptr(scratch), scratch.numel() * scratch.element_size(), stream or _stream(x.device),
                           _dptr(s, torch.float64, m_s + 1)))


def rbsog_rdf(h, x, r_max: float, nbins: int, hist) -> None:
    """Adds the ordered-pair counts by distance bin into hist [nbins] (int64)."""
    import torch
    N, P, _ = _n(h)
    _check(lib().rbsog_rdf(h, _dptr(x, torch.float64, 3 * N), r_max, nbins, _dptr(hist, torch.int64, nbins)))


def rbsog_set_bath(h, kind: int, rate: float, kT: float) -> None:
    _check(lib().rbsog_set_bath(h, kind, rate, kT))


def rbsog_bath_state(h):
    """(xi, eta) of a Nose-Hoover bath."""
    out = (C.c_double * 2)()
    _check(lib().rbsog_bath_state(h, out))
    return out[0], out[1]


def rbsog_track(x, L, x_last, disp, stream=None) -> None:
    """disp += minimum-image (x - x_last); x_last = x (device tensors [3, N]);
    L one edge or the three edges of a cuboid."""
    import torch
    N = x.shape[1]
    args = (_dptr(x, torch.float64, 3 * N), _dptr(x_last, torch.float64, 3 * N), _dptr(disp, torch.float64, 3 * N),
            stream or _stream(x.device))
    if isinstance(L, (tuple, list)):
        _check(lib().rbsog_track_box(N, float(L[0]), float(L[1]), float(L[2]), *args))
    else:
        _check(lib().rbsog_track(N, L, *args))


def rbsog_msd_scratch_size() -> int:
    b = C.c_size_t(0)
    _check(lib().rbsog_msd_scratch_size(C.byref(b)))
    return b.value


def rbsog_msd_vacf(disp, v0, v, scratch, out, stream=None) -> None:
    """out[0] = mean |disp|^2, out[1] = mean v0 . v (device tensors)."""
    import torch
    N = disp.shape[1]
    _check(lib().rbsog_msd_vacf(N, _dptr(disp, torch.float64, 3 * N), _dptr(v0, torch.float64, 3 * N),
                                _dptr(v, torch.float64, 3 * N), _dptr(scratch),
                                scratch.numel() * scratch.element_size(), stream or _stream(disp.device),
                                _dptr(out, torch.float64, 2)))


def rbsog_check(h) -> None:
    _check(lib().rbsog_check(h))


def rbsog_set_kT(h, kT: float) -> None:
    """Re-derives the sampling measure with temperature kT (the instantaneous
    temperature of an NVT run); later evaluations draw from it."""
    _check(lib().rbsog_set_kT(h, kT))


def rbsog_timing_enable(h, enable: bool = True) -> None:
    _check(lib().rbsog_timing_enable(h, int(enable)))


def rbsog_timing_read(h) -> dict:
    """{kernel class: (total ms, launches)} accumulated since the last enable/read."""
    t = rbsog_timing()
    _check(lib().rbsog_timing_read(h, C.byref(t)))
    return {name: (t.ms[i], t.launches[i]) for i, name in enumerate(KERNEL_CLASSES)}


def rbsog_destroy(h) -> None:
    _sizes.pop(h.value if isinstance(h, C.c_void_p) else h, None)
    lib().rbsog_destroy(h)


# --- served ensemble -----------------------------------------------------------

def _hptr(a, numel: int):
    """Host pointer of a contiguous float64 numpy array of at least numel elements."""
    import numpy as np
    if not isinstance(a, np.ndarray) or a.dtype != np.float64 or not a.flags.c_contiguous:
        raise ValueError("expected a contiguous float64 numpy array")
    if a.size < numel:
        raise ValueError(f"expected at least {numel} elements, got {a.size}")
    return C.c_void_p(a.ctypes.data)


def rbsog_ens_create(hbm_budget: int, max_slots: int, stream=None) -> C.c_void_p:
    e = _p()
    _check(lib().rbsog_ens_create(hbm_budget, max_slots, stream if stream is not None else _stream(), C.byref(e)))
    return e


def rbsog_ens_bytes(params: rbsog_params, sog: rbsog_sog, nsteps: int) -> int:
    b = C.c_size_t(0)
    _check(lib().rbsog_ens_bytes(C.byref(params), C.byref(sog), nsteps, C.byref(b)))
    return b.value


def rbsog_ens_admit(e, params: rbsog_params, sog: rbsog_sog, x, v, q, m, nsteps: int, dt: float) -> int:
    """Slot of the admitted replica; raises RbsogError (code RBSOG_EAGAIN) when it does not fit now."""
    N = int(params.N)
    slot = C.c_int(-1)
    _check(lib().rbsog_ens_admit(e, C.byref(params), C.byref(sog), _hptr(x, 3 * N), _hptr(v, 3 * N), _hptr(q, N),
                                 _hptr(m, N), nsteps, dt, C.byref(slot)))
    return slot.value


def rbsog_ens_step(e) -> None:
    _check(lib().rbsog_ens_step(e))


def rbsog_ens_poll(e, max_slots: int) -> list:
    buf = (C.c_int * max(1, max_slots))()
    n = C.c_int(0)
    _check(lib().rbsog_ens_poll(e, buf, C.byref(n)))
    return [buf[i] for i in range(n.value)]


def rbsog_ens_retire(e, slot: int, x=None, v=None, energy_hist=None) -> None:
    ptr = lambda a: None if a is None else _hptr(a, 0)
    _check(lib().rbsog_ens_retire(e, slot, ptr(x), ptr(v), ptr(energy_hist)))


def rbsog_ens_status(e) -> dict:
    r, a, n, f = C.c_int(0), C.c_int(0), C.c_uint64(0), C.c_size_t(0)
    _check(lib().rbsog_ens_status(e, C.byref(r), C.byref(a), C.byref(n), C.byref(f)))
    return {"resident": r.value, "active": a.value, "ens_steps": n.value, "pool_free": f.value}


def rbsog_ens_step_time(e, ens_step: int) -> float:
    ms = C.c_double(0.0)
    _check(lib().rbsog_ens_step_time(e, ens_step, C.byref(ms)))
    return ms.value


def rbsog_ens_destroy(e) -> None:
    lib().rbsog_ens_destroy(e)


class System:
    """Holds one system's device buffers (charges, masses, workspace) and
    handle; all work goes through the C-ABI on the current torch stream."""

    def __init__(self, q, m, L, sog: rbsog_sog, kT: float, P: int, seed: int, replica: int = 0,
                 mmax: int = 0, precision: int = RBSOG_FP64, density: int = RBSOG_ADAPTIVE, skin: float = -1.0,
                 full_k: bool = False, device="cuda", sampler: int = 0):
        import torch
        self.q = torch.as_tensor(q, dtype=torch.float64, device=device).contiguous()
        self.m = torch.as_tensor(m, dtype=torch.float64, device=device).contiguous()
        self.N = self.q.numel()
        self.sog = sog
        self.params = make_params(self.N, L, kT, P, seed, replica, mmax, precision, density, skin, full_k, sampler)
        nbytes = rbsog_workspace_size(self.params, sog)
        self.ws = torch.empty(nbytes // 8 + 64, dtype=torch.float64, device=device)
        self.h = rbsog_create(self.params, sog, self.q, self.m, self.ws)
        self.info = rbsog_get_info(self.h)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            try:
                rbsog_destroy(h)
            except (TypeError, AttributeError):   # interpreter shutdown: module globals already gone
                pass
            self.h = None
