"""CPU oracle for the RBSOG force evaluation (TEST INFRASTRUCTURE).

A plain FP64 implementation of what the paper computes, written in C
(`rbsog_oracle.c`, built by `oracle.build`) and driven through ctypes.  It is
the reference the GPU library is checked against: only the tests, the smoke
check and the CPU-baseline leg of the benchmark may import it.  It shares no
code with the GPU library, and the library never imports it.

Functions that the paper fixes but the C file does not need (the SOG in its
integral form, the brute-force Yukawa image sum used as a pin) are written
here in numpy.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import dataclasses
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

ADAPTIVE, FLAT, K2, DH4PI = 0, 1, 2, 3

_d = C.c_double
_i = C.c_int
_i64 = C.c_int64
_u64 = C.c_uint64
_u32 = C.c_uint32
_p = C.c_void_p


def build(force: bool = True) -> str:
    from . import build_oracle as _b
    return _b.build(force=force)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        sig = {
            "orc_yukawa": (_d, [_d, _d]),
            "orc_yukawa_dr": (_d, [_d, _d]),
            "orc_f": (_d, [_d, _d, _d]),
            "orc_h_star": (_d, [_d, _d]),
            "orc_sog_w": (_d, [_d, _d, _d, _d, _i, _i]),
            "orc_sog_far": (_d, [_d, _d, _d, _d, _i, _i, _d]),
            "orc_sog_c1_residual": (_d, [_d, _d, _d, _d, _i, _i]),
            "orc_sog_c1_root": (_i, [_d, _d, _d, _i, _i, _p, _p]),
            "orc_sog_maxerr": (_d, [_d, _d, _d, _d, _d, _i, _i]),
            "orc_sog_auto": (_i, [_d, _d, _d, _p, _p, _p, _p, _p, _p]),
            "orc_sog_expand": (None, [_d, _d, _d, _d, _i, _i, _p, _p, _p, _p]),
            "orc_sog_expand_s": (None, [_d, _d, _d, _d, _d, _i, _i, _p, _p, _p, _p]),
            "orc_yukawa_dr2": (_d, [_d, _d]),
            "orc_sog_far2": (_d, [_d, _d, _d, _d, _d, _i, _i, _d]),
            "orc_sog_c2_residual": (_d, [_d, _d, _d, _d, _i, _i]),
            "orc_sog_c2_root": (_i, [_d, _d, _d, _i, _i, _p, _p, _p]),
            "orc_sog_maxerr2": (_d, [_d, _d, _d, _d, _d, _d, _i, _i]),
            "orc_sog_auto2": (_i, [_d, _d, _d, _p, _p, _p, _p, _p, _p, _p]),
            "orc_F": (_d, [_i, _p, _p, _d]),
            "orc_Fhat": (_d, [_i, _p, _p, _d]),
            "orc_Fhat_slope": (_d, [_i, _p, _p, _d]),
            "orc_density": (_d, [_i, _d, _d, _d, _d, _d]),
            "orc_mmax_default": (_i, [_i, _p, _p, _d]),
            "orc_lattice_count": (_i64, [_i]),
            "orc_lattice_build": (None, [_i, _p, _p]),
            "orc_shell_table": (_i, [_i, _p, _i, _p, _p, _d, _i, _d, _d, _d, _i, _p, _p, _p]),
            "orc_philox4x64_10": (None, [_p, _p, _p]),
            "orc_cells": (_i, [_i64, _p, _d, _d, _p, _p]),
            "orc_near": (None, [_i64, _p, _p, _d, _d, _d, _i, _p, _p, _p, _p, _p]),
            "orc_near_subset": (_i, [_i64, _p, _p, _d, _d, _d, _i, _p, _p, _i64, _p, _p]),
            "orc_rho": (None, [_i64, _p, _p, _d, _i, _p, _p]),
            "orc_far_rb": (None, [_i64, _p, _p, _d, _i, _p, _p, _p, _p]),
            "orc_far_rb_energy": (_d, [_i, _p, _p]),
            "orc_far_rb_virial": (_d, [_i, _p, _p, _p, _d, _i, _p, _p]),
            "orc_far_full": (_d, [_i64, _p, _p, _d, _i, _p, _p, _i, _p, _p]),
            "orc_kernel_Y": (_d, [_i, _p, _p, _d]),
            "orc_egs_split": (_i, [_d, _d, _p, _p]),
            "orc_kernel_maxerr": (_d, [_i, _p, _p, _d, _d, _i, _p, _p]),
            "orc_density_k": (_d, [_i, _d, _d, _d, _i, _p, _p, _d]),
            "orc_near_k": (_i, [_i64, _p, _p, _d, _i, _p, _p, _d, _i, _p, _p, _p, _p, _p]),
            "orc_near_subset_k": (_i, [_i64, _p, _p, _d, _i, _p, _p, _d, _i, _p, _p, _i64, _p, _p]),
            "orc_sys_create_k": (_p, [_i64, _d, _i, _p, _p, _d, _d, _i, _i, _u64, _u32, _i, _i, _i, _p, _p, _p, _p,
                                      _p, _p]),
            "orc_cells_box": (None, [_i64, _p, _p, _d, _p, _p, _p]),
            "orc_near_box": (_i, [_i64, _p, _p, _p, _i, _p, _p, _d, _i, _p, _p, _p, _p, _p]),
            "orc_near_subset_box": (_i, [_i64, _p, _p, _p, _i, _p, _p, _d, _i, _p, _p, _i64, _p, _p]),
            "orc_rho_box": (None, [_i64, _p, _p, _p, _i, _p, _p]),
            "orc_far_rb_box": (None, [_i64, _p, _p, _p, _i, _p, _p, _p, _p]),
            "orc_far_rb_virial_box": (_d, [_i, _p, _p, _p, _p, _i, _p, _p]),
            "orc_far_full_box": (_d, [_i64, _p, _p, _p, _i, _p, _p, _p, _p]),
            "orc_box_lattice": (_i64, [_p, _i, _p, _p, _p, _p]),
            "orc_box_draw": (None, [_i, _u64, _u64, _u32, _i64, _p, _p, _p, _p, _p]),
            "orc_rdf_box": (None, [_i64, _p, _p, _d, _i, _p, _p]),
            "orc_sys_create_box": (_p, [_i64, _p, _i, _p, _p, _d, _d, _i, _i, _u64, _u32, _i, _i, _i, _p, _p, _p, _p,
                                        _p, _p]),
            "orc_sys_create": (_p, [_i64, _d, _d, _d, _d, _i, _i, _u64, _u32, _i, _i, _i, _p, _p, _p, _p, _p, _p]),
            "orc_sys_destroy": (None, [_p]),
            "orc_sys_mmax": (_i, [_p]),
            "orc_sys_nshell": (_i, [_p]),
            "orc_sys_nlat": (_i64, [_p]),
            "orc_sys_tables": (None, [_p, _p, _p, _p]),
            "orc_sys_lattice": (None, [_p, _p, _p]),
            "orc_sys_draw": (None, [_p, _u64, _p, _p]),
            "orc_sys_force": (None, [_p, _u64, _p, _p, _p, _p]),
            "orc_sys_run": (_i, [_p, _p, _p, _p, _u64, _i, _d, _p]),
            "orc_num_threads": (_i, []),
            "orc_ssf": (None, [_i64, _p, _p, _d, _i, _p]),
            "orc_langevin_normals": (None, [_u64, _u64, _u64, _u32, _p]),
            "orc_sys_set_langevin": (None, [_p, _d, _d]),
            "orc_sys_set_sampler": (_i, [_p, _i]),
            "orc_sys_set_bath": (_i, [_p, _i, _d, _d]),
            "orc_sys_bath_state": (None, [_p, _p]),
            "orc_mh_draw": (None, [_i, _u64, _u64, _u32, _i, _p, _p, _p, _p, _p, _p, _p, _p]),
            "orc_rdf": (None, [_i64, _p, _d, _d, _i, _p, _p]),
            "orc_track": (None, [_i64, _d, _p, _p, _p]),
            "orc_track_box": (None, [_i64, _p, _p, _p, _p]),
            "orc_msd_vacf": (None, [_i64, _p, _p, _p, _p]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# SOG decomposition (Section 3, Algorithm 1)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class SOG:
    lam: float
    rc: float
    h: float
    t0: float
    w: float
    M1: int
    M2: int
    c: np.ndarray = None
    s: np.ndarray = None
    A: np.ndarray = None
    B: np.ndarray = None
    err: float = float("nan")
    sigma: float = 1.0    # bandwidth factor of the narrowest Gaussian (Appendix C; 1 for C1)
    smooth: int = 1
    ya: Optional[np.ndarray] = None   # the kernel's Yukawa terms, sum_j ya_j e^{-r/yl_j}/r
    yl: Optional[np.ndarray] = None   # (None: the Yukawa kernel at lam)
    nu: float = 0.0                   # EGS gradient-correction strength (0: Yukawa)

    @property
    def n(self) -> int:
        if self.c is not None:
            return len(self.c)
        return self.M1 + self.M2 + 1

    @property
    def terms(self):
        """(count, a, l) of the kernel sum_j a_j e^{-r/l_j}/r."""
        if self.yl is None:
            return 1, np.array([1.0]), np.array([float(self.lam)])
        a = np.ascontiguousarray(self.ya, dtype=np.float64)
        l = np.ascontiguousarray(self.yl, dtype=np.float64)
        return len(l), a, l

    @property
    def F0(self) -> float:
        return float(sum(self.c))

    @property
    def Fhat0(self) -> float:
        return float(sum(self.A))

    def expand(self) -> "SOG":
        n = self.M1 + self.M2 + 1
        self.c, self.s, self.A, self.B = (np.zeros(n) for _ in range(4))
        lib().orc_sog_expand_s(self.lam, self.h, self.t0, self.w, self.sigma, self.M1, self.M2, _ptr(self.c),
                               _ptr(self.s), _ptr(self.A), _ptr(self.B))
        return self

    def F(self, r) -> np.ndarray:
        r = np.asarray(r, dtype=np.float64)
        return np.array([lib().orc_F(self.n, _ptr(self.c), _ptr(self.s), float(x)) for x in r.ravel()]).reshape(r.shape)

    def Fhat(self, k2) -> np.ndarray:
        k2 = np.asarray(k2, dtype=np.float64)
        return np.array([lib().orc_Fhat(self.n, _ptr(self.A), _ptr(self.B), float(x)) for x in k2.ravel()]).reshape(k2.shape)

    def Fhat_slope(self, k2) -> np.ndarray:
        """-dFhat/d(k^2)."""
        k2 = np.asarray(k2, dtype=np.float64)
        return np.array([lib().orc_Fhat_slope(self.n, _ptr(self.A), _ptr(self.B), float(x))
                         for x in k2.ravel()]).reshape(k2.shape)


def h_star(eps: float, delta: float) -> float:
    return lib().orc_h_star(eps, delta)


def sog_c1(lam: float, rc: float, h: float, M1: int, M2: int) -> SOG:
    t0, w = C.c_double(), C.c_double()
    rc_ = lib().orc_sog_c1_root(lam, rc, h, M1, M2, C.byref(t0), C.byref(w))
    if rc_ != 0:
        raise ValueError("no C1 root with positive weight")
    return SOG(lam, rc, h, t0.value, w.value, M1, M2).expand()


def sog_auto(lam: float, rc: float, eps: float) -> SOG:
    M1, M2 = C.c_int(), C.c_int()
    h, t0, w, err = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    r = lib().orc_sog_auto(lam, rc, eps, C.byref(M1), C.byref(M2), C.byref(h), C.byref(t0), C.byref(w), C.byref(err))
    if r != 0:
        raise ValueError("no SOG found")
    s = SOG(lam, rc, h.value, t0.value, w.value, M1.value, M2.value).expand()
    s.err = err.value
    return s


def sog_c2(lam: float, rc: float, h: float, M1: int, M2: int) -> SOG:
    """The C2-continuous decomposition of Appendix C for given M1, M2."""
    t0, w, sg = C.c_double(), C.c_double(), C.c_double()
    if lib().orc_sog_c2_root(lam, rc, h, M1, M2, C.byref(t0), C.byref(w), C.byref(sg)) != 0:
        raise ValueError("no C2 root with positive weight and bandwidth")
    return SOG(lam, rc, h, t0.value, w.value, M1, M2, sigma=sg.value, smooth=2).expand()


def sog_auto2(lam: float, rc: float, eps: float) -> SOG:
    M1, M2 = C.c_int(), C.c_int()
    h, t0, w, sg, err = (C.c_double() for _ in range(5))
    r = lib().orc_sog_auto2(lam, rc, eps, C.byref(M1), C.byref(M2), C.byref(h), C.byref(t0), C.byref(w),
                            C.byref(sg), C.byref(err))
    if r != 0:
        raise ValueError("no C2 SOG found")
    s = SOG(lam, rc, h.value, t0.value, w.value, M1.value, M2.value, sigma=sg.value, smooth=2).expand()
    s.err = err.value
    return s


def egs_split(lam: float, nu: float):
    """(a, l): the EGS kernel of Section 1 as sum_j a_j e^{-r/l_j}/r."""
    a, l = np.zeros(2), np.zeros(2)
    if lib().orc_egs_split(lam, nu, _ptr(a), _ptr(l)) != 0:
        raise ValueError("EGS needs lambda > 0 and 0 < nu < 1")
    return a, l


def kernel_Y(s: SOG, r) -> np.ndarray:
    nY, ya, yl = s.terms
    r = np.asarray(r, dtype=np.float64)
    return np.array([lib().orc_kernel_Y(nY, _ptr(ya), _ptr(yl), float(x)) for x in r.ravel()]).reshape(r.shape)


def kernel_maxerr(s: SOG, R: float) -> float:
    nY, ya, yl = s.terms
    return lib().orc_kernel_maxerr(nY, _ptr(ya), _ptr(yl), s.rc, R, s.n, _ptr(s.c), _ptr(s.s))


EGS_RANGE = 33.0   # the approximation range [r_c, 33 l] of Algorithm 1, per Yukawa term


def sog_egs(lam: float, nu: float, rc: float, eps: float, smooth: int = 1) -> SOG:
    """The EGS kernel (Section 1) decomposed term by term: each Yukawa term
    a_j e^{-r/l_j}/r gets the decomposition of Algorithm 1 (smooth = 1) or of
    Appendix C (smooth = 2) at length l_j and tolerance eps / (|a_1| + |a_2|),
    and F is the sum of a_j times each term's Gaussians, so that |Y - F| <=
    eps on [r_c, 33 l_1] and N = Y - F inherits each term's continuity at r_c.
    A term with r_c >= 33 l_j has no Gaussians: it lies wholly in the near
    field, cut at r_c where it is below e^{-33}/r_c."""
    a, l = egs_split(lam, nu)
    eps_j = eps / float(np.abs(a).sum())
    cs, ss, As, Bs = [], [], [], []
    for aj, lj in zip(a, l):
        if rc >= EGS_RANGE * lj:
            continue
        t = sog_auto(lj, rc, eps_j) if smooth == 1 else sog_auto2(lj, rc, eps_j)
        cs.append(aj * t.c)
        ss.append(t.s)
        As.append(aj * t.A)
        Bs.append(t.B)
    out = SOG(lam, rc, float("nan"), float("nan"), float("nan"), 0, 0, smooth=smooth, ya=a, yl=l, nu=nu)
    out.c, out.s, out.A, out.B = (np.ascontiguousarray(np.concatenate(v)) for v in (cs, ss, As, Bs))
    out.err = kernel_maxerr(out, EGS_RANGE * float(l[0]))
    return out


def sog_far2(s: SOG, r) -> float:
    return lib().orc_sog_far2(s.lam, s.h, s.t0, s.w, s.sigma, s.M1, s.M2, r)


def sog_w(lam, rc, h, t0, M1, M2) -> float:
    return lib().orc_sog_w(lam, rc, h, t0, M1, M2)


def sog_far(lam, h, t0, w, M1, M2, r) -> float:
    return lib().orc_sog_far(lam, h, t0, w, M1, M2, r)


def sog_c1_residual(lam, rc, h, t0, M1, M2) -> float:
    return lib().orc_sog_c1_residual(lam, rc, h, t0, M1, M2)


def sog_maxerr(s: SOG) -> float:
    return lib().orc_sog_maxerr(s.lam, s.rc, s.h, s.t0, s.w, s.M1, s.M2)


# ---------------------------------------------------------------------------
# Random numbers, lattice, sampling tables (Section 4.3)
# ---------------------------------------------------------------------------

def philox(counter, key) -> np.ndarray:
    ctr = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_ptr(ctr), _ptr(k), _ptr(out))
    return out


def lattice(mmax: int):
    cnt = lib().orc_lattice_count(mmax)
    n3 = np.zeros((cnt, 3), dtype=np.int32)
    start = np.zeros(mmax + 2, dtype=np.int64)
    lib().orc_lattice_build(mmax, _ptr(n3), _ptr(start))
    return n3, start


def mmax_default(s: SOG, L: float) -> int:
    return lib().orc_mmax_default(s.n, _ptr(s.A), _ptr(s.B), L)


def density(kind: int, kT: float, V: float, Q2: float, lam: float, k2: float) -> float:
    return lib().orc_density(kind, kT, V, Q2, lam, k2)


# ---------------------------------------------------------------------------
# Cells, near field, far field
# ---------------------------------------------------------------------------

def cells(x: np.ndarray, L: float, rc: float):
    x = _f64(x)
    N = x.shape[1]
    nc = int(math.floor(L / rc))
    cs = np.zeros(nc ** 3 + 1, dtype=np.int32)
    order = np.zeros(N, dtype=np.int32)
    lib().orc_cells(N, _ptr(x), L, rc, _ptr(cs), _ptr(order))
    return cs, order


def box(L) -> np.ndarray:
    """Edges (L_x, L_y, L_z) of a box given as one edge or three."""
    b = np.ascontiguousarray(np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)))
    return b.copy()


def is_cube(L) -> bool:
    b = box(L)
    return bool(b[0] == b[1] == b[2])


def cells_box(x: np.ndarray, L, rc: float):
    """The cell list of a box of edges L (three values): (cell_start, order, nc[3])."""
    x = _f64(x)
    N = x.shape[1]
    Lb = box(L)
    nc = np.floor(Lb / rc).astype(np.int64)
    cs = np.zeros(int(nc.prod()) + 1, dtype=np.int32)
    order = np.zeros(N, dtype=np.int32)
    nco = np.zeros(3, dtype=np.int32)
    lib().orc_cells_box(N, _ptr(x), _ptr(Lb), rc, _ptr(cs), _ptr(order), _ptr(nco))
    return cs, order, nco


def near(x, q, L, s: SOG, virial: bool = False):
    """Near-field forces [3, N] and energy U_N; with virial, also W_N.  L: one
    edge or the three edges of a cuboid."""
    x, q = _f64(x), _f64(q)
    N = x.shape[1]
    f = np.zeros((3, N))
    U, W = C.c_double(), C.c_double()
    nY, ya, yl = s.terms
    if np.ndim(L) == 0:
        r = lib().orc_near_k(N, _ptr(x), _ptr(q), L, nY, _ptr(ya), _ptr(yl), s.rc, s.n, _ptr(s.c), _ptr(s.s),
                             _ptr(f), C.byref(U), C.byref(W))
    else:
        Lb = box(L)
        r = lib().orc_near_box(N, _ptr(x), _ptr(q), _ptr(Lb), nY, _ptr(ya), _ptr(yl), s.rc, s.n, _ptr(s.c),
                               _ptr(s.s), _ptr(f), C.byref(U), C.byref(W))
    if r != 0:
        raise ValueError("near: bad kernel")
    return (f, U.value, W.value) if virial else (f, U.value)


def near_subset(x, q, L, s: SOG, idx):
    """Near-field forces [3, len(idx)] on the particles idx."""
    x, q = _f64(x), _f64(q)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    f = np.zeros((3, len(idx)))
    nY, ya, yl = s.terms
    if np.ndim(L) == 0:
        rc = lib().orc_near_subset_k(x.shape[1], _ptr(x), _ptr(q), L, nY, _ptr(ya), _ptr(yl), s.rc, s.n,
                                     _ptr(s.c), _ptr(s.s), len(idx), _ptr(idx), _ptr(f))
    else:
        Lb = box(L)
        rc = lib().orc_near_subset_box(x.shape[1], _ptr(x), _ptr(q), _ptr(Lb), nY, _ptr(ya), _ptr(yl), s.rc, s.n,
                                       _ptr(s.c), _ptr(s.s), len(idx), _ptr(idx), _ptr(f))
    if rc != 0:
        raise ValueError("near_subset: particle index out of range or bad kernel")
    return f


def rho(x, q, L, n3) -> np.ndarray:
    x, q = _f64(x), _f64(q)
    n3 = np.ascontiguousarray(n3, dtype=np.int32)
    P = n3.shape[0]
    out = np.zeros((P, 2))
    if np.ndim(L) == 0:
        lib().orc_rho(x.shape[1], _ptr(x), _ptr(q), L, P, _ptr(n3), _ptr(out))
    else:
        lib().orc_rho_box(x.shape[1], _ptr(x), _ptr(q), _ptr(box(L)), P, _ptr(n3), _ptr(out))
    return out


def far_rb(x, q, L, n3, coef, rho_):
    x, q = _f64(x), _f64(q)
    n3 = np.ascontiguousarray(n3, dtype=np.int32)
    coef, rho_ = _f64(coef), _f64(rho_)
    f = np.zeros_like(x)
    if np.ndim(L) == 0:
        lib().orc_far_rb(x.shape[1], _ptr(x), _ptr(q), L, n3.shape[0], _ptr(n3), _ptr(coef), _ptr(rho_), _ptr(f))
    else:
        lib().orc_far_rb_box(x.shape[1], _ptr(x), _ptr(q), _ptr(box(L)), n3.shape[0], _ptr(n3), _ptr(coef),
                             _ptr(rho_), _ptr(f))
    return f


def far_full(x, q, L, s: SOG, mmax: int, virial: bool = False):
    """Full-lattice far forces [3, N] and energy U_F; with virial, also W_F."""
    x, q = _f64(x), _f64(q)
    f = np.zeros_like(x)
    W = C.c_double()
    U = lib().orc_far_full(x.shape[1], _ptr(x), _ptr(q), L, s.n, _ptr(s.A), _ptr(s.B), mmax, _ptr(f),
                           C.byref(W))
    return (f, U, W.value) if virial else (f, U)


def far_rb_virial(n3, coef, rho_, L, s: SOG) -> float:
    """The random-batch estimator of the far-field virial for the modes n3."""
    n3 = np.ascontiguousarray(n3, dtype=np.int32)
    coef, rho_ = _f64(coef), _f64(rho_)
    if np.ndim(L) == 0:
        return lib().orc_far_rb_virial(n3.shape[0], _ptr(n3), _ptr(coef), _ptr(rho_), L, s.n, _ptr(s.A), _ptr(s.B))
    return lib().orc_far_rb_virial_box(n3.shape[0], _ptr(n3), _ptr(coef), _ptr(rho_), _ptr(box(L)), s.n,
                                       _ptr(s.A), _ptr(s.B))


def box_lattice(L, s: SOG):
    """(n3 [count, 3], k2 [count]): the Fourier lattice of a box, sorted by k^2."""
    Lb = box(L)
    cnt = lib().orc_box_lattice(_ptr(Lb), s.n, _ptr(s.A), _ptr(s.B), None, None)
    if cnt < 0:
        raise ValueError("lattice beyond |n_d| = 511")
    n3 = np.zeros((cnt, 3), dtype=np.int32)
    k2 = np.zeros(cnt)
    lib().orc_box_lattice(_ptr(Lb), s.n, _ptr(s.A), _ptr(s.B), _ptr(n3), _ptr(k2))
    return n3, k2


def far_full_box(x, q, L, s: SOG, virial: bool = False):
    """Full-lattice far forces and energy of a box over box_lattice's modes."""
    x, q = _f64(x), _f64(q)
    f = np.zeros_like(x)
    W = C.c_double()
    U = lib().orc_far_full_box(x.shape[1], _ptr(x), _ptr(q), _ptr(box(L)), s.n, _ptr(s.A), _ptr(s.B), _ptr(f),
                               C.byref(W))
    return (f, U, W.value) if virial else (f, U)


# ---------------------------------------------------------------------------
# A whole system (Algorithm 2)
# ---------------------------------------------------------------------------

class System:
    """Sampling tables plus force evaluation and velocity-Verlet stepping."""

    def __init__(self, q, m, L: float, s: SOG, kT: float, P: int, seed: int, replica: int = 0, mmax: int = 0,
                 density: int = ADAPTIVE, full_k: bool = False, sampler: int = 0):
        self.q = _f64(q)
        self.m = _f64(m)
        self.N = self.q.shape[0]
        self.L, self.sog, self.kT, self.P = L, s, kT, P
        self.V = float(np.prod(box(L)))
        nY, self._ya, self._yl = s.terms
        if np.ndim(L) == 0:
            self._h = lib().orc_sys_create_k(self.N, L, nY, _ptr(self._ya), _ptr(self._yl), s.rc, kT, P, mmax, seed,
                                             replica, density, int(full_k), s.n, _ptr(s.c), _ptr(s.s), _ptr(s.A),
                                             _ptr(s.B), _ptr(self.q), _ptr(self.m))
        else:
            self._Lb = box(L)
            self._h = lib().orc_sys_create_box(self.N, _ptr(self._Lb), nY, _ptr(self._ya), _ptr(self._yl), s.rc, kT,
                                               P, mmax, seed, replica, density, int(full_k), s.n, _ptr(s.c),
                                               _ptr(s.s), _ptr(s.A), _ptr(s.B), _ptr(self.q), _ptr(self.m))
        if not self._h:
            raise ValueError("oracle system creation failed")
        self.mmax = lib().orc_sys_mmax(self._h)
        self.nshell = lib().orc_sys_nshell(self._h)
        if sampler:
            self.set_sampler(sampler)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_sys_destroy(h)
            self._h = None

    def tables(self):
        ns = self.nshell
        m = np.zeros(ns, dtype=np.int32)
        cdf = np.zeros(ns)
        coef = np.zeros(ns)
        lib().orc_sys_tables(self._h, _ptr(m), _ptr(cdf), _ptr(coef))
        return m, cdf, coef

    def lattice(self):
        cnt = lib().orc_sys_nlat(self._h)
        n3 = np.zeros((cnt, 3), dtype=np.int32)
        start = np.zeros(self.mmax + 2, dtype=np.int64)
        lib().orc_sys_lattice(self._h, _ptr(n3), _ptr(start))
        return n3, start

    def draw(self, step: int):
        n = np.zeros((self.P, 3), dtype=np.int32)
        coef = np.zeros(self.P)
        lib().orc_sys_draw(self._h, step, _ptr(n), _ptr(coef))
        return n, coef

    def force(self, x, step: int):
        """Returns (f, f_near, energy[8]): U_N, U_F, U_k0, U_self, U_bg, 0, W_N, W_F."""
        x = _f64(x)
        f = np.zeros_like(x)
        fn = np.zeros_like(x)
        e = np.zeros(8)
        lib().orc_sys_force(self._h, step, _ptr(x), _ptr(f), _ptr(fn), _ptr(e))
        return f, fn, e

    def set_sampler(self, sampler: int):
        """0: i.i.d. inverse-CDF draws; 1: the Metropolis-Hastings chain (emptied)."""
        if lib().orc_sys_set_sampler(self._h, sampler) != 0:
            raise ValueError("sampler must be 0 or 1")

    def set_bath(self, kind: int, rate: float, bath_kT: float):
        """Global bath for run(): 2 Nose-Hoover, 3 Berendsen (rate = 1/tau), 0 off."""
        if lib().orc_sys_set_bath(self._h, kind, rate, bath_kT) != 0:
            raise ValueError("bad bath")

    def bath_state(self):
        """(xi, eta) of the Nose-Hoover bath."""
        out = np.zeros(2)
        lib().orc_sys_bath_state(self._h, _ptr(out))
        return float(out[0]), float(out[1])

    def set_langevin(self, friction: float, bath_kT: float):
        """Langevin thermostat for run() (friction 0: plain velocity-Verlet)."""
        lib().orc_sys_set_langevin(self._h, friction, bath_kT)

    def run(self, x, v, f, step0: int, nsteps: int, dt: float):
        """Advances (x, v, f) in place; returns the [nsteps, 8] energy history (KE in column 5)."""
        eh = np.zeros((nsteps, 8))
        r = lib().orc_sys_run(self._h, _ptr(x), _ptr(v), _ptr(f), step0, nsteps, dt, _ptr(eh))
        if r != 0:
            raise RuntimeError("a particle moved a full box length in one step")
        return eh


def langevin_normals(i: int, step: int, seed: int, replica: int = 0) -> np.ndarray:
    z = np.zeros(3)
    lib().orc_langevin_normals(i, step, seed, replica, _ptr(z))
    return z


def ssf(x, w, L: float, mmax: int) -> np.ndarray:
    """Shell means of |sum_j w_j exp(i k.r_j)|^2 for |n|^2 = 0..mmax (0 where a
    shell is empty); S(k) = ssf / N with unit weights."""
    x, w = _f64(x), _f64(w)
    out = np.zeros(mmax + 1)
    lib().orc_ssf(x.shape[1], _ptr(x), _ptr(w), L, mmax, _ptr(out))
    return out


def rdf(x, L, r_max: float, nbins: int):
    """(counts, ambiguous) of ordered pairs by minimum-image distance bin (L one
    edge or a cuboid's three)."""
    x = _f64(x)
    counts = np.zeros(nbins, dtype=np.int64)
    amb = np.zeros(nbins, dtype=np.int64)
    if np.ndim(L) == 0:
        lib().orc_rdf(x.shape[1], _ptr(x), L, r_max, nbins, _ptr(counts), _ptr(amb))
    else:
        lib().orc_rdf_box(x.shape[1], _ptr(x), _ptr(box(L)), r_max, nbins, _ptr(counts), _ptr(amb))
    return counts, amb


def track(x, L, x_last, disp) -> None:
    """disp += minimum-image (x - x_last); x_last = x (in place); L one edge
    or the three edges of a cuboid."""
    x = _f64(x)
    assert x_last.flags.c_contiguous and disp.flags.c_contiguous
    if is_cube(L):
        lib().orc_track(x.shape[1], box(L)[0], _ptr(x), _ptr(x_last), _ptr(disp))
    else:
        lib().orc_track_box(x.shape[1], _ptr(box(L)), _ptr(x), _ptr(x_last), _ptr(disp))


def msd_vacf(disp, v0, v):
    out = np.zeros(2)
    disp, v0, v = _f64(disp), _f64(v0), _f64(v)
    lib().orc_msd_vacf(disp.shape[1], _ptr(disp), _ptr(v0), _ptr(v), _ptr(out))
    return float(out[0]), float(out[1])


def num_threads() -> int:
    return lib().orc_num_threads()


# ---------------------------------------------------------------------------
# Plain definitions used as pins
# ---------------------------------------------------------------------------

def yukawa_image_sum(x, q, L, lam, r_max: float):
    """Energy and forces of the periodic Yukawa system by direct summation over
    every image with |r_ij + n L| < r_max (the plain definition the method
    approximates; Section 2; L one edge or the three of a cuboid).  Pure
    numpy, for a handful of particles."""
    x = _f64(x)
    q = _f64(q)
    N = x.shape[1]
    Lb = box(L)
    ax = [np.arange(-(int(math.ceil(r_max / Lb[d])) + 1), int(math.ceil(r_max / Lb[d])) + 2) for d in range(3)]
    sh = np.stack(np.meshgrid(*ax, indexing="ij"), -1).reshape(-1, 3) * Lb[None, :]
    U = 0.0
    f = np.zeros((3, N))
    pos = x.T
    for i in range(N):
        d = pos[i][None, None, :] - pos[:, None, :] - sh[None, :, :]   # (N, nsh, 3), d = r_i - r_j - nL
        r = np.sqrt((d * d).sum(-1))
        mask = (r < r_max) & (r > 0)
        rr = np.where(mask, r, 1.0)
        y = np.where(mask, np.exp(-rr / lam) / rr, 0.0)
        U += 0.5 * q[i] * float((q[:, None] * y).sum())
        fac = np.where(mask, np.exp(-rr / lam) * (1.0 + rr / lam) / rr ** 3, 0.0)
        f[:, i] = q[i] * ((q[:, None, None] * fac[:, :, None] * d).sum(axis=(0, 1)))
    return U, f
