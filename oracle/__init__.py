"""FP64 CPU oracle for the sliding-window vector filters.

TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import, call or execute anything in this package. It
shares no code with the GPU library: its filters are plain C (oracle.c, built
with gcc, FP64, no fused multiply-add, no fast-math), its Remez exchange is
numpy (remez.py), and its brute-force twin is numpy (twin.py).

Approximants are described to the C code by small structs. Coefficients the
GPU evaluates in FP32 are rounded here to the nearest FP32 value before use, so
the oracle's "same approximant" mode evaluates exactly the polynomial the GPU
evaluates, in FP64.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from . import paper_tables as PT
from .remez import rational, remez

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

MAXC = 16
FILTERS = {"vdf": 0, "ddf": 1, "amnfe": 2, "evmf": 3, "amnfg": 4}


class _Acos(C.Structure):
    _fields_ = [("kind", C.c_int), ("n_lo", C.c_int), ("n_hi", C.c_int),
                ("lo", C.c_double * MAXC), ("hi", C.c_double * MAXC)]


class _Exp(C.Structure):
    _fields_ = [("kind", C.c_int), ("n", C.c_int), ("c", C.c_double * MAXC),
                ("cutoff", C.c_double), ("n_q", C.c_int), ("q", C.c_double * MAXC)]


class _Ent(C.Structure):
    _fields_ = [("kind", C.c_int), ("n_p", C.c_int), ("n_q", C.c_int),
                ("p", C.c_double * MAXC), ("q", C.c_double * MAXC), ("cutoff", C.c_double)]


class _Cfg(C.Structure):
    _fields_ = [("filter", C.c_int), ("window", C.c_int), ("param", C.c_double),
                ("acos_ap", _Acos), ("exp_ap", _Exp), ("ent_ap", _Ent)]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-std=c11", "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB_PATH)
        L.orc_filter.restype = C.c_int
        L.orc_filter.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int64, C.c_void_p,
                                 C.c_int64, C.POINTER(_Cfg), C.c_void_p, C.c_void_p, C.c_int64,
                                 C.c_int]
        L.orc_inspect.restype = C.c_int
        L.orc_inspect.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int64,
                                  C.POINTER(_Cfg), C.c_int, C.c_int, C.POINTER(C.c_double)]
        L.orc_eval_angle.restype = C.c_double
        L.orc_eval_angle.argtypes = [C.POINTER(_Acos), C.c_double]
        L.orc_eval_expneg.restype = C.c_double
        L.orc_eval_expneg.argtypes = [C.POINTER(_Exp), C.c_double]
        L.orc_eval_ent.restype = C.c_double
        L.orc_eval_ent.argtypes = [C.POINTER(_Ent), C.c_double]
        L.orc_cosine.restype = C.c_double
        L.orc_cosine.argtypes = [C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.orc_max_threads.restype = C.c_int
        _lib = L
    return _lib


def f32(c: Sequence[float]) -> np.ndarray:
    """Round each coefficient to the nearest FP32 value (kept as float64)."""
    return np.asarray(c, dtype=np.float64).astype(np.float32).astype(np.float64)


# ---------------------------------------------------------------- approximants

@dataclass
class AngleApprox:
    """How A(x_i, x_j) = acos(z) is evaluated.

    kind 'exact'  : acos(z)
    kind 'paper2' : Table 1 two-piece form, full-basis degree-d pieces
    kind 'split'  : odd split over [-1, 1] (degree d odd)
    kind 'chord'  : one odd polynomial in the chord s = sqrt(2(1 - z)) over
                    z in [0, 1] (mirrored through acos(-z) = pi - acos(z))
    """
    kind: str = "exact"
    degree: int = 0
    lo: Optional[np.ndarray] = None
    hi: Optional[np.ndarray] = None
    eps: float = 0.0

    def struct(self) -> _Acos:
        s = _Acos()
        s.kind = {"exact": 0, "paper2": 1, "split": 2, "chord": 3}[self.kind]
        if self.kind != "exact":
            s.n_lo, s.n_hi = len(self.lo), len(self.hi)
            for i, v in enumerate(self.lo):
                s.lo[i] = float(v)
            for i, v in enumerate(self.hi):
                s.hi[i] = float(v)
        return s


def angle_approx(kind: str = "exact", degree: int = 0, source: str = "remez",
                 round_f32: bool = True, precision: str = "fp32") -> AngleApprox:
    """Build an angle approximant.

    paper2 + source 'paper' -> Table 1 coefficients (degree 4);
    paper2 + source 'remez' -> this oracle's Remez on the Table 1 intervals;
    split                   -> odd asin fit on [-1/2, 1/2] (middle piece) and odd
                               chord fit 2 asin(s/2) on [-1, 1] (outer pieces).
    chord + precision 'fp16x2' -> the chord fit with every coefficient after the
                               first rounded (to nearest even) to IEEE half
                               precision: the polynomial a packed-FP16 evaluation
                               of the correction term uses.
    """
    if precision == "fp16x2":
        if kind != "chord":
            raise ValueError("fp16x2 is defined for the chord approximant")
        a = angle_approx("chord", degree, source, round_f32)
        hi = a.hi.copy()
        hi[1:] = hi[1:].astype(np.float32).astype(np.float16).astype(np.float64)
        return AngleApprox("chord", degree, a.lo, hi, a.eps)
    rnd = f32 if round_f32 else (lambda c: np.asarray(c, dtype=np.float64))
    if kind == "exact":
        return AngleApprox("exact")
    if kind == "paper2":
        if source == "paper":
            return AngleApprox("paper2", 4, rnd(PT.TABLE1_ARCCOS), rnd(PT.TABLE1_ARCSIN),
                               max(PT.TABLE1_ARCCOS_EPS, PT.TABLE1_ARCSIN_EPS))
        lo, e_lo, _ = remez("acos", 0.0, 0.5, degree)
        hi, e_hi, _ = remez("asin2_tau", 0.0, 1.0 / math.sqrt(2.0), degree)
        return AngleApprox("paper2", degree, rnd(lo), rnd(hi), max(e_lo, e_hi))
    if kind == "split":
        lo, e_lo, _ = remez("asin", -0.5, 0.5, degree, odd=True)
        hi, e_hi, _ = remez("chord", -1.0, 1.0, degree, odd=True)
        return AngleApprox("split", degree, rnd(lo), rnd(hi), max(e_lo, e_hi))
    if kind == "chord":
        hi, e_hi, _ = remez("chord", -math.sqrt(2.0), math.sqrt(2.0), degree, odd=True)
        return AngleApprox("chord", degree, np.zeros(0), rnd(hi), e_hi)
    raise ValueError(kind)


@dataclass
class ExpApprox:
    kind: str = "exact"            # 'exact' | 'poly' | 'rational'
    coeffs: Optional[np.ndarray] = None
    cutoff: float = PT.EXP_CUTOFF
    eps: float = 0.0
    q: Optional[np.ndarray] = None  # denominator of the rational form

    def struct(self) -> _Exp:
        s = _Exp()
        s.kind = {"exact": 0, "poly": 1, "rational": 2}[self.kind]
        s.cutoff = self.cutoff
        if self.kind != "exact":
            s.n = len(self.coeffs)
            for i, v in enumerate(self.coeffs):
                s.c[i] = float(v)
        if self.kind == "rational":
            s.n_q = len(self.q)
            for i, v in enumerate(self.q):
                s.q[i] = float(v)
        return s


def amnfe_range(window: int, kappa: float = PT.KAPPA) -> float:
    """Upper end of the kernel argument: z_i <= n^(kappa/3) (derived from the
    AMNF equation: sum_j |x_i - x_j|_1 >= |x_i - x_C|_1)."""
    return float((window * window) ** (kappa / 3.0))


def amnfg_range(window: int, kappa: float = PT.KAPPA) -> float:
    """Upper end of the Gaussian kernel's EXP argument z_i = 0.5 |x|_2^2,
    x = (x_C - x_i) / h_i: z_i <= 0.5 n^(2 kappa/3) (|x_C - x_i|_2 <=
    |x_C - x_i|_1 <= sum_j |x_i - x_j|_1 = n^(kappa/3) h_i)."""
    return 0.5 * float((window * window) ** (2.0 * kappa / 3.0))


def exp_fit_range(window: int, kappa: float = PT.KAPPA, kernel: str = "exp") -> float:
    """Interval [0, b] of the minimax exp fit: up to the argument bound of the
    kernel, and no further than the cutoff T (K is 0 above T, Section 3.2)."""
    b = amnfe_range(window, kappa) if kernel == "exp" else amnfg_range(window, kappa)
    return min(b, PT.EXP_CUTOFF)


def f16_tail(c: np.ndarray) -> np.ndarray:
    """c_1, c_2, ... rounded (to nearest even) to IEEE half precision, c_0
    kept: the polynomial whose correction sum_{k>=1} c_k x^k a packed-FP16
    evaluation forms (c_0 is added in FP32)."""
    c = np.asarray(c, dtype=np.float64).copy()
    c[1:] = c[1:].astype(np.float32).astype(np.float16).astype(np.float64)
    return c


def exp_approx(kind: str = "exact", degree: int = 0, source: str = "remez", window: int = 5,
               kappa: float = PT.KAPPA, round_f32: bool = True, precision: str = "fp32",
               kernel: str = "exp") -> ExpApprox:
    """exp(-z) for AMNFE (kernel 'exp') and AMNFG (kernel 'gauss'): exact, a
    Table 2 polynomial (source 'paper'), the Table 3 rational R^4_4 (kind
    'rational'), this oracle's best rational R^d_d (kind 'ratfit') or its
    minimax polynomial (kind 'poly') on [0, min(b, T)] with b the
    kernel's argument bound (exp_fit_range); precision 'fp16x2' (minimax only)
    rounds the fit's c_1.. to FP16 (see f16_tail). All forms give 0 above the
    Section 3.2 cutoff T."""
    if precision == "fp16x2":
        if kind != "poly" or source != "remez":
            raise ValueError("fp16x2 is defined for the minimax exp fit")
        a = exp_approx(kind, degree, source, window, kappa, round_f32, kernel=kernel)
        return ExpApprox("poly", f16_tail(a.coeffs), a.cutoff, a.eps)
    rnd = f32 if round_f32 else (lambda c: np.asarray(c, dtype=np.float64))
    if kind == "exact":
        return ExpApprox("exact")
    if kind == "rational":
        return ExpApprox("rational", rnd(PT.TABLE3_NUM), PT.EXP_CUTOFF, PT.TABLE3_EPS,
                         rnd(PT.TABLE3_DEN))
    if kind == "ratfit":
        # this oracle's best R^d_d (Section 2, rational class) on the range the
        # kernel's argument reaches, as the Table 3 form p(z) / q(z)
        p, q, eps, _ = rational("expneg", 0.0, exp_fit_range(window, kappa, kernel), degree, degree)
        return ExpApprox("rational", rnd(p), PT.EXP_CUTOFF, eps, rnd(q))
    if source == "paper":
        c, eps = PT.TABLE2[degree]
        return ExpApprox("poly", rnd(c), PT.EXP_CUTOFF, eps)
    c, eps, _ = remez("expneg", 0.0, exp_fit_range(window, kappa, kernel), degree)
    return ExpApprox("poly", rnd(c), PT.EXP_CUTOFF, eps)


@dataclass
class EntApprox:
    kind: str = "exact"            # 'exact' | 'rational' | 'rangered'
    p: Optional[np.ndarray] = None
    q: Optional[np.ndarray] = None
    cutoff: float = 0.0
    eps: float = 0.0

    def struct(self) -> _Ent:
        s = _Ent()
        s.kind = {"exact": 0, "rational": 1, "rangered": 2}[self.kind]
        s.cutoff = self.cutoff
        if self.p is not None:
            s.n_p = len(self.p)
            for i, v in enumerate(self.p):
                s.p[i] = float(v)
        if self.q is not None:
            s.n_q = len(self.q)
            for i, v in enumerate(self.q):
                s.q[i] = float(v)
        return s


def ent_approx(kind: str = "exact", degree: int = 0, round_f32: bool = True,
               precision: str = "fp32", cutoff: Optional[float] = None) -> EntApprox:
    """ENT(P) = P ln P for EVMF: exact, the Table 4 rational, or range
    reduction P = m 2^e with a minimax fit of ln(1 + t) on [0, 1]; precision
    'fp16x2' (range-reduced only) rounds that fit's c_1.. to FP16. cutoff: the
    T of Section 3.3 (ENT = 0 below it, every kind); None: the paper's 0.05
    for its rational (fitted on [0.05, 1]), no cutoff otherwise."""
    if cutoff is None:
        cutoff = PT.ENT_CUTOFF if kind == "rational" else 0.0
    if precision == "fp16x2":
        if kind != "rangered":
            raise ValueError("fp16x2 is defined for the range-reduced ln fit")
        a = ent_approx(kind, degree, round_f32)
        return EntApprox("rangered", f16_tail(a.p), None, cutoff, a.eps)
    rnd = f32 if round_f32 else (lambda c: np.asarray(c, dtype=np.float64))
    if kind == "exact":
        return EntApprox("exact", cutoff=cutoff)
    if kind == "rational":
        return EntApprox("rational", rnd(PT.TABLE4_NUM), rnd(PT.TABLE4_DEN), cutoff, PT.TABLE4_EPS)
    if kind == "rangered":
        c, eps, _ = remez("ln1p", 0.0, 1.0, degree)
        return EntApprox("rangered", rnd(c), None, cutoff, eps)
    raise ValueError(kind)


# ---------------------------------------------------------------- filters

def _cfg(filter: str, window: int, param: float, angle: Optional[AngleApprox],
         expap: Optional[ExpApprox], ent: Optional[EntApprox]) -> _Cfg:
    c = _Cfg()
    c.filter = FILTERS[filter]
    c.window = window
    c.param = param
    c.acos_ap = (angle or AngleApprox()).struct()
    c.exp_ap = (expap or ExpApprox()).struct()
    c.ent_ap = (ent or EntApprox()).struct()
    return c


def default_param(filter: str) -> float:
    return {"vdf": 0.0, "ddf": 0.5, "amnfe": PT.KAPPA, "evmf": 0.0, "amnfg": PT.KAPPA}[filter]


def run_filter(img: np.ndarray, filter: str, window: int = 3, param: Optional[float] = None,
               angle: Optional[AngleApprox] = None, expap: Optional[ExpApprox] = None,
               ent: Optional[EntApprox] = None, pixels: Optional[np.ndarray] = None,
               nthreads: int = 0) -> np.ndarray:
    """Filter an H x W x 3 uint8/uint16 image. With pixels (K x 2 array of
    (y, x)) only those outputs are computed and a K x 3 array is returned."""
    img = np.ascontiguousarray(img)
    assert img.ndim == 3 and img.shape[2] == 3 and img.dtype in (np.uint8, np.uint16)
    if window not in (3, 5, 7):
        raise ValueError("window must be 3, 5 or 7")
    H, W, _ = img.shape
    cfg = _cfg(filter, window, default_param(filter) if param is None else param, angle, expap, ent)
    bpc = img.itemsize
    L = lib()
    out = np.zeros_like(img)
    if pixels is None:
        L.orc_filter(img.ctypes.data, H, W, bpc, W * 3, out.ctypes.data, W * 3, C.byref(cfg),
                     None, None, 0, nthreads)
        return out
    pix = np.ascontiguousarray(pixels, dtype=np.int32)
    ys = np.ascontiguousarray(pix[:, 0])
    xs = np.ascontiguousarray(pix[:, 1])
    L.orc_filter(img.ctypes.data, H, W, bpc, W * 3, out.ctypes.data, W * 3, C.byref(cfg),
                 ys.ctypes.data, xs.ctypes.data, len(pix), nthreads)
    return out[ys, xs]


def inspect(img: np.ndarray, filter: str, y: int, x: int, window: int = 3,
            param: Optional[float] = None, angle: Optional[AngleApprox] = None,
            expap: Optional[ExpApprox] = None, ent: Optional[EntApprox] = None):
    """(return value, internal quantities) of one window; see orc_inspect in oracle.c."""
    img = np.ascontiguousarray(img)
    H, W, _ = img.shape
    cfg = _cfg(filter, window, default_param(filter) if param is None else param, angle, expap, ent)
    buf = (C.c_double * (4 * 49 + 8))()
    rv = lib().orc_inspect(img.ctypes.data, H, W, img.itemsize, W * 3, C.byref(cfg), y, x, buf)
    return rv, np.frombuffer(buf, dtype=np.float64).copy()


def eval_angle(ap: AngleApprox, z: float) -> float:
    s = ap.struct()
    return lib().orc_eval_angle(C.byref(s), float(z))


def eval_expneg(ep: ExpApprox, z: float) -> float:
    s = ep.struct()
    return lib().orc_eval_expneg(C.byref(s), float(z))


def eval_ent(en: EntApprox, z: float) -> float:
    s = en.struct()
    return lib().orc_eval_ent(C.byref(s), float(z))


def cosine(a, b) -> float:
    A = (C.c_int64 * 3)(*[int(v) for v in a])
    B = (C.c_int64 * 3)(*[int(v) for v in b])
    return lib().orc_cosine(A, B)


def max_threads() -> int:
    return lib().orc_max_threads()


# ---------------------------------------------------------------- window level

def _win_arg(v):
    v = np.ascontiguousarray(np.asarray(v, dtype=np.int64).reshape(-1, 3))
    return v, v.shape[0]


def window_vdf(v, angle: Optional[AngleApprox] = None):
    """(selected index, angle sums) of one window given as an (n, 3) array."""
    v, n = _win_arg(v)
    L = lib()
    S = np.zeros(n)
    ap = (angle or AngleApprox()).struct()
    L.orc_window_vdf.restype = C.c_int
    idx = L.orc_window_vdf(C.c_void_p(v.ctypes.data), n, C.byref(ap), C.c_void_p(S.ctypes.data))
    return idx, S


def window_ddf(v, p: float = 0.5, angle: Optional[AngleApprox] = None):
    v, n = _win_arg(v)
    L = lib()
    SA, SD, Psi = np.zeros(n), np.zeros(n), np.zeros(n)
    ap = (angle or AngleApprox()).struct()
    L.orc_window_ddf.restype = C.c_int
    idx = L.orc_window_ddf(C.c_void_p(v.ctypes.data), n, C.c_double(p), C.byref(ap),
                           C.c_void_p(SA.ctypes.data), C.c_void_p(SD.ctypes.data),
                           C.c_void_p(Psi.ctypes.data))
    return idx, SA, SD, Psi


def window_amnfe(v, kappa: float = PT.KAPPA, expap: Optional[ExpApprox] = None):
    """(uniform flag, unrounded weighted mean) of one window."""
    v, n = _win_arg(v)
    L = lib()
    mean = np.zeros(3)
    ep = (expap or ExpApprox()).struct()
    L.orc_window_amnfe.restype = C.c_int
    u = L.orc_window_amnfe(C.c_void_p(v.ctypes.data), n, C.c_double(kappa), C.byref(ep),
                           C.c_void_p(mean.ctypes.data))
    return u, mean


def window_amnfg(v, kappa: float = PT.KAPPA, expap: Optional[ExpApprox] = None):
    """(uniform flag, unrounded weighted mean) of one window, Gaussian kernel."""
    v, n = _win_arg(v)
    L = lib()
    mean = np.zeros(3)
    ep = (expap or ExpApprox()).struct()
    L.orc_window_amnfg.restype = C.c_int
    u = L.orc_window_amnfg(C.c_void_p(v.ctypes.data), n, C.c_double(kappa), C.byref(ep),
                           C.c_void_p(mean.ctypes.data))
    return u, mean


def window_evmf(v, ent: Optional[EntApprox] = None):
    """(selected index, (P_C, H, ENT(P_C), switched), vector-median sums)."""
    v, n = _win_arg(v)
    L = lib()
    info = np.zeros(4)
    S = np.zeros(n)
    en = (ent or EntApprox()).struct()
    L.orc_window_evmf.restype = C.c_int
    idx = L.orc_window_evmf(C.c_void_p(v.ctypes.data), n, C.byref(en),
                            C.c_void_p(info.ctypes.data), C.c_void_p(S.ctypes.data))
    return idx, info, S
