"""Python binding of libvf.so (argument marshalling only).

Every filter step runs in the library's HIP kernels; PyTorch provides device
memory (tensors) and the HIP stream (torch.cuda.current_stream()). torch is
imported before the library is loaded so that both use the same HIP runtime.
There is no CPU fallback: if libvf.so is missing or no GPU is present the
calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import torch  # noqa: F401  (loads the HIP runtime the library links against)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvf.so")

VF_OK, VF_EINVAL, VF_EDOMAIN, VF_ENOCONV, VF_EHIP, VF_ENOMEM, VF_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
VF_U8, VF_U16 = 1, 2
FILTERS = {"vdf": 0, "ddf": 1, "amnfe": 2, "fuzzy_exp": 2, "evmf": 3, "log": 3, "amnfg": 4}
KERNELS = {"exp": 0, "gauss": 1}
EVALS = {"exact": 0, "paper": 1, "split": 2, "chord": 3, "minimax": 4, "rational": 5, "ratfit": 6}
FUNCS = {"acos": 1, "asin": 2, "asin2_tau": 3, "chord": 4, "expneg": 5, "ln1p": 6, "xlnx": 7}
VF_NO_RECHECK = 0x1
VF_DIRECT = 0x2
VF_DEFER_RECHECK = 0x4
VF_TUNED = 0x8

# the symbols include/vf.h declares
EXPORTS = ("vf_create", "vf_destroy", "vf_filter_vdf", "vf_filter_ddf", "vf_filter_fuzzy_exp",
           "vf_filter_log", "vf_filter_batch", "vf_minimax_coeffs", "vf_get_approximant",
           "vf_eval_function", "vf_get_stats", "vf_status_string", "vf_last_error",
           "vf_recheck_pending", "vf_autotune", "vf_tune_save", "vf_tune_load", "vf_tune_clear",
           "vf_filter_vdf_noalloc", "vf_minimax_rational", "vf_quality")


class VfError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"vf status {status}: {detail}")
        self.status = status


class _Approx(C.Structure):
    _fields_ = [("eval", C.c_int32), ("degree", C.c_int32), ("precision", C.c_int32),
                ("scheme", C.c_int32), ("flags", C.c_uint32)]


class _Image(C.Structure):
    _fields_ = [("src", C.c_void_p), ("dst", C.c_void_p), ("height", C.c_int32),
                ("width", C.c_int32), ("src_pitch", C.c_int64), ("dst_pitch", C.c_int64),
                ("dtype", C.c_int32)]


class _BatchItem(C.Structure):
    _fields_ = [("img", _Image), ("filter", C.c_int32), ("window", C.c_int32),
                ("param", C.c_double), ("approx", _Approx)]


class _TuneResult(C.Structure):
    _fields_ = [("direct", C.c_int32), ("strip_rows", C.c_int32), ("degree", C.c_int32),
                ("scheme", C.c_int32), ("precision", C.c_int32), ("candidates", C.c_int32),
                ("ms", C.c_double), ("func_err", C.c_double)]


class _Stats(C.Structure):
    _fields_ = [("windows", C.c_uint64), ("flagged", C.c_uint64), ("tile_w", C.c_int32),
                ("tile_h", C.c_int32), ("workgroups", C.c_int32), ("streaming", C.c_int32)]


@dataclass
class Approx:
    """How a filter evaluates its elementary function (vf_approx)."""
    eval: str = "exact"
    degree: int = 0
    recheck: bool = True
    direct: bool = False      # VDF/DDF: per-window pair scoring instead of streaming
    defer: bool = False       # list near ties but leave the re-check to recheck_pending()
    precision: str = "fp32"   # 'fp32' | 'fp16x2' (chord angle / minimax exp, ln; streaming kernels)
                              # | 'fp64' (every window in FP64: the correctness anchor)
    scheme: str = "horner"    # 'horner' | 'estrin' (chord angle approximant, streaming kernels)
    tuned: bool = False       # use the context's autotuned configuration (see autotune())

    def struct(self) -> _Approx:
        a = _Approx()
        a.eval = EVALS[self.eval]
        a.degree = self.degree
        a.precision = {"fp32": 0, "fp16x2": 1, "fp64": 2}[self.precision]
        a.scheme = {"horner": 0, "estrin": 1}[self.scheme]
        a.flags = ((0 if self.recheck else VF_NO_RECHECK) | (VF_DIRECT if self.direct else 0) |
                   (VF_DEFER_RECHECK if self.defer else 0) | (VF_TUNED if self.tuned else 0))
        return a


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_1009_0959_amd.build")
        L = C.CDLL(LIB_PATH)
        for name in EXPORTS:
            getattr(L, name).restype = C.c_int32
        L.vf_status_string.restype = C.c_char_p
        L.vf_last_error.restype = C.c_char_p
        L.vf_create.argtypes = [C.c_int32, C.POINTER(C.c_void_p)]
        L.vf_destroy.argtypes = [C.c_void_p]
        L.vf_filter_vdf.argtypes = [C.c_void_p, C.POINTER(_Image), C.c_int32, C.POINTER(_Approx), C.c_void_p]
        L.vf_filter_vdf_noalloc.argtypes = [C.c_int32, C.POINTER(_Image), C.c_int32, C.POINTER(_Approx),
                                            C.c_void_p]
        L.vf_filter_ddf.argtypes = [C.c_void_p, C.POINTER(_Image), C.c_int32, C.c_double,
                                    C.POINTER(_Approx), C.c_void_p]
        L.vf_filter_fuzzy_exp.argtypes = [C.c_void_p, C.POINTER(_Image), C.c_int32, C.c_double, C.c_int32,
                                          C.POINTER(_Approx), C.c_void_p]
        L.vf_filter_log.argtypes = [C.c_void_p, C.POINTER(_Image), C.c_int32, C.c_double, C.POINTER(_Approx),
                                    C.c_void_p]
        L.vf_filter_batch.argtypes = [C.c_void_p, C.POINTER(_BatchItem), C.c_int32, C.c_void_p]
        L.vf_quality.argtypes = [C.c_void_p, C.POINTER(_Image), C.POINTER(_Quality), C.c_void_p]
        L.vf_minimax_coeffs.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_int32, C.c_int32,
                                        C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.vf_minimax_rational.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_int32, C.c_int32,
                                          C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.vf_get_approximant.argtypes = [C.c_int32, C.c_int32, C.c_double, C.POINTER(_Approx),
                                         C.POINTER(C.c_float), C.POINTER(C.c_int32),
                                         C.POINTER(C.c_float), C.POINTER(C.c_int32),
                                         C.POINTER(C.c_double)]
        L.vf_eval_function.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.POINTER(_Approx),
                                       C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
        L.vf_get_stats.argtypes = [C.c_void_p, C.POINTER(_Stats)]
        L.vf_recheck_pending.argtypes = [C.c_void_p, C.c_void_p]
        L.vf_autotune.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.POINTER(_Approx),
                                  C.POINTER(_Image), C.c_double, C.POINTER(_TuneResult), C.c_void_p]
        L.vf_tune_save.argtypes = [C.c_void_p, C.c_char_p]
        L.vf_tune_load.argtypes = [C.c_void_p, C.c_char_p]
        L.vf_tune_clear.argtypes = [C.c_void_p]
        L.vf_status_string.argtypes = [C.c_int32]
        L.vf_last_error.argtypes = []
        _lib = L
    return _lib


def _check(status: int):
    if status != VF_OK:
        detail = lib().vf_last_error().decode()
        raise VfError(status, f"{lib().vf_status_string(status).decode()} ({detail})")


# ---------------------------------------------------------------- host-only calls

def minimax_coeffs(func: str, a: float, b: float, degree: int, odd: bool = False):
    """(coefficients, levelled error) from the library's Remez exchange."""
    n = (degree + 1) // 2 if odd else degree + 1
    buf = (C.c_double * 17)()
    err = C.c_double()
    _check(lib().vf_minimax_coeffs(FUNCS[func], a, b, degree, 1 if odd else 0, buf, C.byref(err)))
    return [buf[i] for i in range(n)], err.value


def minimax_rational(func: str, a: float, b: float, n: int, m: int):
    """(numerator, denominator with den[0] = 1, levelled error) of the library's
    best R^n_m approximation (rational Remez exchange)."""
    num = (C.c_double * 9)()
    den = (C.c_double * 9)()
    err = C.c_double()
    _check(lib().vf_minimax_rational(FUNCS[func], a, b, n, m, num, den, C.byref(err)))
    return [num[i] for i in range(n + 1)], [den[i] for i in range(m + 1)], err.value


def get_approximant(filter: str, window: int, param: float, approx: Approx):
    """(lo constants, hi constants, minimax error) a filter call evaluates."""
    lo = (C.c_float * 16)()
    hi = (C.c_float * 16)()
    nlo, nhi = C.c_int32(), C.c_int32()
    eps = C.c_double()
    a = approx.struct()
    _check(lib().vf_get_approximant(FILTERS[filter], window, param, C.byref(a), lo, C.byref(nlo), hi,
                                    C.byref(nhi), C.byref(eps)))
    return [lo[i] for i in range(nlo.value)], [hi[i] for i in range(nhi.value)], eps.value


# ---------------------------------------------------------------- contexts

_contexts: Dict[int, C.c_void_p] = {}


def context(device: Optional[int] = None) -> C.c_void_p:
    dev = torch.cuda.current_device() if device is None else device
    if dev not in _contexts:
        h = C.c_void_p()
        _check(lib().vf_create(dev, C.byref(h)))
        _contexts[dev] = h
    return _contexts[dev]


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _image(src: torch.Tensor, dst: torch.Tensor) -> _Image:
    if not (src.is_cuda and dst.is_cuda):
        raise ValueError("src and dst must be GPU tensors")
    if src.dim() != 3 or src.shape[2] != 3:
        raise ValueError("expected an H x W x 3 tensor")
    if src.dtype not in (torch.uint8, torch.uint16) or dst.dtype != src.dtype or dst.shape != src.shape:
        raise ValueError("uint8/uint16 tensors of identical shape and dtype required")
    for t in (src, dst):
        if t.stride(2) != 1 or t.stride(1) != 3:
            raise ValueError("rows must be interleaved RGB (stride (pitch, 3, 1))")
    es = src.element_size()
    im = _Image()
    im.src = src.data_ptr()
    im.dst = dst.data_ptr()
    im.height, im.width = src.shape[0], src.shape[1]
    im.src_pitch = src.stride(0) * es
    im.dst_pitch = dst.stride(0) * es
    im.dtype = VF_U16 if src.dtype == torch.uint16 else VF_U8
    return im


def _out(img: torch.Tensor, out: Optional[torch.Tensor]) -> torch.Tensor:
    return torch.empty_like(img, memory_format=torch.contiguous_format) if out is None else out


# ---------------------------------------------------------------- filters

def filter_vdf(img: torch.Tensor, window: int = 3, approx: Approx = Approx(),
               out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Vector directional filter (Section 3.1); see vf_filter_vdf in include/vf.h."""
    out = _out(img, out)
    im, a = _image(img, out), approx.struct()
    _check(lib().vf_filter_vdf(context(img.device.index), C.byref(im), window, C.byref(a), _stream()))
    return out


def filter_vdf_noalloc(img: torch.Tensor, window: int = 3, approx: Approx = Approx(),
                       out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """vf_filter_vdf_noalloc: the VDF without device allocation or context
    (the library's static scratch); out is allocated here when not given."""
    out = _out(img, out)
    im, a = _image(img, out), approx.struct()
    _check(lib().vf_filter_vdf_noalloc(img.device.index, C.byref(im), window, C.byref(a), _stream()))
    return out


def filter_ddf(img: torch.Tensor, window: int = 3, p: float = 0.5, approx: Approx = Approx(),
               out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Directional-distance filter; see vf_filter_ddf."""
    out = _out(img, out)
    im, a = _image(img, out), approx.struct()
    _check(lib().vf_filter_ddf(context(img.device.index), C.byref(im), window, p, C.byref(a), _stream()))
    return out


def filter_fuzzy_exp(img: torch.Tensor, window: int = 3, kappa: float = 0.33,
                     approx: Approx = Approx(), out: Optional[torch.Tensor] = None,
                     kernel: str = "exp") -> torch.Tensor:
    """AMNF filters (Section 3.2): kernel 'exp' (AMNFE) or 'gauss' (AMNFG);
    see vf_filter_fuzzy_exp."""
    out = _out(img, out)
    im, a = _image(img, out), approx.struct()
    _check(lib().vf_filter_fuzzy_exp(context(img.device.index), C.byref(im), window, kappa, KERNELS[kernel],
                                     C.byref(a), _stream()))
    return out


def filter_log(img: torch.Tensor, window: int = 3, approx: Approx = Approx(),
               out: Optional[torch.Tensor] = None, cutoff: Optional[float] = None) -> torch.Tensor:
    """Entropy vector median filter (Section 3.3); see vf_filter_log. cutoff:
    the ENT cutoff T (None: 0.05 for the paper's rational, else 0)."""
    out = _out(img, out)
    im, a = _image(img, out), approx.struct()
    t = default_param("evmf", approx) if cutoff is None else cutoff
    _check(lib().vf_filter_log(context(img.device.index), C.byref(im), window, t, C.byref(a), _stream()))
    return out


def default_param(filter: str, approx: Optional[Approx] = None) -> float:
    """p (DDF), kappa (AMNF) or the ENT cutoff T (EVMF: the paper's 0.05 with
    its Table 4 rational, which holds only above it; otherwise no cutoff)."""
    if filter in ("evmf", "log"):
        return 0.05 if approx is not None and approx.eval == "paper" else 0.0
    return {"vdf": 0.0, "ddf": 0.5, "amnfe": 0.33, "fuzzy_exp": 0.33, "amnfg": 0.33}[filter]


def run(filter: str, img: torch.Tensor, window: int = 3, approx: Approx = Approx(),
        param: Optional[float] = None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    p = default_param(filter, approx) if param is None else param
    if filter == "vdf":
        return filter_vdf(img, window, approx, out)
    if filter == "ddf":
        return filter_ddf(img, window, p, approx, out)
    if filter in ("amnfe", "fuzzy_exp"):
        return filter_fuzzy_exp(img, window, p, approx, out)
    if filter == "amnfg":
        return filter_fuzzy_exp(img, window, p, approx, out, kernel="gauss")
    return filter_log(img, window, approx, out, cutoff=p)


def filter_batch(items: Sequence[Tuple[torch.Tensor, str, int, Optional[float], Approx]],
                 outs: Optional[List[torch.Tensor]] = None) -> List[torch.Tensor]:
    """Filter many images in one submission; items are (img, filter, window, param, approx)."""
    if not items:
        return []
    outs = outs or [torch.empty_like(it[0]) for it in items]
    arr = (_BatchItem * len(items))()
    for k, (img, filt, window, param, approx) in enumerate(items):
        arr[k].img = _image(img, outs[k])
        arr[k].filter = FILTERS[filt]
        arr[k].window = window
        arr[k].param = default_param(filt, approx) if param is None else param
        arr[k].approx = approx.struct()
    _check(lib().vf_filter_batch(context(items[0][0].device.index), arr, len(items), _stream()))
    return outs


def eval_function(filter: str, x: torch.Tensor, approx: Approx, window: int = 5,
                  param: Optional[float] = None) -> torch.Tensor:
    """The filter's elementary function evaluated as its kernels do (FP32)."""
    x = x.contiguous().float()
    out = torch.empty_like(x)
    a = approx.struct()
    p = default_param(filter, approx) if param is None else param
    _check(lib().vf_eval_function(context(x.device.index), FILTERS[filter], window, p, C.byref(a),
                                  C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()), x.numel(),
                                  _stream()))
    return out


def autotune(filter: str, img: torch.Tensor, window: int = 3, approx: Approx = Approx(),
             max_func_err: float = 0.0, param: Optional[float] = None,
             out: Optional[torch.Tensor] = None) -> dict:
    """Time every configuration of this filter family on img (vf_autotune) and
    store the fastest in the context; calls with Approx(..., tuned=True) use it."""
    out = _out(img, out)
    im, a, r = _image(img, out), approx.struct(), _TuneResult()
    p = default_param(filter, approx) if param is None else param
    _check(lib().vf_autotune(context(img.device.index), FILTERS[filter], window, p, C.byref(a), C.byref(im),
                             max_func_err, C.byref(r), _stream()))
    return {"direct": bool(r.direct), "strip_rows": r.strip_rows, "degree": r.degree,
            "scheme": ("horner", "estrin")[r.scheme], "precision": ("fp32", "fp16x2")[r.precision],
            "candidates": r.candidates, "ms": r.ms, "func_err": r.func_err}


def tune_save(path: str, device: Optional[int] = None) -> None:
    _check(lib().vf_tune_save(context(device), os.fsencode(path)))


def tune_load(path: str, device: Optional[int] = None) -> None:
    _check(lib().vf_tune_load(context(device), os.fsencode(path)))


def tune_clear(device: Optional[int] = None) -> None:
    _check(lib().vf_tune_clear(context(device)))


def recheck_pending(device: Optional[int] = None) -> None:
    """Run the re-check left pending by a call with Approx(defer=True)."""
    _check(lib().vf_recheck_pending(context(device), _stream()))


class _Quality(C.Structure):
    _fields_ = [("pixels", C.c_uint64), ("l1_sum", C.c_uint64), ("l2sq_sum", C.c_uint64),
                ("lab_diff_sum", C.c_double), ("lab_ref_sum", C.c_double), ("mae", C.c_double),
                ("mse", C.c_double), ("ncd", C.c_double)]


def quality(original: torch.Tensor, filtered: torch.Tensor) -> dict:
    """Section 4's criteria of `filtered` against `original` (vf_quality):
    MAE, MSE, NCD and the sums they come from. Waits for the current stream."""
    im, q = _image(original, filtered), _Quality()
    _check(lib().vf_quality(context(original.device.index), C.byref(im), C.byref(q), _stream()))
    return {k: getattr(q, k) for k, _ in _Quality._fields_}


def get_stats(device: Optional[int] = None) -> dict:
    s = _Stats()
    _check(lib().vf_get_stats(context(device), C.byref(s)))
    return {"windows": s.windows, "flagged": s.flagged, "tile_w": s.tile_w, "tile_h": s.tile_h,
            "workgroups": s.workgroups, "streaming": s.streaming}
