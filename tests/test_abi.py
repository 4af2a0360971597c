"""CPU tests of the C-ABI library: it loads, exports every declared symbol, and
its host-only calls (the library's own Remez exchange and the approximant
preparation) agree with the oracle and the paper. No GPU call is made here."""
import math
import os
import re

import numpy as np
import pytest

import oracle
from oracle import paper_tables as PT
from conftest import ROOT, golden_table
from oracle.remez import FUNCTIONS, eval_odd, horner, remez as oracle_remez

vf = pytest.importorskip("paper_1009_0959_amd.vf")

G = golden_table("paper_tables.txt")


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "vf.h")).read()
    return sorted(set(re.findall(r"^(?:vf_status|const char\*)\s+(vf_\w+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(vf.LIB_PATH):
        pytest.skip("libvf.so not built")
    return vf.lib()


def test_exports_every_declared_symbol(L):
    names = declared_symbols()
    assert len(names) >= 13
    assert set(names) == set(vf.EXPORTS)
    for n in names:
        assert hasattr(L, n)


def test_status_strings(L):
    assert L.vf_status_string(0) == b"ok"
    assert b"invalid" in L.vf_status_string(-1)
    assert L.vf_status_string(12345) == b"unknown status"


@pytest.mark.parametrize("func,a,b,d,odd", [
    ("asin2_tau", 0.0, 1 / math.sqrt(2), 4, False), ("acos", 0.0, 0.5, 4, False),
    ("expneg", 0.0, 10.0, 2, False), ("expneg", 0.0, 10.0, 3, False), ("expneg", 0.0, 10.0, 4, False),
    ("expneg", 0.0, 25 ** 0.11, 6, False), ("ln1p", 0.0, 1.0, 7, False),
    ("asin", -0.5, 0.5, 5, True), ("chord", -1.0, 1.0, 9, True),
    ("chord", -math.sqrt(2), math.sqrt(2), 11, True), ("expneg", 0.0, 10.0, 12, False),
])
def test_library_remez_matches_oracle(L, func, a, b, d, odd):
    c_lib, e_lib = vf.minimax_coeffs(func, a, b, d, odd)
    c_orc, e_orc, _ = oracle_remez(func, a, b, d, odd=odd)
    assert abs(e_lib - e_orc) <= 2e-12 + 1e-9 * e_orc
    scale = max(1.0, max(abs(c) for c in c_orc))
    assert np.max(np.abs(np.array(c_lib) - np.array(c_orc))) <= 1e-9 * scale
    # and the library's polynomial really has max error E (within the 1e-12 stop)
    z = np.linspace(a, b, 200001)
    f = FUNCTIONS[func](z)
    p = eval_odd(np.array(c_lib), z) if odd else horner(np.array(c_lib), z)
    assert abs(np.max(np.abs(f - p)) - e_lib) <= 2e-12 + 1e-7 * e_lib


def test_library_remez_reproduces_table1_and_2(L):
    for row, func, a, b in [("T1_ARCSIN", "asin2_tau", 0.0, 1 / math.sqrt(2)), ("T1_ARCCOS", "acos", 0.0, 0.5)]:
        eps, *printed = G[row]
        c, E = vf.minimax_coeffs(func, a, b, 4)
        assert E <= eps * (1 + 1e-6) and abs(E - eps) / eps <= 1e-4
        for u, v in zip(c, printed):
            assert abs(u - v) <= 2e-5 * abs(v) + 1e-9
    for d in (2, 3, 4):
        eps, *printed = G[f"T2_P{d}"]
        c, E = vf.minimax_coeffs("expneg", 0.0, 10.0, d)
        assert abs(E - eps) / eps <= 1e-4
        for u, v in zip(c, printed):
            assert abs(u - v) <= 2e-5 * abs(v) + 1e-9


@pytest.mark.parametrize("args,status", [
    (("acos", 0.5, 0.5, 3, False), vf.VF_EINVAL),       # empty interval
    (("acos", 0.0, 0.5, 17, False), vf.VF_EINVAL),      # degree too high
    (("asin", -0.5, 0.5, 4, True), vf.VF_EINVAL),       # odd basis needs an odd degree
    (("asin", -0.5, 0.6, 5, True), vf.VF_EINVAL),       # and a symmetric interval
    (("acos", 0.0, 1.5, 3, False), vf.VF_EDOMAIN),
    (("ln1p", -1.0, 1.0, 3, False), vf.VF_EDOMAIN),
    (("xlnx", -0.1, 1.0, 3, False), vf.VF_EDOMAIN),
])
def test_minimax_errors(L, args, status):
    with pytest.raises(vf.VfError) as e:
        vf.minimax_coeffs(*args)
    assert e.value.status == status


def f32list(x):
    return list(np.asarray(x, dtype=np.float32))


def test_paper_constants_are_the_printed_ones(L):
    lo, hi, eps = vf.get_approximant("vdf", 3, 0.0, vf.Approx("paper", 4))
    assert lo == f32list(G["T1_ARCCOS"][1:]) and hi == f32list(G["T1_ARCSIN"][1:])
    for d in (2, 3, 4):
        lo, hi, eps = vf.get_approximant("amnfe", 5, 0.33, vf.Approx("paper", d))
        assert lo == f32list(G[f"T2_P{d}"][1:]) and hi == []
    lo, hi, eps = vf.get_approximant("evmf", 3, 0.05, vf.Approx("paper", 4))
    assert lo == f32list(G["T4_NUM"][1:]) and hi == f32list(G["T4_DEN"][1:])
    for w in (3, 5, 7):
        lo, hi, eps = vf.get_approximant("amnfe", w, 0.33, vf.Approx("rational", 4))
        assert lo == f32list(G["T3_NUM"][1:]) and hi == f32list(G["T3_DEN"][1:])
        assert eps == pytest.approx(2.227050e-06, rel=1e-6)


@pytest.mark.parametrize("kind,degree", [("split", 3), ("split", 5), ("split", 7), ("split", 9),
                                         ("chord", 7), ("chord", 9), ("chord", 11), ("chord", 13)])
def test_angle_constants_match_oracle(L, kind, degree):
    lo, hi, eps = vf.get_approximant("vdf", 5, 0.0, vf.Approx(kind, degree))
    if kind == "split":
        ap = oracle.angle_approx("split", degree)
        assert lo == f32list(ap.lo)
    else:
        ap = oracle.angle_approx("chord", degree)
        assert lo == []
    assert hi == f32list(ap.hi)
    assert abs(eps - ap.eps) <= 2e-12 + 1e-9 * ap.eps


@pytest.mark.parametrize("degree", [7, 9, 11, 13])
def test_fp16_chord_constants_match_oracle(L, degree):
    """The packed-FP16 variant's constants: c_0 as in FP32, c_1.. rounded to
    half precision by the library exactly as the oracle rounds them; its
    reported error is the error of that rounded polynomial."""
    lo, hi, eps = vf.get_approximant("vdf", 5, 0.0, vf.Approx("chord", degree, precision="fp16x2"))
    ap = oracle.angle_approx("chord", degree, precision="fp16x2")
    assert hi == f32list(ap.hi)
    assert np.all(np.asarray(hi[1:], dtype=np.float32).astype(np.float16).astype(np.float32) == np.asarray(hi[1:], dtype=np.float32))
    s = np.linspace(0.0, math.sqrt(2.0), 65537)
    x = s * s
    acc = np.zeros_like(x)
    for c in reversed(ap.hi):
        acc = acc * x + c
    err = np.abs(2.0 * np.arcsin(0.5 * s) - s * acc).max()
    assert abs(eps - err) <= 1e-9 + 1e-6 * err
    # the FP32 fit's own error is smaller: rounding to FP16 costs accuracy
    assert eps >= oracle.angle_approx("chord", degree).eps


@pytest.mark.parametrize("window", [3, 5, 7])
@pytest.mark.parametrize("degree", [2, 3, 4, 5, 6, 7, 8, 9])
def test_exp_and_ent_constants_match_oracle(L, window, degree):
    """Every degree the ABI admits (2..9): the library either evaluates the
    oracle's Remez result rounded to FP32 (same constants), or refuses the
    degree because its minimax error lies below 2^-24 of the function's
    largest value (1 for exp(-z), ln 2 for ln(1 + t)), which the oracle's own
    fit confirms."""
    u = 2.0 ** -24
    fits = [(filt, window, 0.33, oracle.exp_approx("poly", degree, window=window, kernel=kernel), 1.0)
            for filt, kernel in (("amnfe", "exp"), ("amnfg", "gauss"))]
    fits.append(("evmf", window, 0.0, oracle.ent_approx("rangered", degree), math.log(2.0)))
    for filt, w, param, ap, fmax in fits:
        c = ap.coeffs if filt != "evmf" else ap.p
        try:
            lo, hi, eps = vf.get_approximant(filt, w, param, vf.Approx("minimax", degree))
        except vf.VfError as e:
            assert e.status == vf.VF_EUNSUPPORTED
            assert ap.eps < u * fmax, (filt, degree, ap.eps)
            continue
        assert ap.eps >= u * fmax * (1 - 1e-6), (filt, degree)
        assert lo == f32list(c), (filt, degree)
        assert abs(eps - ap.eps) <= 1e-12 + 1e-9 * ap.eps


def test_large_kappa_fit_stops_at_the_cutoff(L):
    """kappa = 4 puts the argument bound past T = 10; the fit covers [0, T]."""
    for filt, kernel in (("amnfe", "exp"), ("amnfg", "gauss")):
        lo, hi, eps = vf.get_approximant(filt, 7, 4.0, vf.Approx("minimax", 6))
        ep = oracle.exp_approx("poly", 6, window=7, kappa=4.0, kernel=kernel)
        assert lo == f32list(ep.coeffs)


@pytest.mark.parametrize("window", [3, 5, 7])
@pytest.mark.parametrize("degree", [4, 5, 6])
def test_fp16_exp_ent_constants_match_oracle(L, window, degree):
    """The packed-FP16 exp / ln1p variants: c_0 as in FP32, c_1.. rounded to
    half precision exactly as the oracle rounds them; the reported error is
    that of the rounded polynomial against the function itself."""
    zmax = oracle.amnfe_range(window)
    for filt, param, ap_o, f, xmax in (
            ("amnfe", 0.33, oracle.exp_approx("poly", degree, window=window, precision="fp16x2"),
             lambda x: np.exp(-x), zmax),
            ("evmf", 0.0, oracle.ent_approx("rangered", degree, precision="fp16x2"), np.log1p, 1.0)):
        lo, hi, eps = vf.get_approximant(filt, window, param, vf.Approx("minimax", degree, precision="fp16x2"))
        c = ap_o.coeffs if filt == "amnfe" else ap_o.p
        assert lo == f32list(c)
        lo32, _, eps32 = vf.get_approximant(filt, window, param, vf.Approx("minimax", degree))
        assert lo[0] == lo32[0]
        tail = np.asarray(lo[1:], dtype=np.float32)
        assert np.all(tail.astype(np.float16).astype(np.float32) == tail)
        x = np.linspace(0.0, xmax, 65537)
        acc = np.zeros_like(x)
        for ck in reversed(c):
            acc = acc * x + ck
        err = np.abs(f(x) - acc).max()
        assert abs(eps - err) <= 1e-12 + 1e-6 * err
        assert eps >= 0.5 * eps32


@pytest.mark.parametrize("filt,window,param,ap,status", [
    ("vdf", 9, 0.0, vf.Approx("exact"), vf.VF_EUNSUPPORTED),
    ("vdf", 4, 0.0, vf.Approx("exact"), vf.VF_EINVAL),
    ("vdf", 3, 0.0, vf.Approx("split", 4), vf.VF_EUNSUPPORTED),
    ("vdf", 3, 0.0, vf.Approx("minimax", 4), vf.VF_EUNSUPPORTED),
    ("ddf", 3, 1.5, vf.Approx("exact"), vf.VF_EINVAL),
    ("amnfe", 3, -1.0, vf.Approx("exact"), vf.VF_EINVAL),
    ("amnfg", 3, 0.0, vf.Approx("exact"), vf.VF_EINVAL),
    ("amnfg", 3, 0.33, vf.Approx("split", 5), vf.VF_EUNSUPPORTED),
    ("vdf", 3, 0.0, vf.Approx("chord", 11, precision="fp64", scheme="estrin"), vf.VF_EUNSUPPORTED),
    ("amnfe", 3, 0.33, vf.Approx("paper", 5), vf.VF_EUNSUPPORTED),
    ("amnfe", 3, 0.33, vf.Approx("rational", 3), vf.VF_EUNSUPPORTED),
    ("amnfe", 3, 0.33, vf.Approx("rational", 4, precision="fp16x2"), vf.VF_EUNSUPPORTED),
    ("vdf", 3, 0.0, vf.Approx("rational", 4), vf.VF_EUNSUPPORTED),
    ("evmf", 3, 0.0, vf.Approx("rational", 4), vf.VF_EUNSUPPORTED),
    ("evmf", 3, 0.0, vf.Approx("split", 5), vf.VF_EUNSUPPORTED),
    ("vdf", 3, 0.0, vf.Approx("split", 5, scheme="estrin"), vf.VF_EUNSUPPORTED),
    ("vdf", 3, 0.0, vf.Approx("split", 5, precision="fp16x2"), vf.VF_EUNSUPPORTED),
    ("amnfe", 3, 0.33, vf.Approx("paper", 4, precision="fp16x2"), vf.VF_EUNSUPPORTED),
    ("amnfe", 3, 0.33, vf.Approx("exact", precision="fp16x2"), vf.VF_EUNSUPPORTED),
    ("evmf", 3, 0.0, vf.Approx("paper", 4, precision="fp16x2"), vf.VF_EUNSUPPORTED),
    ("amnfe", 3, 0.33, vf.Approx("minimax", 5, scheme="estrin"), vf.VF_EUNSUPPORTED),
    ("vdf", 3, 0.0, vf.Approx("chord", 11, scheme="estrin", precision="fp16x2"), vf.VF_EUNSUPPORTED),
    # the ENT cutoff T: within [0, 1]; the Table 4 rational holds only above 0.05
    ("evmf", 3, 0.0, vf.Approx("paper", 4), vf.VF_EDOMAIN),
    ("evmf", 5, 0.049, vf.Approx("paper", 4), vf.VF_EDOMAIN),
    ("evmf", 3, -0.01, vf.Approx("exact"), vf.VF_EINVAL),
    ("evmf", 3, 1.01, vf.Approx("minimax", 6), vf.VF_EINVAL),
    ("evmf", 3, float("nan"), vf.Approx("exact"), vf.VF_EINVAL),
])
def test_approximant_validation(L, filt, window, param, ap, status):
    with pytest.raises(vf.VfError) as e:
        vf.get_approximant(filt, window, param, ap)
    assert e.value.status == status


# ---------------------------------------------------------------- rational class R^n_m

@pytest.mark.parametrize("func,a,b,n,m", [
    ("expneg", 0.0, 10.0, 4, 4), ("xlnx", 0.05, 1.0, 4, 4), ("expneg", 0.0, 25 ** 0.11, 2, 2),
    ("expneg", 0.0, 0.5 * 49 ** 0.22, 2, 2), ("expneg", 0.0, 9 ** 0.11, 1, 1), ("expneg", 0.0, 10.0, 3, 2),
    ("expneg", 0.0, 1.5, 5, 0), ("expneg", 0.0, 10.0, 3, 3)])
def test_library_rational_matches_oracle(L, func, a, b, n, m):
    """The library's rational exchange (Newton on the levelled system) and the
    oracle's (generalized eigenproblem) find the same best R^n_m."""
    pl, ql, El = vf.minimax_rational(func, a, b, n, m)
    po, qo, Eo, _ = oracle.rational(func, a, b, n, m)
    assert abs(El - Eo) <= 1e-9 * Eo + 1e-15
    assert np.all(np.abs(np.array(pl) - po) <= 1e-8 * np.abs(po) + 1e-15)
    assert np.all(np.abs(np.array(ql) - qo) <= 1e-8 * np.abs(qo) + 1e-15)
    assert ql[0] == 1.0


@pytest.mark.parametrize("row,func,a,b", [("T3", "expneg", 0.0, 10.0), ("T4", "xlnx", 0.05, 1.0)])
def test_library_rational_reproduces_tables_3_and_4(L, row, func, a, b):
    num_p, den_p = G[f"{row}_NUM"][1:], G[f"{row}_DEN"][1:]
    eps = G[f"{row}_NUM"][0]
    p, q, E = vf.minimax_rational(func, a, b, 4, 4)
    assert E <= eps * (1 + 1e-6) and abs(E - eps) / eps <= 5e-3
    pn, qn = np.array(num_p) / den_p[0], np.array(den_p) / den_p[0]
    assert np.all(np.abs(np.array(p) - pn) <= 5e-4 * np.abs(pn))
    assert np.all(np.abs(np.array(q) - qn) <= 5e-4 * np.abs(qn) + 1e-15)


@pytest.mark.parametrize("args,status", [
    (("expneg", 1.0, 1.0, 2, 2), vf.VF_EINVAL), (("expneg", 0.0, 1.0, 9, 1), vf.VF_EINVAL),
    (("expneg", 0.0, 1.0, 2, -1), vf.VF_EINVAL), (("ln1p", -2.0, 1.0, 2, 2), vf.VF_EDOMAIN),
    (("acos", 0.0, 1.5, 2, 2), vf.VF_EDOMAIN)])
def test_minimax_rational_errors(L, args, status):
    with pytest.raises(vf.VfError) as e:
        vf.minimax_rational(*args)
    assert e.value.status == status


def test_remez_iteration_cap_reports_no_convergence(L, monkeypatch):
    """VF_REMEZ_MAX_ITER lowers the exchange's iteration cap: with one
    exchange allowed neither exchange converges (VF_ENOCONV, with its message);
    without it the same calls succeed."""
    monkeypatch.setenv("VF_REMEZ_MAX_ITER", "1")
    with pytest.raises(vf.VfError) as e:
        vf.minimax_coeffs("expneg", 0.0, 10.0, 6)
    assert e.value.status == vf.VF_ENOCONV and "converge" in str(e.value)
    with pytest.raises(vf.VfError) as e:
        vf.minimax_rational("expneg", 0.0, 10.0, 4, 4)
    assert e.value.status == vf.VF_ENOCONV
    monkeypatch.delenv("VF_REMEZ_MAX_ITER")
    vf.minimax_coeffs("expneg", 0.0, 10.0, 6)
    vf.minimax_rational("expneg", 0.0, 10.0, 4, 4)


@pytest.mark.parametrize("window", [3, 5, 7])
def test_ratfit_degree4_refused(L, window):
    """R^4_4 on the AMNF argument ranges lies far below FP32 resolution (the
    degree-3 fit is already under 2^-24): refused."""
    for filt in ("amnfe", "amnfg"):
        with pytest.raises(vf.VfError) as e:
            vf.get_approximant(filt, window, 0.33, vf.Approx("ratfit", 4))
        assert e.value.status == vf.VF_EUNSUPPORTED


@pytest.mark.parametrize("window", [3, 5, 7])
@pytest.mark.parametrize("degree", [1, 2, 3])
def test_ratfit_constants_match_oracle(L, window, degree):
    """The fitted R^d_d exp approximants (VF_EVAL_RATFIT): the oracle's rational
    exchange rounded to FP32, or refused below FP32 resolution."""
    u = 2.0 ** -24
    for filt, kernel in (("amnfe", "exp"), ("amnfg", "gauss")):
        ep = oracle.exp_approx("ratfit", degree, window=window, kernel=kernel)
        try:
            lo, hi, eps = vf.get_approximant(filt, window, 0.33, vf.Approx("ratfit", degree))
        except vf.VfError as e:
            assert e.status == vf.VF_EUNSUPPORTED and ep.eps < u
            continue
        assert ep.eps >= u * (1 - 1e-6)
        assert lo == f32list(ep.coeffs) and hi == f32list(ep.q)
        assert abs(eps - ep.eps) <= 1e-9 * ep.eps


def test_create_without_a_device_reports_ehip(L):
    """Error propagation without a GPU: creating a context where HIP finds no
    device returns VF_EHIP, with the failing HIP call in vf_last_error."""
    import ctypes as C
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    ctx = C.c_void_p()
    st = L.vf_create(0, C.byref(ctx))
    assert st == vf.VF_EHIP
    assert ctx.value is None
    assert L.vf_last_error().decode() != ""
