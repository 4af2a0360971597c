"""Oracle: minimax polynomial approximation by the Remez exchange algorithm, in FP64.

TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product library never does.

What it computes (paper, Section 2): for f continuous on [a, b] and a degree n,
the polynomial P in P_n (monomial form a_0 + a_1 z + ... + a_n z^n, the form of
the equation defining P_n and of Tables 1-2) that minimises
    eps = max_{z in [a,b]} |f(z) - P(z)|      (the minimax error of Section 2).
The paper computes P with the Remez exchange algorithm (named in Section 2; the
implementation details it defers to a cited report that is not reproduced).
This file writes the textbook exchange iteration out plainly:

  1. start from the n+2 Chebyshev extrema of [a, b];
  2. solve  sum_k c_k t_i^k + (-1)^i E = f(z_i)  for the coefficients and the
     levelled error E (a dense linear solve is the library primitive used);
  3. locate the local extrema of e = f - P (dense grid + golden-section);
  4. exchange: keep one extremum per run of equal sign, trim to n+2 points;
  5. stop once max|e| - |E| <= tol (and <= 1e-10 |E|, above FP64 noise).

The work variable is t = (z - mid)/half in [-1, 1] (monomials in t are well
conditioned); the result is re-expanded into monomials of z at the end.

Odd approximants on a symmetric interval [-b, b] are obtained the plain way:
the best approximation of an odd function from P_{d+1} (d odd) on a symmetric
interval is odd and is also its best approximation from P_d, so the oracle
runs the full-basis iteration at degree d+1 and reads off the odd coefficients
(the even ones come out at round-off level and are checked to be so).
"""
from __future__ import annotations

import math
from typing import Callable, Dict, Tuple

import numpy as np


def _xlnx(z):
    z = np.asarray(z, dtype=np.float64)
    out = np.zeros_like(z)
    pos = z > 0
    out[pos] = z[pos] * np.log(z[pos])
    return out


# The elementary functions of Section 3 and the forms the paper approximates.
FUNCTIONS: Dict[str, Callable[[np.ndarray], np.ndarray]] = {
    # Section 3.1: arccos on [0, 0.5] (Table 1, ARCCOS row)
    "acos": np.arccos,
    # arcsin, used for the odd split of arccos around z = 0
    "asin": np.arcsin,
    # Section 3.1: 2 asin(tau / sqrt 2) with tau = sqrt(1 - z) (Table 1, ARCSIN row)
    "asin2_tau": lambda t: 2.0 * np.arcsin(np.asarray(t) / math.sqrt(2.0)),
    # the same angle as a function of the chord s = sqrt(2 (1 - z)) = sqrt(2) tau
    "chord": lambda s: 2.0 * np.arcsin(np.asarray(s) / 2.0),
    # Section 3.2: exp(-z) (Table 2)
    "expneg": lambda z: np.exp(-np.asarray(z)),
    # natural log of the reduced mantissa, ln(1 + t), for the entropy term
    "ln1p": np.log1p,
    # Section 3.3: z ln z (the ENT function)
    "xlnx": _xlnx,
}


class RemezError(RuntimeError):
    pass


def _golden_max(g: Callable[[float], float], lo: float, hi: float, iters: int = 80) -> float:
    """Argmax of a unimodal g on [lo, hi] by golden-section search."""
    r = (math.sqrt(5.0) - 1.0) / 2.0
    a, b = lo, hi
    c = b - r * (b - a)
    d = a + r * (b - a)
    gc, gd = g(c), g(d)
    for _ in range(iters):
        if gc >= gd:
            b, d, gd = d, c, gc
            c = b - r * (b - a)
            gc = g(c)
        else:
            a, c, gc = c, d, gd
            d = a + r * (b - a)
            gd = g(d)
        if b - a < 1e-17 * max(1.0, abs(a)):
            break
    return 0.5 * (a + b)


def _poly_t(c_t: np.ndarray, t):
    # Horner in t; c_t[k] multiplies t**k
    acc = np.zeros_like(np.asarray(t, dtype=np.float64)) + c_t[-1]
    for ck in c_t[-2::-1]:
        acc = acc * t + ck
    return acc


def remez_full(f: Callable, a: float, b: float, n: int, tol: float = 1e-12,
               max_iter: int = 80, grid_per_point: int = 4000) -> Tuple[np.ndarray, float, dict]:
    """Minimax P in P_n on [a, b] for f.

    Returns (coefficients of z^0..z^n, levelled error |E|, info) where info holds
    the final reference points, the signed errors there and the observed max|e|.
    """
    if not (b > a):
        raise ValueError("empty interval")
    if n < 0:
        raise ValueError("negative degree")
    mid, half = 0.5 * (a + b), 0.5 * (b - a)
    fz = lambda t: np.asarray(f(mid + half * np.asarray(t, dtype=np.float64)), dtype=np.float64)
    m = n + 2
    k = np.arange(m)
    t_ref = -np.cos(k * math.pi / (n + 1))          # Chebyshev extrema, ascending
    signs = np.where(k % 2 == 0, 1.0, -1.0)
    grid = np.linspace(-1.0, 1.0, grid_per_point * m + 1)
    f_grid = fz(grid)
    history = []
    for it in range(max_iter):
        # step 2: levelled system
        A = np.empty((m, m))
        A[:, :n + 1] = np.vander(t_ref, n + 1, increasing=True)
        A[:, n + 1] = signs
        sol = np.linalg.solve(A, fz(t_ref))
        c_t, E = sol[:n + 1], sol[n + 1]
        # step 3: extrema of the error curve
        e_grid = f_grid - _poly_t(c_t, grid)
        de = np.diff(e_grid)
        cand = [0]
        for i in range(1, len(grid) - 1):
            if de[i - 1] * de[i] <= 0.0 and not (de[i - 1] == 0.0 and de[i] == 0.0):
                cand.append(i)
        cand.append(len(grid) - 1)
        pts, vals = [], []
        for i in cand:
            if i == 0 or i == len(grid) - 1:
                t_i = grid[i]
            else:
                s = 1.0 if e_grid[i] > 0 else -1.0
                g = lambda t, s=s: s * float(fz(t) - _poly_t(c_t, t))
                t_i = _golden_max(g, grid[i - 1], grid[i + 1])
            pts.append(t_i)
            vals.append(float(fz(t_i) - _poly_t(c_t, t_i)))
        # step 4: one extremum per sign run
        run_t, run_e = [pts[0]], [vals[0]]
        for t_i, e_i in zip(pts[1:], vals[1:]):
            if (e_i > 0) == (run_e[-1] > 0):
                if abs(e_i) > abs(run_e[-1]):
                    run_t[-1], run_e[-1] = t_i, e_i
            else:
                run_t.append(t_i)
                run_e.append(e_i)
        max_err = max(abs(v) for v in run_e)
        history.append((abs(E), max_err))
        if len(run_t) < m:
            raise RemezError(f"only {len(run_t)} alternating extrema (need {m}) at iteration {it}")
        while len(run_t) > m:
            if abs(run_e[0]) < abs(run_e[-1]):
                run_t.pop(0); run_e.pop(0)
            else:
                run_t.pop(); run_e.pop()
        # stop once the extrema equal the levelled error within tol, and
        # within 1e-10 of |E| relative (no tighter than FP64 evaluation of the
        # error curve allows, about 1e-15)
        if max_err - abs(E) <= min(tol, max(1e-10 * abs(E), 1e-15)):
            coeffs = _t_to_z(c_t, mid, half)
            info = {"ref_t": np.array(run_t), "ref_z": mid + half * np.array(run_t),
                    "ref_err": np.array(run_e), "max_err": max_err, "iterations": it + 1,
                    "history": history}
            return coeffs, abs(E), info
        t_ref = np.array(run_t)
        signs = np.where(np.array(run_e) > 0, 1.0, -1.0)
        # keep the sign pattern consistent with the system's (-1)^i column
    raise RemezError(f"no convergence after {max_iter} iterations (last {history[-1]})")


def _t_to_z(c_t: np.ndarray, mid: float, half: float) -> np.ndarray:
    """Re-expand sum c_k ((z - mid)/half)^k into monomials of z."""
    n = len(c_t) - 1
    out = np.zeros(n + 1)
    for k in range(n + 1):
        scale = c_t[k] / half ** k
        for j in range(k + 1):
            out[j] += scale * math.comb(k, j) * (-mid) ** (k - j)
    return out


def remez(func: str, a: float, b: float, degree: int, odd: bool = False, tol: float = 1e-12):
    """Coefficients (monomials in the function's own variable) and levelled error.

    func names an entry of FUNCTIONS. With odd=True the interval must be
    symmetric (a == -b), degree odd, and only the odd coefficients
    c_1, c_3, ..., c_degree are returned (in that order).
    """
    f = FUNCTIONS[func]
    if not odd:
        c, E, info = remez_full(f, a, b, degree, tol=tol)
        return c, E, info
    if a != -b or degree % 2 != 1:
        raise ValueError("odd approximants need a symmetric interval and an odd degree")
    c, E, info = remez_full(f, a, b, degree + 1, tol=tol)
    even = c[0::2]
    if np.max(np.abs(even)) > 1e-9:
        raise RemezError(f"even coefficients not negligible: {even}")
    return c[1::2].copy(), E, info


def horner(c: np.ndarray, z):
    acc = np.zeros_like(np.asarray(z, dtype=np.float64)) + c[-1]
    for ck in c[-2::-1]:
        acc = acc * z + ck
    return acc


def eval_odd(c_odd: np.ndarray, z):
    """sum_k c_odd[k] z^(2k+1), evaluated as z * P(z*z)."""
    z = np.asarray(z, dtype=np.float64)
    return z * horner(np.asarray(c_odd), z * z)


# ---------------------------------------------------------------- rational class R^n_m

def _q_sign_ok(q_t: np.ndarray) -> bool:
    """The denominator keeps one sign on [-1, 1] (dense check)."""
    t = np.linspace(-1.0, 1.0, 20001)
    v = _poly_t(q_t, t)
    return bool(np.all(v > 0) or np.all(v < 0))


def remez_rational(f: Callable, a: float, b: float, n: int, m: int, tol: float = 1e-12,
                   max_iter: int = 80, grid_per_point: int = 4000):
    """Best approximation of f on [a, b] from the rational class R^n_m of
    Section 2 (p in P_n over q in P_m), by the rational Remez exchange.

    Steps, as for remez_full, in t = (z - mid)/half:
      1. reference: the n+m+2 Chebyshev extrema of [-1, 1];
      2. levelled system p(t_i) = (f(t_i) - (-1)^i E) q(t_i): homogeneous in
         (p, q) and linear in E, i.e. the generalized eigenproblem
         A u = E (-B) u with A = [V_n, -diag(f) V_m], B = [0, diag(s) V_m]
         (a library eigen-solver is the primitive); of its real eigenvalues
         the one of least |E| whose q keeps one sign on the interval is taken;
      3.-5. extrema of e = f - p/q, exchange, stop as in remez_full.
    Returns (numerator coefficients of z^0..z^n, denominator coefficients of
    z^0..z^m scaled so that the z^0 one is 1, levelled error |E|, info)."""
    import scipy.linalg
    if not (b > a):
        raise ValueError("empty interval")
    if n < 0 or m < 0:
        raise ValueError("negative degree")
    mid, half = 0.5 * (a + b), 0.5 * (b - a)
    fz = lambda t: np.asarray(f(mid + half * np.asarray(t, dtype=np.float64)), dtype=np.float64)
    N = n + m + 2
    k = np.arange(N)
    t_ref = -np.cos(k * math.pi / (N - 1))
    signs = np.where(k % 2 == 0, 1.0, -1.0)
    grid = np.linspace(-1.0, 1.0, grid_per_point * N + 1)
    f_grid = fz(grid)
    history = []
    for it in range(max_iter):
        fi = fz(t_ref)
        Vn = np.vander(t_ref, n + 1, increasing=True)
        Vm = np.vander(t_ref, m + 1, increasing=True)
        A = np.hstack([Vn, -fi[:, None] * Vm])
        B = np.hstack([np.zeros((N, n + 1)), signs[:, None] * Vm])
        w, vr = scipy.linalg.eig(A, -B)
        best = None
        for lam, vec in zip(w, vr.T):
            if not np.isfinite(lam) or abs(lam.imag) > 1e-9 * max(1.0, abs(lam.real)):
                continue
            vec = np.real(vec)
            p_t, q_t = vec[:n + 1], vec[n + 1:]
            if not np.any(q_t) or not _q_sign_ok(q_t):
                continue
            if best is None or abs(lam.real) < abs(best[0]):
                best = (lam.real, p_t, q_t)
        if best is None:
            raise RemezError(f"no admissible levelled solution at iteration {it}")
        E, p_t, q_t = best
        r = lambda t: _poly_t(p_t, t) / _poly_t(q_t, t)
        e_grid = f_grid - r(grid)
        de = np.diff(e_grid)
        cand = [0]
        for i in range(1, len(grid) - 1):
            if de[i - 1] * de[i] <= 0.0 and not (de[i - 1] == 0.0 and de[i] == 0.0):
                cand.append(i)
        cand.append(len(grid) - 1)
        pts, vals = [], []
        for i in cand:
            if i == 0 or i == len(grid) - 1:
                t_i = grid[i]
            else:
                s = 1.0 if e_grid[i] > 0 else -1.0
                g = lambda t, s=s: s * float(fz(t) - r(t))
                t_i = _golden_max(g, grid[i - 1], grid[i + 1])
            pts.append(t_i)
            vals.append(float(fz(t_i) - r(t_i)))
        run_t, run_e = [pts[0]], [vals[0]]
        for t_i, e_i in zip(pts[1:], vals[1:]):
            if (e_i > 0) == (run_e[-1] > 0):
                if abs(e_i) > abs(run_e[-1]):
                    run_t[-1], run_e[-1] = t_i, e_i
            else:
                run_t.append(t_i)
                run_e.append(e_i)
        max_err = max(abs(v) for v in run_e)
        history.append((abs(E), max_err))
        # (the quotient's FP64 evaluation puts the error curve's noise near
        # 1e-14, above the polynomial case's)
        if max_err - abs(E) <= min(tol, max(1e-10 * abs(E), 1e-14)):
            num = _t_to_z(p_t, mid, half)
            den = _t_to_z(q_t, mid, half)
            num, den = num / den[0], den / den[0]
            info = {"ref_t": np.array(run_t), "ref_z": mid + half * np.array(run_t),
                    "ref_err": np.array(run_e), "max_err": max_err, "iterations": it + 1,
                    "history": history}
            return num, den, abs(E), info
        if len(run_t) < N:
            raise RemezError(f"only {len(run_t)} alternating extrema (need {N}) at iteration {it}")
        while len(run_t) > N:
            if abs(run_e[0]) < abs(run_e[-1]):
                run_t.pop(0); run_e.pop(0)
            else:
                run_t.pop(); run_e.pop()
        t_ref = np.array(run_t)
        signs = np.where(np.array(run_e) > 0, 1.0, -1.0)
    raise RemezError(f"no convergence after {max_iter} iterations (last {history[-1]})")


def rational(func: str, a: float, b: float, n: int, m: int, tol: float = 1e-12):
    """(numerator, denominator, |E|, info) of the best R^n_m approximation of
    a function of FUNCTIONS (denominator's z^0 coefficient 1)."""
    return remez_rational(FUNCTIONS[func], a, b, n, m, tol=tol)
