"""Oracle twin: a numpy brute-force version of the filters for tiny images.

TEST INFRASTRUCTURE. It exists to cross-check the C oracle (oracle.c) with a
second, independently written implementation: vectorised numpy instead of C
loops, the angle taken as atan2(|x_i x x_j|, x_i . x_j) instead of acos of the
cosine in exact mode, and the window gathered with numpy's edge padding.
Conventions are the ones stated in oracle.c (replicated borders, row-major
window order, centre-first tie rule, identical/collinear/zero-vector cosines,
uniform-window outputs, floor(v + 0.5) rounding, multiplied-through EVMF test).
"""
from __future__ import annotations

import math

import numpy as np


def windows(img: np.ndarray, w: int) -> np.ndarray:
    """(H, W, n, 3) int64 array of every pixel's window, edge-replicated."""
    r = (w - 1) // 2
    pad = np.pad(img.astype(np.int64), ((r, r), (r, r), (0, 0)), mode="edge")
    H, W = img.shape[:2]
    out = np.empty((H, W, w * w, 3), dtype=np.int64)
    for dy in range(w):
        for dx in range(w):
            out[:, :, dy * w + dx, :] = pad[dy:dy + H, dx:dx + W, :]
    return out


def pair_cosines(v: np.ndarray) -> np.ndarray:
    """(n, n) cosines of a window's members with the documented conventions."""
    a = v[:, None, :]
    b = v[None, :, :]
    na = (a * a).sum(-1)
    nb = (b * b).sum(-1)
    cross = np.cross(a, b)
    collinear = (cross == 0).all(-1)
    dot = (a * b).sum(-1).astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        z = dot / (np.sqrt(na.astype(np.float64)) * np.sqrt(nb.astype(np.float64)))
    z = np.clip(z, -1.0, 1.0)
    z = np.where(collinear, 1.0, z)
    z = np.where((na == 0) ^ (nb == 0), 0.0, z)
    z = np.where((na == 0) & (nb == 0), 1.0, z)
    return z


def pair_angles_exact(v: np.ndarray) -> np.ndarray:
    """Exact angles via atan2 of the cross-product norm and the dot product."""
    a = v[:, None, :].astype(np.float64)
    b = v[None, :, :].astype(np.float64)
    cr = np.linalg.norm(np.cross(a, b), axis=-1)
    dot = (a * b).sum(-1)
    ang = np.arctan2(cr, dot)
    na = (v * v).sum(-1)
    zero_a = (na == 0)[:, None]
    zero_b = (na == 0)[None, :]
    ang = np.where(zero_a ^ zero_b, math.pi / 2, ang)
    ang = np.where(zero_a & zero_b, 0.0, ang)
    return ang


def _argmin_tie(S: np.ndarray) -> int:
    n = len(S)
    C = (n - 1) // 2
    m = S.min()
    if S[C] == m:
        return C
    return int(np.flatnonzero(S == m)[0])


def angle_matrix(v: np.ndarray, angle_fn) -> np.ndarray:
    if angle_fn is None:
        return pair_angles_exact(v)
    return angle_fn(pair_cosines(v))


def vdf(img, w, angle_fn=None):
    win = windows(img, w)
    H, W = img.shape[:2]
    out = np.empty_like(img)
    for y in range(H):
        for x in range(W):
            v = win[y, x]
            S = angle_matrix(v, angle_fn).sum(1)
            out[y, x] = v[_argmin_tie(S)]
    return out


def ddf(img, w, p=0.5, angle_fn=None):
    win = windows(img, w)
    H, W = img.shape[:2]
    out = np.empty_like(img)
    for y in range(H):
        for x in range(W):
            v = win[y, x]
            SA = angle_matrix(v, angle_fn).sum(1)
            d = v[:, None, :] - v[None, :, :]
            SD = np.sqrt((d * d).sum(-1).astype(np.float64)).sum(1)
            out[y, x] = v[_argmin_tie(SD ** (1 - p) * SA ** p)]
    return out


def amnfe(img, w, kappa=0.33, exp_fn=None, maxval=255, gauss=False):
    exp_fn = exp_fn or (lambda z: np.where(z > 10.0, 0.0, np.exp(-z)))
    win = windows(img, w)
    H, W = img.shape[:2]
    n = w * w
    C = (n - 1) // 2
    out = np.empty_like(img)
    for y in range(H):
        for x in range(W):
            v = win[y, x]
            L1 = np.abs(v[:, None, :] - v[None, :, :]).sum(-1)
            S1 = L1.sum(1)
            if (S1 == 0).any():
                out[y, x] = v[C]
                continue
            h = n ** (-kappa / 3.0) * S1.astype(np.float64)
            if gauss:
                # Gaussian kernel: half the squared Euclidean norm of (x_C - x_i) / h_i
                xs = (v[C][None, :] - v).astype(np.float64) / h[:, None]
                z = 0.5 * np.einsum("ik,ik->i", xs, xs)
            else:
                z = L1[C].astype(np.float64) / h
            wgt = exp_fn(z) / h ** 3
            if not wgt.sum() > 0:
                out[y, x] = v[C]
                continue
            mean = (wgt[:, None] * v).sum(0) / wgt.sum()
            out[y, x] = np.clip(np.floor(mean + 0.5), 0, maxval)
    return out


def evmf(img, w, ent_fn=None):
    def ent_exact(P):
        P = np.asarray(P, dtype=np.float64)
        with np.errstate(divide="ignore", invalid="ignore"):
            return np.where(P > 0, P * np.log(np.where(P > 0, P, 1.0)), 0.0)
    ent_fn = ent_fn or ent_exact
    win = windows(img, w)
    H, W = img.shape[:2]
    n = w * w
    C = (n - 1) // 2
    out = np.empty_like(img)
    for y in range(H):
        for x in range(W):
            v = win[y, x]
            xbar = v.mean(0)
            d = np.sqrt(((v - xbar) ** 2).sum(-1))
            D = d.sum()
            if D == 0:
                out[y, x] = v[C]
                continue
            P = d / D
            H_ = -ent_fn(P).sum()
            entC = ent_fn(P[C:C + 1])[0]
            if P[C] * H_ > -entC:
                dd = v[:, None, :] - v[None, :, :]
                S = np.sqrt((dd * dd).sum(-1).astype(np.float64)).sum(1)
                out[y, x] = v[_argmin_tie(S)]
            else:
                out[y, x] = v[C]
    return out
