"""FP64 oracle of the quality criteria (Section 4) and the exact-versus-
approximate statistics of Tables 5 and 6.

TEST INFRASTRUCTURE (see the package docstring): plain numpy in FP64, written
from the definitions, no blocking or reordering beyond numpy's own sums.

Criteria between an original image X and a filtered image Y of M x N RGB
pixels (Section 4, the three criteria):
  MAE = 1/(3MN) sum_rc |x(r,c) - y(r,c)|_1
  MSE = 1/(3MN) sum_rc |x(r,c) - y(r,c)|_2^2
  NCD = sum_rc |x^Lab(r,c) - y^Lab(r,c)|_2 / sum_rc |x^Lab(r,c)|_2
MAE and MSE are in the image's own units (0..255 or 0..65535).

Reading of the colour space (the paper cites its CIELAB source without the
convention): the RGB values are sRGB (IEC 61966-2-1) scaled to [0, 1] by the
type's maximum, decoded with the sRGB transfer function, taken to CIE XYZ by
the sRGB primaries' matrix (four-digit form), and to CIE 1976 L*a*b* relative
to the reference white that same matrix gives the RGB white (its row sums), so
that white is exactly (100, 0, 0). f(t) = t^(1/3) above (6/29)^3, else
t (29/6)^2 / 3 + 4/29. An all-black original (zero denominator) gives NCD 0
when Y equals it, else infinity.

Tables 5 and 6 (Section 4, the text around them): for every image, each
criterion of the exact filter and of the approximate one against the original;
the percentage 100 (E_exact - E_approx) / E_exact is negative where the
approximation is worse and positive where it is better; the time column is
100 T_exact / T_approx (the text's example: 1371% is 13.71 times faster). Each
cell is the mean and the standard deviation over the image set (reading: the
sample standard deviation, n - 1 in the denominator). An exact output equal to
the original (criterion 0) gives 0% when the approximate one is too, else
minus infinity.
"""
from __future__ import annotations

import numpy as np

# sRGB primaries to CIE XYZ (IEC 61966-2-1, four-digit form); rows X, Y, Z
SRGB_TO_XYZ = np.array([[0.4124, 0.3576, 0.1805],
                        [0.2126, 0.7152, 0.0722],
                        [0.0193, 0.1192, 0.9505]])
WHITE = SRGB_TO_XYZ.sum(axis=1)   # the RGB white through the same matrix
_EPS = (6.0 / 29.0) ** 3


def srgb_decode(c: np.ndarray) -> np.ndarray:
    """sRGB transfer function inverted: encoded c in [0, 1] -> linear."""
    c = np.asarray(c, dtype=np.float64)
    return np.where(c <= 0.04045, c / 12.92, ((c + 0.055) / 1.055) ** 2.4)


def _f(t: np.ndarray) -> np.ndarray:
    return np.where(t > _EPS, np.cbrt(t), t * (29.0 / 6.0) ** 2 / 3.0 + 4.0 / 29.0)


def to_lab(img: np.ndarray) -> np.ndarray:
    """(..., 3) uint8 / uint16 sRGB -> (..., 3) L*, a*, b* in FP64."""
    maxv = float(np.iinfo(img.dtype).max)
    lin = srgb_decode(img.astype(np.float64) / maxv)
    xyz = lin @ SRGB_TO_XYZ.T
    fx, fy, fz = (_f(xyz[..., k] / WHITE[k]) for k in range(3))
    return np.stack([116.0 * fy - 16.0, 500.0 * (fx - fy), 200.0 * (fy - fz)], axis=-1)


def sums(x: np.ndarray, y: np.ndarray) -> dict:
    """The criteria's sums: exact integer L1 and squared-L2 sums, and the two
    CIELAB sums of NCD in FP64."""
    if x.shape != y.shape or x.dtype != y.dtype or x.ndim != 3 or x.shape[2] != 3:
        raise ValueError("two RGB images of one shape and type")
    d = x.astype(np.int64) - y.astype(np.int64)
    lx, ly = to_lab(x), to_lab(y)
    return {"pixels": x.shape[0] * x.shape[1],
            "l1": int(np.abs(d).sum()), "l2sq": int((d * d).sum()),
            "lab_diff": float(np.sqrt(((lx - ly) ** 2).sum(-1)).sum()),
            "lab_ref": float(np.sqrt((lx ** 2).sum(-1)).sum())}


def criteria(x: np.ndarray, y: np.ndarray) -> dict:
    """MAE, MSE and NCD of the filtered image y against the original x."""
    s = sums(x, y)
    n3 = 3.0 * s["pixels"]
    if s["lab_ref"] > 0.0:
        ncd = s["lab_diff"] / s["lab_ref"]
    else:
        ncd = 0.0 if s["lab_diff"] == 0.0 else float("inf")
    return {"mae": s["l1"] / n3, "mse": s["l2sq"] / n3, "ncd": ncd}


def psnr(x: np.ndarray, y: np.ndarray) -> float:
    """PSNR in dB from the MSE above and the type's maximum."""
    mse = criteria(x, y)["mse"]
    maxv = float(np.iinfo(x.dtype).max)
    return float("inf") if mse == 0 else 10.0 * np.log10(maxv * maxv / mse)


def table_row(exact: list, approx: list, t_exact: list, t_approx: list) -> dict:
    """Mean and sample standard deviation over the image set of the
    exact-versus-approximate percentages (criteria dicts per image; times)."""
    out = {}
    for key in ("mae", "mse", "ncd"):
        e = np.array([m[key] for m in exact], dtype=np.float64)
        a = np.array([m[key] for m in approx], dtype=np.float64)
        with np.errstate(divide="ignore", invalid="ignore"):
            pct = np.where(e > 0, 100.0 * (e - a) / np.where(e > 0, e, 1.0), np.where(a > 0, -np.inf, 0.0))
        out[key] = (float(pct.mean()), float(pct.std(ddof=1)) if len(pct) > 1 else 0.0)
    r = 100.0 * np.asarray(t_exact, dtype=np.float64) / np.asarray(t_approx, dtype=np.float64)
    out["time"] = (float(r.mean()), float(r.std(ddof=1)) if len(r) > 1 else 0.0)
    return out
