"""Exact-versus-approximate comparison in the manner of Tables 5 and 6
(Section 4): every image of a set is filtered with the exact evaluation and
with an approximant; the criteria of both outputs against the original
(vf_quality: MAE, MSE, NCD) and both filter times give, per image, the
percentages 100 (E_exact - E_approx) / E_exact (negative: the approximation is
worse) and 100 T_exact / T_approx (the text's 1371% is 13.71 times faster);
each table cell is the mean and the sample standard deviation over the set.

Filtering and the criteria run in the library's kernels; this module only
times the calls (HIP events on the current stream) and averages.
"""
from __future__ import annotations

from typing import Optional, Sequence, Tuple

import numpy as np
import torch

from . import vf


def _timed_filter(filt: str, img: torch.Tensor, window: int, approx: vf.Approx, param: Optional[float],
                  out: torch.Tensor, repeats: int) -> float:
    """Median time (ms) of one filter call, re-check included."""
    vf.run(filt, img, window, approx, param, out=out)   # warm-up (tables, workspace)
    times = []
    for _ in range(repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        vf.run(filt, img, window, approx, param, out=out)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times))


def compare(pairs: Sequence[Tuple[torch.Tensor, torch.Tensor]], filt: str, window: int, approx: vf.Approx,
            param: Optional[float] = None, exact: Optional[vf.Approx] = None, repeats: int = 3) -> dict:
    """pairs: (original, noisy) GPU images. Returns the table row
    {"mae"|"mse"|"ncd"|"time": (mean, std)} and the per-image values."""
    exact = exact or vf.Approx("exact")
    per_image = []
    for clean, noisy in pairs:
        out_e = torch.empty_like(noisy)
        out_a = torch.empty_like(noisy)
        t_e = _timed_filter(filt, noisy, window, exact, param, out_e, repeats)
        t_a = _timed_filter(filt, noisy, window, approx, param, out_a, repeats)
        per_image.append({"exact": vf.quality(clean, out_e), "approx": vf.quality(clean, out_a),
                          "t_exact_ms": t_e, "t_approx_ms": t_a})
    row = {}
    n = len(per_image)
    for key in ("mae", "mse", "ncd"):
        e = np.array([r["exact"][key] for r in per_image])
        a = np.array([r["approx"][key] for r in per_image])
        with np.errstate(divide="ignore", invalid="ignore"):
            # an exact output equal to the original: 0% if the approximation's
            # is too, else an unbounded degradation
            pct = np.where(e > 0, 100.0 * (e - a) / np.where(e > 0, e, 1.0), np.where(a > 0, -np.inf, 0.0))
        row[key] = (float(pct.mean()), float(pct.std(ddof=1)) if n > 1 else 0.0)
    ratio = np.array([100.0 * r["t_exact_ms"] / r["t_approx_ms"] for r in per_image])
    row["time"] = (float(ratio.mean()), float(ratio.std(ddof=1)) if n > 1 else 0.0)
    return {"row": row, "images": per_image}
