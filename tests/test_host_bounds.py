"""Host-side checks of facts the kernels' FP32 decision bounds rely on (no GPU).

* The EVMF test windows whose P_j equals the Table 4 cutoff T = 0.05 exactly
  (Section 3.3) really do, and their switching decision depends on the side of T.
* The FP32 arithmetic of P_j = d_j / sum d (the EVMF finishers' order of
  operations, emulated in float32) stays within the band the kernels flag
  around T: (n + 4) u relative, with the kernels' band four times that.
"""
import numpy as np
import pytest

import oracle
from parity_util import CUT_WINDOWS

def test_cut_windows_are_exact():
    """(host) the listed multisets put P_j = 1/20 exactly and their centres'
    decisions depend on the side of T (exact rational arithmetic)."""
    from fractions import Fraction as F
    for w, (counts, centres) in CUT_WINDOWS.items():
        n = w * w
        assert sum(counts.values()) == n
        mean = F(sum(t * c for t, c in counts.items()), n)
        S = sum(c * abs(t - mean) for t, c in counts.items())
        P = {t: abs(t - mean) / S for t in counts}
        assert any(p == F(1, 20) for p in P.values())
        en = oracle.ent_approx("rational", round_f32=False)
        for c in centres:
            dec = []
            for at_T in (True, False):
                def ent(p):
                    if p == F(1, 20) and not at_T:
                        return 0.0
                    return oracle.eval_ent(en, float(p))
                H = -sum(cnt * ent(P[t]) for t, cnt in counts.items())
                dec.append(float(P[c]) * H > -ent(P[c]))
            assert dec[0] != dec[1], (w, c)


def _p_float32(win):
    """P_j of one window (n x 3 integer members) the way the FP32 finishers
    form it: a = n x_j - sum x (exact), d_j = sqrt(a.a) (rounded squares and
    sums), D = sum_j d_j in member order, P_j = d_j * (1 / D)."""
    f = np.float32
    n = win.shape[1]
    x = win.astype(np.float32)
    s = x.sum(axis=1, dtype=np.float64).astype(np.float32)           # exact integers
    a = (f(n) * x - s[:, None, :]).astype(np.float32)                  # exact integers
    sq = (a[..., 2] * a[..., 2]).astype(np.float32)
    sq = (a[..., 1] * a[..., 1] + sq).astype(np.float32)
    sq = (a[..., 0] * a[..., 0] + sq).astype(np.float32)
    d = np.sqrt(sq).astype(np.float32)
    D = np.zeros(win.shape[0], np.float32)
    for j in range(n):
        D = (D + d[:, j]).astype(np.float32)
    inv = (f(1.0) / D).astype(np.float32)
    return (d * inv[:, None]).astype(np.float32)


def _p_float64(win):
    x = win.astype(np.float64)
    mean = x.mean(axis=1, keepdims=True)
    d = np.sqrt(((x - mean) ** 2).sum(-1))
    return d / d.sum(axis=1, keepdims=True)


@pytest.mark.parametrize("w", [3, 5, 7])
@pytest.mark.parametrize("maxv", [255, 65535])
def test_evmf_p_within_cutoff_band(w, maxv):
    """The relative FP32 error of P_j stays within (n + 4) u (u = 2^-24, with
    a factor 2 to spare for the device square root's one ulp), so the kernels'
    band 4 (n + 4) u T around T covers every P_j that could lie on the other
    side of T in exact arithmetic."""
    from paper_1009_0959_amd import synth
    n = w * w
    u = 2.0 ** -24
    clean, img = synth.workload_image(2, height=120, width=160)
    img = img.astype(np.int64) * (257 if maxv == 65535 else 1)
    rng = np.random.default_rng([w, maxv])
    ys = rng.integers(0, img.shape[0] - w, 4000)
    xs = rng.integers(0, img.shape[1] - w, 4000)
    wins = np.stack([img[y:y + w, x:x + w].reshape(n, 3) for y, x in zip(ys, xs)])
    p32 = _p_float32(wins).astype(np.float64)
    p64 = _p_float64(wins)
    ok = p64 > 0
    rel = np.abs(p32[ok] - p64[ok]) / p64[ok]
    assert rel.max() <= 2.0 * (n + 4) * u, rel.max() / u
    # the flag band around T is 4 (n + 4) u T: twice the margin again
    assert 4 * (n + 4) * u * 0.05 >= 2.0 * rel.max() * 0.05
