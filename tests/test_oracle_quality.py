"""Pins of the quality-criteria oracle (Section 4: MAE, MSE, NCD; Tables 5-6
statistics) against facts that do not come from the oracle's own formulas:
published CIELAB coordinates of the sRGB primaries and secondaries, the grey
axis and white point, continuity of both piecewise functions, closed forms of
MAE/MSE for constant offsets, additivity over image parts, the 8/16-bit
scaling and a hand-computed statistics row."""
import numpy as np
import pytest

from oracle import quality as Q


def lab1(rgb, dtype=np.uint8):
    return Q.to_lab(np.array([[rgb]], dtype=dtype))[0, 0]


# published L*a*b* (D65) of the sRGB primaries and secondaries, to 2 decimals
PUBLISHED = [((255, 0, 0), (53.24, 80.09, 67.20)), ((0, 255, 0), (87.73, -86.18, 83.18)),
             ((0, 0, 255), (32.30, 79.19, -107.86)), ((255, 255, 0), (97.14, -21.55, 94.48)),
             ((0, 255, 255), (91.11, -48.09, -14.13)), ((255, 0, 255), (60.32, 98.23, -60.82))]


@pytest.mark.parametrize("rgb,want", PUBLISHED)
def test_lab_of_primaries_matches_published(rgb, want):
    # (the four-digit matrix and the white read from it move a*, b* by < 0.02)
    assert np.allclose(lab1(rgb), want, atol=0.03), (rgb, lab1(rgb))


def test_white_black_and_grey_axis():
    assert np.allclose(lab1((255, 255, 255)), (100.0, 0.0, 0.0), atol=1e-12)
    assert np.allclose(lab1((0, 0, 0)), (0.0, 0.0, 0.0), atol=1e-12)
    for v in (1, 7, 10, 11, 50, 119, 200, 254):
        L, a, b = lab1((v, v, v))
        assert abs(a) < 1e-12 and abs(b) < 1e-12, v
    # sRGB 119 is the usual mid grey, L* = 50.03
    assert abs(lab1((119, 119, 119))[0] - 50.03) < 0.01
    # L* increases along the grey axis
    Ls = [lab1((v, v, v))[0] for v in range(256)]
    assert np.all(np.diff(Ls) > 0)


def test_piecewise_functions_are_continuous():
    # sRGB decoding at its knee, and f at (6/29)^3
    lo = Q.srgb_decode(np.array([0.04045]))[0]
    hi = ((0.04045 + 0.055) / 1.055) ** 2.4
    assert abs(lo - hi) < 1e-7
    eps = (6.0 / 29.0) ** 3
    assert abs(Q._f(np.array([eps]))[0] - 6.0 / 29.0) < 1e-15
    assert abs(Q._f(np.array([eps * (1 + 1e-12)]))[0] - 6.0 / 29.0) < 1e-12


def test_mae_mse_closed_forms():
    rng = np.random.default_rng(5)
    x = rng.integers(10, 200, (17, 23, 3)).astype(np.uint8)
    for d in (1, 3, 40):
        y = x.copy()
        y[..., 1] += d                        # one channel, no clipping
        c = Q.criteria(x, y)
        assert c["mae"] == pytest.approx(d / 3.0, rel=1e-15)
        assert c["mse"] == pytest.approx(d * d / 3.0, rel=1e-15)
    c = Q.criteria(x, x)
    assert c == {"mae": 0.0, "mse": 0.0, "ncd": 0.0}
    # an all-black original
    z = np.zeros_like(x)
    assert Q.criteria(z, z)["ncd"] == 0.0
    assert Q.criteria(z, x)["ncd"] == float("inf")


def test_ncd_single_pixel_and_additivity():
    x = np.array([[[255, 0, 0]]], np.uint8)
    y = np.array([[[0, 0, 255]]], np.uint8)
    # one pixel: |Lab(x) - Lab(y)| / |Lab(x)| from the published coordinates
    r, b = np.array(PUBLISHED[0][1]), np.array(PUBLISHED[2][1])
    want = np.linalg.norm(r - b) / np.linalg.norm(r)
    assert Q.criteria(x, y)["ncd"] == pytest.approx(want, rel=2e-4)
    # the sums of an image are the sums of its halves
    rng = np.random.default_rng(8)
    a = rng.integers(0, 256, (30, 41, 3)).astype(np.uint8)
    c = rng.integers(0, 256, (30, 41, 3)).astype(np.uint8)
    s = Q.sums(a, c)
    s1, s2 = Q.sums(a[:13], c[:13]), Q.sums(a[13:], c[13:])
    for k in ("pixels", "l1", "l2sq"):
        assert s[k] == s1[k] + s2[k]
    for k in ("lab_diff", "lab_ref"):
        assert s[k] == pytest.approx(s1[k] + s2[k], rel=1e-13)


def test_sixteen_bit_scaling():
    rng = np.random.default_rng(2)
    a = rng.integers(0, 256, (9, 14, 3)).astype(np.uint8)
    c = rng.integers(0, 256, (9, 14, 3)).astype(np.uint8)
    c8 = Q.criteria(a, c)
    c16 = Q.criteria(a.astype(np.uint16) * 257, c.astype(np.uint16) * 257)
    assert c16["mae"] == pytest.approx(257 * c8["mae"], rel=1e-15)
    assert c16["mse"] == pytest.approx(257 * 257 * c8["mse"], rel=1e-15)
    assert c16["ncd"] == pytest.approx(c8["ncd"], rel=1e-14)


def test_table_row_by_hand():
    exact = [{"mae": 2.0, "mse": 10.0, "ncd": 0.5}, {"mae": 4.0, "mse": 10.0, "ncd": 0.25}]
    approx = [{"mae": 1.0, "mse": 11.0, "ncd": 0.5}, {"mae": 4.0, "mse": 9.0, "ncd": 0.5}]
    row = Q.table_row(exact, approx, [10.0, 20.0], [1.0, 4.0])
    # MAE: +50% (better), 0%; MSE: -10% (worse), +10%; NCD: 0%, -100%
    assert row["mae"] == pytest.approx((25.0, np.sqrt(2) * 25.0))
    assert row["mse"] == pytest.approx((0.0, np.sqrt(2) * 10.0))
    assert row["ncd"] == pytest.approx((-50.0, np.sqrt(2) * 50.0))
    # time: 10x and 5x faster -> 1000% and 500%
    assert row["time"] == pytest.approx((750.0, np.sqrt(2) * 250.0))
