"""Pins of the oracle's filters against facts the paper's equations fix:
closed forms, invariants, special cases that reduce to simpler filters, and a
second brute-force implementation (numpy twin) on tiny images and exhaustive
small palettes."""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import twin
from paper_1009_0959_amd import synth
from conftest import golden_table

WK = golden_table("worked_cases.txt")


def flat_with_impulse(w, v, q, pos=None):
    n = w * w
    win = np.tile(np.asarray(v, dtype=np.int64), (n, 1))
    win[(n - 1) // 2 if pos is None else pos] = q
    return win


# ------------------------------------------------------------------ VDF / DDF

@pytest.mark.parametrize("ap", ["exact", "paper", "split9"])
def test_vdf_uniform_and_impulse(ap):
    angle = {"exact": None, "paper": oracle.angle_approx("paper2", source="paper"),
             "split9": oracle.angle_approx("split", 9)}[ap]
    for w in (3, 5, 7):
        n = w * w
        idx, S = oracle.window_vdf(np.tile([40, 90, 200], (n, 1)), angle)
        assert idx == (n - 1) // 2
        # a non-collinear impulse at the centre is replaced by the flat value
        win = flat_with_impulse(w, [40, 90, 200], [250, 10, 30])
        idx, S = oracle.window_vdf(win, angle)
        assert idx != (n - 1) // 2 and tuple(win[idx]) == (40, 90, 200)


def test_vdf_two_colour_majority_closed_form():
    # k copies of a and n-k of b: S_a = (n-k) theta, S_b = k theta
    a, b = np.array([200, 30, 40]), np.array([20, 180, 60])
    theta = math.acos(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
    rng = np.random.default_rng(1)
    for n, k in [(9, 5), (9, 3), (25, 13), (49, 20)]:
        sel = np.zeros(n, dtype=bool)
        sel[rng.choice(n, k, replace=False)] = True
        win = np.where(sel[:, None], a, b)
        idx, S = oracle.window_vdf(win)
        assert np.allclose(S[sel], (n - k) * theta, rtol=1e-13)
        assert np.allclose(S[~sel], k * theta, rtol=1e-13)
        majority = a if k > n - k else b
        assert tuple(win[idx]) == tuple(majority)


def test_angle_acos_matches_atan2():
    rng = np.random.default_rng(2)
    for _ in range(3000):
        a = rng.integers(0, 256, 3)
        b = rng.integers(0, 256, 3)
        if not a.any() or not b.any():
            continue
        z = oracle.cosine(a, b)
        ang = math.atan2(np.linalg.norm(np.cross(a, b)), float(a @ b))
        # acos near z = 1 loses about 1e-16 / angle
        assert abs(math.acos(z) - ang) <= 1e-15 + 4e-16 / max(ang, 1e-8)


def test_cosine_conventions():
    assert oracle.cosine([0, 0, 0], [0, 0, 0]) == 1.0
    assert oracle.cosine([0, 0, 0], [3, 4, 5]) == 0.0
    assert oracle.cosine([3, 4, 5], [6, 8, 10]) == 1.0      # collinear -> exactly 1
    assert oracle.cosine([1, 1, 1], [3, 3, 3]) == 1.0
    assert oracle.cosine([255, 0, 0], [0, 255, 0]) == 0.0


def test_vdf_permutation_invariance():
    rng = np.random.default_rng(3)
    for w in (3, 5):
        n = w * w
        C = (n - 1) // 2
        for _ in range(200):
            win = rng.integers(0, 256, (n, 3))
            idx, S = oracle.window_vdf(win)
            srt = np.sort(S)
            if srt[1] - srt[0] < 1e-9:
                continue                      # unique minimiser only
            perm = np.concatenate([rng.permutation(np.delete(np.arange(n), C))])
            perm = np.insert(perm, C, C)
            idx2, _ = oracle.window_vdf(win[perm])
            assert tuple(win[perm][idx2]) == tuple(win[idx])


def test_ddf_limits_reduce_to_vdf_and_vmf():
    rng = np.random.default_rng(4)
    for _ in range(300):
        win = rng.integers(0, 256, (9, 3))
        i_vdf, _ = oracle.window_vdf(win)
        i1, SA, SD, Psi = oracle.window_ddf(win, p=1.0)
        assert i1 == i_vdf
        i0, SA, SD, Psi = oracle.window_ddf(win, p=0.0)
        # p = 0 is the vector median (sum of Euclidean distances)
        d = np.sqrt(((win[:, None, :] - win[None, :, :]) ** 2).sum(-1))
        assert np.allclose(SD, d.sum(1), rtol=1e-14)
        assert tuple(win[i0]) == tuple(win[np.argmin(d.sum(1))]) or \
            np.isclose(SD[i0], SD.min(), rtol=1e-13)
        ih, SA, SD, Psi = oracle.window_ddf(win, p=0.5)
        assert np.allclose(Psi, np.sqrt(SA * SD), rtol=1e-14)


@pytest.mark.parametrize("filt", ["vdf", "ddf", "evmf"])
def test_scale_invariance_u8_to_u16(filt):
    # angles are scale-free, and Euclidean sums scale uniformly: x -> 257 x
    # selects the same window member
    clean, noisy = synth.workload_image(0, height=16, width=16)
    a = oracle.run_filter(noisy, filt, 3)
    b = oracle.run_filter(noisy.astype(np.uint16) * 257, filt, 3)
    assert np.array_equal(a.astype(np.uint16) * 257, b)


# ------------------------------------------------------------------ AMNFE

def test_amnfe_impulse_closed_form():
    for w in (3, 5, 7):
        n = w * w
        kappa = 0.33
        r = (n - 1) ** -3.0 * math.exp(n ** (kappa / 3.0))
        v, q = np.array([100, 120, 90]), np.array([250, 5, 200])
        u, mean = oracle.window_amnfe(flat_with_impulse(w, v, q), kappa)
        assert u == 0
        expect = v + (q - v) * r / (r + n - 1)
        assert np.allclose(mean, expect, rtol=1e-13)
        if w == 3:
            assert abs(r - WK["AMNFE_WEIGHT_RATIO_N9"][0]) <= 5e-7
            assert abs(r / (r + 8) - WK["AMNFE_IMPULSE_SHIFT_N9"][0]) <= 5e-7
    # ... which rounds back to the flat value
    img = np.tile(np.array([100, 120, 90], dtype=np.uint8), (5, 5, 1))
    img[2, 2] = [250, 5, 200]
    assert tuple(oracle.run_filter(img, "amnfe", 3)[2, 2]) == (100, 120, 90)


def test_amnfe_uniform_and_scale():
    u, mean = oracle.window_amnfe(np.tile([7, 8, 9], (25, 1)))
    assert u == 1 and tuple(mean) == (7, 8, 9)
    rng = np.random.default_rng(5)
    for _ in range(200):
        win = rng.integers(0, 256, (25, 3))
        _, m8 = oracle.window_amnfe(win)
        _, m16 = oracle.window_amnfe(win * 257)
        assert np.allclose(m16, 257 * m8, rtol=1e-12)
        # the weighted mean is a convex combination of the members
        assert np.all(m8 >= win.min(0) - 1e-9) and np.all(m8 <= win.max(0) + 1e-9)


def test_amnfe_rational_close_to_exact():
    # the Table 3 rational is within 2.6e-6 of exp(-z), so each weight is
    # within ~1e-5 relative of the exact one (K >= exp(-n^(kappa/3)) > 0.2)
    # and the mean moves by at most ~2e-5 of the members' spread
    rng = np.random.default_rng(11)
    ex, ra = oracle.exp_approx("exact"), oracle.exp_approx("rational")
    for w in (3, 5, 7):
        for _ in range(50):
            win = rng.integers(0, 256, (w * w, 3))
            _, me = oracle.window_amnfe(win, expap=ex)
            _, mr = oracle.window_amnfe(win, expap=ra)
            assert np.all(np.abs(mr - me) <= 3e-5 * (win.max(0) - win.min(0)) + 1e-12)
            assert not np.array_equal(mr, me)


def test_amnfe_kernel_argument_bound():
    # z_i = |x_C - x_i|_1 / h_i <= n^(kappa/3): the T = 10 cutoff never fires
    rng = np.random.default_rng(6)
    for w in (3, 5, 7):
        n = w * w
        bound = n ** (0.33 / 3)
        for _ in range(100):
            win = rng.integers(0, 256, (n, 3))
            L1 = np.abs(win[:, None, :] - win[None, :, :]).sum(-1)
            h = n ** (-0.33 / 3) * L1.sum(1)
            z = L1[(n - 1) // 2] / h
            assert np.all(z <= bound * (1 + 1e-12))


# ------------------------------------------------------------------ AMNFG

def test_amnfg_impulse_closed_form():
    """Gaussian kernel (Section 3.2), flat window v with the impulse q at the
    centre: S1_C = (n-1) L, S1_j = L (L = |q - v|_1), so the centre's weight is
    h_C^-3 and every other member's h_j^-3 exp(-0.5 (E/L)^2 n^(2 kappa/3))
    (E = |q - v|_2): y = v + (q - v) r / (r + n - 1) with
    r = (n-1)^-3 exp(0.5 (E/L)^2 n^(2 kappa/3))."""
    for w in (3, 5, 7):
        n = w * w
        for q in ([250, 120, 90], [250, 5, 200], [100, 121, 91]):
            v, q = np.array([100, 120, 90]), np.array(q)
            L = np.abs(q - v).sum()
            E = math.sqrt(((q - v) ** 2).sum())
            r = (n - 1) ** -3.0 * math.exp(0.5 * (E / L) ** 2 * n ** (2 * 0.33 / 3.0))
            u, mean = oracle.window_amnfg(flat_with_impulse(w, v, q))
            assert u == 0
            assert np.allclose(mean, v + (q - v) * r / (r + n - 1), rtol=1e-13)
    # one-channel impulse at n = 9: E = L
    r = 8.0 ** -3 * math.exp(0.5 * 9 ** 0.22)
    assert abs(r - WK["AMNFG_WEIGHT_RATIO_N9"][0]) <= 5e-7
    assert abs(r / (r + 8) - WK["AMNFG_IMPULSE_SHIFT_N9"][0]) <= 5e-7


def test_amnfg_two_colour_closed_form():
    """k copies of a (the centre among them) and n - k of b: h_a = s (n-k) L,
    h_b = s k L (s = n^(-kappa/3), L = |a - b|_1), K_a = 1, K_b =
    exp(-0.5 |a - b|_2^2 / h_b^2); y = a + (b - a) (n-k) w_b / (k w_a + (n-k) w_b)."""
    rng = np.random.default_rng(13)
    for w in (3, 5, 7):
        n = w * w
        s = n ** (-0.33 / 3.0)
        for _ in range(20):
            a, b = rng.integers(0, 256, 3), rng.integers(0, 256, 3)
            if np.array_equal(a, b):
                continue
            k = int(rng.integers(1, n))
            win = np.tile(b, (n, 1))
            idx = rng.permutation([i for i in range(n) if i != (n - 1) // 2])[:k - 1]
            win[idx] = a
            win[(n - 1) // 2] = a
            L = np.abs(a - b).sum()
            E2 = float(((a - b) ** 2).sum())
            ha, hb = s * (n - k) * L, s * k * L
            wa, wb = ha ** -3, hb ** -3 * math.exp(-0.5 * E2 / hb ** 2)
            u, mean = oracle.window_amnfg(win)
            assert np.allclose(mean, a + (b - a) * (n - k) * wb / (k * wa + (n - k) * wb), rtol=1e-12, atol=1e-10)


def test_amnfg_uniform_scale_and_argument_bound():
    u, mean = oracle.window_amnfg(np.tile([7, 8, 9], (25, 1)))
    assert u == 1 and tuple(mean) == (7, 8, 9)
    rng = np.random.default_rng(8)
    for w in (3, 5, 7):
        n = w * w
        for _ in range(100):
            win = rng.integers(0, 256, (n, 3))
            _, m8 = oracle.window_amnfg(win)
            _, m16 = oracle.window_amnfg(win * 257)
            assert np.allclose(m16, 257 * m8, rtol=1e-12)
            assert np.all(m8 >= win.min(0) - 1e-9) and np.all(m8 <= win.max(0) + 1e-9)
            # and it is not the exponential-kernel filter
            _, me = oracle.window_amnfe(win)
            assert not np.allclose(me, m8, rtol=1e-9)
            # EXP argument 0.5 |x|_2^2 <= 0.5 n^(2 kappa/3) (= amnfg_range)
            L1 = np.abs(win[:, None, :] - win[None, :, :]).sum(-1)
            h = n ** (-0.33 / 3) * L1.sum(1)
            z = 0.5 * (((win[(n - 1) // 2] - win) / h[:, None]) ** 2).sum(-1)
            assert np.all(z <= oracle.amnfg_range(w) * (1 + 1e-12))


def test_exp_fit_range_stops_at_the_cutoff():
    """The minimax exp fit covers [0, min(argument bound, T)]: K is 0 above T."""
    assert oracle.exp_fit_range(5) == pytest.approx(25 ** 0.11)
    assert oracle.exp_fit_range(5, kernel="gauss") == pytest.approx(0.5 * 25 ** 0.22)
    assert oracle.exp_fit_range(7, kappa=4.0) == 10.0
    assert oracle.exp_fit_range(7, kappa=4.0, kernel="gauss") == 10.0


# ------------------------------------------------------------------ EVMF

def test_evmf_impulse_closed_form():
    win = flat_with_impulse(3, [60, 70, 80], [255, 0, 128])
    idx, info, S = oracle.window_evmf(win)
    PC, H, entC, switched = info
    assert abs(PC - WK["EVMF_IMPULSE_PC_N9"][0]) <= 1e-15
    assert abs(H - 2.5 * math.log(2)) <= 1e-14
    beta = -entC / H
    assert abs(beta - WK["EVMF_IMPULSE_BETA_N9"][0]) <= 1e-14
    assert switched == 1 and tuple(win[idx]) == (60, 70, 80)


def test_evmf_switch_equals_exp_minus_H():
    # P_C > beta_C  <=>  P_C > exp(-H)  (beta_C = -P_C ln P_C / H)
    rng = np.random.default_rng(7)
    for w in (3, 5):
        n = w * w
        for _ in range(500):
            win = rng.integers(0, 256, (n, 3))
            win[rng.random(n) < 0.6] = win[0]
            idx, info, S = oracle.window_evmf(win)
            PC, H, entC, sw = info
            assert PC <= 0.5 + 1e-15
            if H > 0 and abs(PC - math.exp(-H)) > 1e-12:
                assert bool(sw) == (PC > math.exp(-H))


def test_evmf_paper_cutoff_keeps_impulse_at_5x5():
    # the T = 0.05 cutoff zeroes P_j = 1/48 terms: beta_C becomes 1, impulse kept
    win = flat_with_impulse(5, [60, 70, 80], [255, 0, 128])
    idx, info, _ = oracle.window_evmf(win)
    assert info[3] == 1 and abs(-info[2] / info[1] - 0.1519) < 1e-4
    idx, info, _ = oracle.window_evmf(win, oracle.ent_approx("rational"))
    assert info[3] == 0 and idx == 12


def test_ent_cutoff_applies_to_every_kind():
    # Section 3.3: ENT(z) := 0 for z < T; the same rule for the exact function,
    # the Table 4 rational and the range-reduced fit
    kinds = [("exact", 0), ("rational", 0), ("rangered", 6)]
    for kind, deg in kinds:
        for T in (0.05, 0.2):
            en = oracle.ent_approx(kind, deg, cutoff=T)
            for z in (1e-9, 0.01, T * (1 - 1e-12)):
                assert oracle.eval_ent(en, z) == 0.0, (kind, T, z)
            for z in (T, 0.3, 0.9):
                if z >= T:
                    assert abs(oracle.eval_ent(en, z) - z * math.log(z)) < 1e-5, (kind, T, z)
    # T = 0: the plain function, and 0 only at 0
    en = oracle.ent_approx("exact", cutoff=0.0)
    assert oracle.eval_ent(en, 0.0) == 0.0
    assert oracle.eval_ent(en, 1e-300) == pytest.approx(1e-300 * math.log(1e-300), rel=1e-15)


@pytest.mark.parametrize("kind,deg", [("exact", 0), ("rangered", 6)])
def test_evmf_cutoff_one_is_the_identity(kind, deg):
    # T = 1 zeroes ENT below 1, and every P_j <= 1/2: H = 0 and ENT(P_C) = 0,
    # so P_C H > -ENT(P_C) never holds and every pixel keeps its value
    clean, noisy = synth.workload_image(2, height=19, width=23)
    out = oracle.run_filter(noisy, "evmf", 3, ent=oracle.ent_approx(kind, deg, cutoff=1.0))
    assert np.array_equal(out, noisy)
    # and T = 0 is the filter without cutoff
    a = oracle.run_filter(noisy, "evmf", 3, ent=oracle.ent_approx(kind, deg, cutoff=0.0))
    b = oracle.run_filter(noisy, "evmf", 3, ent=oracle.ent_approx(kind, deg))
    assert np.array_equal(a, b)


def test_evmf_cutoff_centre_below_t_switches():
    # a centre closer to the mean than T of the total deviation: without the
    # cutoff P_C < e^-H keeps the centre (H <= ln 9 < -ln T for n = 9); with
    # the cutoff ENT(P_C) = 0 and the window switches to the vector median
    win = np.array([[100, 100, 100]] * 4 + [[104, 100, 100]] + [[110, 100, 100]] * 4)
    idx, info, _ = oracle.window_evmf(win, oracle.ent_approx("exact"))
    assert info[0] < 0.05 and info[3] == 0 and idx == 4
    idx, info, _ = oracle.window_evmf(win, oracle.ent_approx("exact", cutoff=0.05))
    assert info[3] == 1


# ------------------------------------------------------------------ twin

@pytest.mark.parametrize("w", [3, 5])
def test_oracle_matches_twin_on_noisy_tiles(w):
    for cfg in (0, 1, 2):
        clean, noisy = synth.workload_image(cfg, height=13, width=11)
        sp = oracle.angle_approx("split", 7)
        fsp = lambda z, ap=sp: np.vectorize(lambda t: oracle.eval_angle(ap, t))(z)
        pairs = [
            (oracle.run_filter(noisy, "vdf", w), twin.vdf(noisy, w)),
            (oracle.run_filter(noisy, "vdf", w, angle=sp), twin.vdf(noisy, w, fsp)),
            (oracle.run_filter(noisy, "ddf", w), twin.ddf(noisy, w)),
            (oracle.run_filter(noisy, "amnfe", w), twin.amnfe(noisy, w)),
            (oracle.run_filter(noisy, "amnfg", w), twin.amnfe(noisy, w, gauss=True)),
            (oracle.run_filter(noisy, "amnfe", w, param=2.5), twin.amnfe(noisy, w, kappa=2.5)),
            (oracle.run_filter(noisy, "evmf", w), twin.evmf(noisy, w)),
        ]
        for a, b in pairs:
            assert np.array_equal(a, b)


def test_oracle_matches_twin_exhaustive_palette():
    # every 3x3 window over a 3-colour palette (3^9 windows), as one 1 x 19683
    # strip per window is too slow: use the window-level functions directly
    pal = np.array([[200, 40, 40], [40, 200, 40], [120, 120, 20]], dtype=np.int64)
    mismatch = 0
    for combo in itertools.product(range(3), repeat=9):
        v = pal[list(combo)]
        i_o, S = oracle.window_vdf(v)
        A = twin.pair_angles_exact(v)
        S2 = A.sum(1)
        assert np.allclose(S, S2, rtol=1e-12, atol=1e-12)
        # selections may differ only between (numerically) tied minimisers
        if tuple(v[i_o]) != tuple(v[twin._argmin_tie(S2)]):
            mismatch += 1
            assert S[i_o] <= S.min() + 1e-12
    assert mismatch <= 200
