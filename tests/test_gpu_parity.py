"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Selection filters (VDF, DDF, EVMF) output one of the window's input vectors;
AMNFE outputs a rounded weighted mean. The bar, from the method's target: at
least 99.9% of output pixels byte-identical to the oracle evaluating the same
approximant (the GPU re-checks near-tie windows in FP64, so in practice all of
them are), and every pixel valid: a selected vector is a member of the window
whose oracle criterion is within 1e-9 (relative) of the window's minimum, an
AMNFE channel differs by at most 1 where the oracle's mean lies within 1e-6 of a
rounding boundary.
"""
import math
import zlib

import numpy as np
import pytest

import oracle
from paper_1009_0959_amd import synth
from parity_util import check_valid, gpu_run, oracle_approx, sample_pixels

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1009_0959_amd import vf
    vf.lib()
    return vf


@pytest.fixture(scope="module")
def vf():
    return _need_gpu()


CASES = [
    ("vdf", 3, ("exact", 0)), ("vdf", 3, ("paper", 4)), ("vdf", 3, ("split", 3)),
    ("vdf", 3, ("split", 9)), ("vdf", 3, ("chord", 9)), ("vdf", 3, ("chord", 11)),
    ("vdf", 5, ("exact", 0)), ("vdf", 5, ("paper", 4)), ("vdf", 5, ("split", 7)),
    ("vdf", 5, ("chord", 11)), ("vdf", 7, ("chord", 11)), ("vdf", 7, ("exact", 0)),
    ("ddf", 3, ("exact", 0)), ("ddf", 3, ("split", 9)), ("ddf", 5, ("chord", 11)),
    ("ddf", 5, ("paper", 4)), ("ddf", 5, ("exact", 0)), ("ddf", 7, ("split", 5)),
    ("ddf", 7, ("chord", 11)), ("ddf", 7, ("exact", 0)),
    ("amnfe", 3, ("exact", 0)), ("amnfe", 3, ("paper", 4)), ("amnfe", 5, ("minimax", 6)),
    ("amnfe", 5, ("paper", 2)), ("amnfe", 7, ("minimax", 5)), ("amnfe", 3, ("rational", 4)),
    ("amnfe", 5, ("rational", 4)), ("amnfe", 7, ("rational", 0)),
    ("evmf", 3, ("exact", 0)), ("evmf", 3, ("paper", 4)), ("evmf", 5, ("minimax", 6)),
    ("evmf", 5, ("exact", 0)), ("evmf", 7, ("minimax", 7)),
    ("amnfg", 3, ("exact", 0)), ("amnfg", 3, ("minimax", 5)), ("amnfg", 5, ("minimax", 5)),
    ("amnfg", 5, ("paper", 3)), ("amnfg", 7, ("rational", 4)), ("amnfg", 7, ("exact", 0)),
    ("amnfe", 5, ("ratfit", 2)), ("amnfg", 3, ("ratfit", 2)), ("amnfe", 7, ("ratfit", 1)),
]


@pytest.mark.parametrize("filt,window,spec", CASES)
@pytest.mark.parametrize("config", [0, 1, 2])
@pytest.mark.parametrize("direct", [False, True])
def test_parity_small(vf, filt, window, spec, config, direct):
    # 37 x 131: two full 64-wide tiles plus a ragged column tail, ragged rows;
    # every filter runs both the streaming (pair-sharing) and the per-window kernels
    clean, img = synth.workload_image(config, height=37, width=131)
    ap = vf.Approx(*spec, direct=direct)
    got = gpu_run(vf, img, filt, window, ap)
    want = oracle.run_filter(img, filt, window, **oracle_approx(filt, ap, window))
    match = (got == want).all(-1).mean()
    assert match >= 0.999, match
    check_valid(img, filt, window, ap, None, got, want)


@pytest.mark.parametrize("window", [3, 5, 7])
@pytest.mark.parametrize("spec", [("exact", 0), ("minimax", 6), ("paper", 4)])
@pytest.mark.parametrize("cutoff", [0.05, 0.12])
@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
@pytest.mark.parametrize("direct", [False, True])
def test_evmf_cutoff_parity(vf, window, spec, cutoff, dtype, direct):
    """EVMF with the ENT cutoff T in every evaluation mode (Section 3.3)."""
    clean, img = synth.workload_image(2, height=37, width=131)
    img = img.astype(dtype) * (257 if dtype == np.uint16 else 1)
    ap = vf.Approx(*spec, direct=direct)
    got = gpu_run(vf, img, "evmf", window, ap, param=cutoff)
    want = oracle.run_filter(img, "evmf", window, **oracle_approx("evmf", ap, window, cutoff=cutoff))
    assert (got == want).all(-1).mean() >= 0.999
    check_valid(img, "evmf", window, ap, cutoff, got, want)


def test_evmf_cutoff_fp16_variant_and_validation(vf):
    clean, img = synth.workload_image(2, height=40, width=90)
    ap = vf.Approx("minimax", 6, precision="fp16x2")
    got = gpu_run(vf, img, "evmf", 5, ap, param=0.05)
    want = oracle.run_filter(img, "evmf", 5, **oracle_approx("evmf", ap, 5, cutoff=0.05))
    assert np.array_equal(got, want)
    t = torch.from_numpy(img).cuda()
    with pytest.raises(vf.VfError) as e:
        vf.filter_log(t, 3, vf.Approx("paper", 4), cutoff=0.01)   # the rational holds on [0.05, 1]
    assert e.value.status == vf.VF_EDOMAIN
    for bad in (-0.1, 1.5, float("nan")):
        with pytest.raises(vf.VfError) as e:
            vf.filter_log(t, 3, vf.Approx("exact"), cutoff=bad)
        assert e.value.status == vf.VF_EINVAL


def near_cutoff_windows(T, count, tol=1e-7, seed=123):
    """3x3 integer windows (row-major, 9 x 3) whose FP64 P_j = |x_j - mean| /
    sum_i |x_i - mean| lies within tol of T for some member, found by a seeded
    search (mostly flat windows, so that the deviations are small integers)."""
    rng = np.random.default_rng(seed)
    found = []
    for _ in range(200):
        base = rng.integers(20, 230, (100000, 1, 3))
        win = base + rng.integers(-6, 7, (100000, 9, 3)) * (rng.random((100000, 9, 1)) < 0.7)
        win = np.clip(win, 0, 255)
        dev = np.sqrt(((win - win.mean(1, keepdims=True)) ** 2).sum(-1))
        D = dev.sum(1, keepdims=True)
        with np.errstate(invalid="ignore", divide="ignore"):
            P = dev / D
        hit = np.flatnonzero((np.abs(P - T) < tol).any(1) & (D[:, 0] > 0))
        found.extend(win[hit])
        if len(found) >= count:
            break
    return found[:count]


@pytest.mark.parametrize("spec", [("exact", 0), ("minimax", 6), ("paper", 4)])
@pytest.mark.parametrize("direct", [False, True])
def test_evmf_near_cutoff_windows_are_decided_in_fp64(vf, spec, direct):
    """A P_j within the FP32 error band of T is flagged and decided in FP64:
    3x3 images that are exactly such a window (the centre pixel's window)."""
    wins = near_cutoff_windows(0.05, 6)
    assert len(wins) >= 3
    ap = vf.Approx(*spec, direct=direct)
    for win in wins:
        img = win.reshape(3, 3, 3).astype(np.uint8)
        got = gpu_run(vf, img, "evmf", 3, ap, param=0.05)
        assert vf.get_stats()["flagged"] >= 1, win.tolist()
        want = oracle.run_filter(img, "evmf", 3, **oracle_approx("evmf", ap, 3, cutoff=0.05))
        assert np.array_equal(got[1, 1], want[1, 1]), (win.tolist(), got[1, 1], want[1, 1])


def palette_image(shape, seed, dtype=np.uint8):
    """Three colours a unit apart (A - B = (1, -1, 0), A - C = (1, 0, 0)) at
    random, with 3% impulses (zeros among them): windows full of exact ties
    between distinct vectors (equal multisets of pair values), next to pixels
    whose pair values are hundreds of times larger."""
    rng = np.random.default_rng(seed)
    pal = np.array([[203, 179, 157], [202, 180, 157], [202, 179, 157]])
    img = pal[rng.choice(3, size=shape, p=[0.45, 0.45, 0.1])]
    imp = rng.random(shape) < 0.03
    img[imp] = rng.integers(0, 256, (int(imp.sum()), 3))
    img[imp & (rng.random(shape) < 0.3)] = 0
    img = img.astype(np.uint8)
    return img.astype(dtype) * (257 if dtype == np.uint16 else 1)


@pytest.mark.parametrize("filt,window,spec", [
    ("vdf", 3, ("chord", 11)), ("vdf", 5, ("chord", 11)), ("vdf", 7, ("chord", 11)),
    ("ddf", 3, ("chord", 11)), ("ddf", 5, ("chord", 9)), ("ddf", 7, ("split", 9)), ("ddf", 7, ("chord", 11)),
    ("evmf", 3, ("minimax", 6)), ("evmf", 5, ("minimax", 6)), ("evmf", 7, ("minimax", 7))])
@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
@pytest.mark.parametrize("direct", [False, True])
def test_tie_rule_exact_on_palette_images(vf, filt, window, spec, dtype, direct):
    """Where distinct vectors tie exactly, the oracle keeps the centre, else the
    lowest index: every pixel must equal the oracle's (no tolerance). Small
    images run in strips of a few rows, so most windows sit near a strip's
    first row, whose state starts from padding rows."""
    img = palette_image((40, 150), zlib.crc32(repr((filt, window, dtype)).encode()), dtype)
    ap = vf.Approx(*spec, direct=direct)
    got = gpu_run(vf, img, filt, window, ap)
    want = oracle.run_filter(img, filt, window, **oracle_approx(filt, ap, window))
    bad = np.argwhere((got != want).any(-1))
    assert len(bad) == 0, (len(bad), bad[:5].tolist(), got[tuple(bad[0])].tolist(), want[tuple(bad[0])].tolist())


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (9, 1), (2, 2), (3, 70), (65, 5), (130, 61),
                                   (200, 3), (70, 125)])
@pytest.mark.parametrize("filt,window,spec", [("vdf", 5, ("chord", 11)), ("ddf", 3, ("exact", 0)),
                                              ("amnfe", 7, ("minimax", 6)), ("evmf", 5, ("paper", 4)),
                                              ("vdf", 7, ("split", 9)), ("vdf", 3, ("exact", 0)),
                                              ("ddf", 5, ("chord", 9))])
def test_parity_edge_shapes(vf, dtype, shape, filt, window, spec):
    rng = np.random.default_rng(zlib.crc32(repr((shape, filt)).encode()))
    maxv = np.iinfo(dtype).max
    img = rng.integers(0, maxv + 1, size=shape + (3,)).astype(dtype)
    ap = vf.Approx(*spec)
    got = gpu_run(vf, img, filt, window, ap)
    want = oracle.run_filter(img, filt, window, **oracle_approx(filt, ap, window))
    assert (got == want).all(-1).mean() >= 0.999 or got.shape[0] * got.shape[1] < 1000
    check_valid(img, filt, window, ap, None, got, want)


@pytest.mark.parametrize("shape", [(1, 70001), (70001, 1), (3, 40000), (40000, 2), (2, 2)])
@pytest.mark.parametrize("filt,window,spec", [("vdf", 5, ("chord", 11)), ("ddf", 7, ("chord", 11)),
                                              ("amnfe", 3, ("minimax", 6)), ("evmf", 7, ("minimax", 7)),
                                              ("vdf", 7, ("exact", 0)), ("amnfg", 5, ("minimax", 5))])
def test_extreme_aspect_ratios(vf, shape, filt, window, spec):
    """Single rows and columns tens of thousands of pixels long (strip sizing,
    tile numbering and replicated borders at both ends), streaming and
    per-window kernels, u8."""
    rng = np.random.default_rng(zlib.crc32(repr((shape, filt, window)).encode()))
    img = rng.integers(0, 256, size=shape + (3,)).astype(np.uint8)
    img[rng.random(shape) < 0.5] = img.reshape(-1, 3)[0]    # repeated vectors: ties
    want = oracle.run_filter(img, filt, window, **oracle_approx(filt, vf.Approx(*spec), window))
    for direct in (False, True):
        ap = vf.Approx(*spec, direct=direct)
        got = gpu_run(vf, img, filt, window, ap)
        assert (got == want).all(-1).mean() >= 0.999, direct
        check_valid(img, filt, window, ap, None, got, want)


@pytest.mark.parametrize("filt", ["vdf", "ddf", "amnfe", "evmf"])
def test_degenerate_images(vf, filt):
    # uniform image, zero vectors, collinear greys, two-colour checkerboard
    imgs = [np.full((20, 70, 3), 77, np.uint8), np.zeros((20, 70, 3), np.uint8)]
    g = np.arange(20 * 70).reshape(20, 70) % 7 * 30
    imgs.append(np.stack([g, g, g], -1).astype(np.uint8))
    cb = (np.indices((20, 70)).sum(0) % 2)[..., None] * np.array([200, 30, 40]) + \
        (1 - np.indices((20, 70)).sum(0) % 2)[..., None] * np.array([10, 150, 90])
    imgs.append(cb.astype(np.uint8))
    z = np.random.default_rng(1).integers(0, 256, (20, 70, 3)).astype(np.uint8)
    z[::3, ::4] = 0
    imgs.append(z)
    for img in imgs:
        for window in (3, 5):
            ap = vf.Approx("exact") if filt != "vdf" else vf.Approx("chord", 11)
            got = gpu_run(vf, img, filt, window, ap)
            want = oracle.run_filter(img, filt, window, **oracle_approx(filt, ap, window))
            check_valid(img, filt, window, ap, None, got, want)
            assert (got == want).all(-1).mean() >= 0.999


def test_uint16_matches_scaled_uint8(vf):
    clean, img = synth.workload_image(0, height=40, width=100)
    for filt in ("vdf", "ddf", "evmf"):
        a = gpu_run(vf, img, filt, 5, vf.Approx("exact"))
        b = gpu_run(vf, img.astype(np.uint16) * 257, filt, 5, vf.Approx("exact"))
        assert np.array_equal(a.astype(np.uint16) * 257, b)


def test_pitched_tensors(vf):
    clean, img = synth.workload_image(1, height=50, width=90)
    big = torch.zeros((50, 128, 3), dtype=torch.uint8, device="cuda")
    big[:, :90] = torch.from_numpy(img).cuda()
    src = big[:, :90]
    dst_big = torch.zeros((50, 100, 3), dtype=torch.uint8, device="cuda")
    dst = dst_big[:, :90]
    vf.filter_vdf(src, 3, vf.Approx("chord", 11), out=dst)
    torch.cuda.synchronize()
    want = oracle.run_filter(img, "vdf", 3, angle=oracle.angle_approx("chord", 11))
    assert np.array_equal(dst.cpu().numpy(), want)
    assert int(dst_big[:, 90:].abs().sum()) == 0      # padding untouched


def test_deterministic(vf):
    clean, img = synth.workload_image(1, height=300, width=300)
    t = torch.from_numpy(img).cuda()
    for filt, ap in [("vdf", vf.Approx("chord", 9)), ("evmf", vf.Approx("minimax", 6)),
                     ("amnfe", vf.Approx("minimax", 6))]:
        a = vf.run(filt, t, 5, ap)
        b = vf.run(filt, t, 5, ap)
        torch.cuda.synchronize()
        assert torch.equal(a, b)


def test_invalid_arguments_raise_without_writing(vf):
    img = torch.zeros((8, 8, 3), dtype=torch.uint8, device="cuda")
    out = torch.full_like(img, 5)
    with pytest.raises(vf.VfError):
        vf.filter_vdf(img, 9, vf.Approx("exact"), out=out)
    with pytest.raises(vf.VfError):
        vf.filter_vdf(img, 3, vf.Approx("split", 4), out=out)
    with pytest.raises(vf.VfError):
        vf.filter_ddf(img, 3, 2.0, vf.Approx("exact"), out=out)
    with pytest.raises(vf.VfError):   # overlapping src / dst
        vf.filter_vdf(img, 3, vf.Approx("exact"), out=img)
    torch.cuda.synchronize()
    assert int((out != 5).sum()) == 0


@pytest.mark.parametrize("spec", [("paper", 4), ("split", 3), ("split", 5), ("split", 7), ("split", 9),
                                  ("chord", 7), ("chord", 9), ("chord", 11), ("chord", 13),
                                  ("exact", 0)])
def test_angle_function_error(vf, spec):
    """FP32 evaluation vs FP64 evaluation of the same constants from the same
    (FP32) squared chord: within the evaluation part of the kernels' per-pair
    bound (relative 9.5e-7 for the polynomial, 2^-23 for the square root), and
    vs arccos within eps + 5e-7."""
    ap = vf.Approx(*spec)
    z = np.concatenate([np.linspace(0.0, 1.0, 400001), 1 - np.logspace(-12, -1, 20001)])
    s2 = np.clip(2.0 * (1.0 - z), 0.0, 2.0).astype(np.float32)
    got = vf.eval_function("vdf", torch.from_numpy(s2).cuda(), ap).cpu().numpy().astype(np.float64)
    zz = 1.0 - s2.astype(np.float64) / 2.0
    oap = oracle_approx("vdf", ap, 3)["angle"]
    ref = np.array([oracle.eval_angle(oap, v) for v in zz[::7]])
    err_same = np.max(np.abs(got[::7] - ref))
    if spec[0] == "exact":
        # acosf of a cosine rounded to FP32: about 2^-25 / sin(angle) away from
        # z = 1 and up to sqrt(2^-24) where z rounds to 1; the kernels' flag bound
        # per pair is 2^-23 / sqrt(s^2 + 2^-24) + 6e-7 (0 for s^2 = 0)
        s2d = s2[::7].astype(np.float64)
        bound = np.where(s2d > 0, 2.0 ** -23 / np.sqrt(s2d + 2.0 ** -24) + 6e-7, 0.0) + 1e-30
        ratio = np.abs(got[::7] - ref) / bound
        assert ratio.max() <= 1.0, (ratio.max(), zz[::7][ratio.argmax()], got[::7][ratio.argmax()])
    else:
        assert err_same <= 4e-7, err_same
        rel = np.abs(got[::7] - ref) / (1e-8 + 1.1e-6 * np.abs(ref))
        assert rel.max() <= 1.0, (rel.max(), zz[::7][rel.argmax()])
        assert np.max(np.abs(got[::7] - np.arccos(zz[::7]))) <= oap.eps + 5e-7


def test_exp_ent_function_error(vf):
    for w in (3, 5, 7):
        for d in (4, 6):
            ap = vf.Approx("minimax", d)
            z = np.linspace(0, oracle.amnfe_range(w), 100001).astype(np.float32)
            got = vf.eval_function("amnfe", torch.from_numpy(z).cuda(), ap, window=w).cpu().numpy()
            ep = oracle.exp_approx("poly", d, window=w)
            ref = np.array([oracle.eval_expneg(ep, v) for v in z[::11].astype(np.float64)])
            assert np.max(np.abs(got[::11] - ref)) <= 4e-7
    # the Table 3 rational, over its whole interval and past the T = 10 cutoff
    z = np.linspace(0, 10.5, 100001).astype(np.float32)
    got = vf.eval_function("amnfe", torch.from_numpy(z).cuda(), vf.Approx("rational", 4), window=5).cpu().numpy()
    ex = oracle.exp_approx("rational")
    ref = np.array([oracle.eval_expneg(ex, v) for v in z[::7].astype(np.float64)])
    assert np.max(np.abs(got[::7] - ref)) <= 4e-7
    assert np.all(got[z > 10.0] == 0.0)
    # fitted R^d_d rationals over the range each kernel reaches
    for filt, kernel, w, d in (("amnfe", "exp", 5, 2), ("amnfg", "gauss", 7, 2), ("amnfe", "exp", 3, 1)):
        ex = oracle.exp_approx("ratfit", d, window=w, kernel=kernel)
        b = oracle.exp_fit_range(w, kernel=kernel)
        z = np.linspace(0, b, 100001).astype(np.float32)
        got = vf.eval_function(filt, torch.from_numpy(z).cuda(), vf.Approx("ratfit", d), window=w).cpu().numpy()
        ref = np.array([oracle.eval_expneg(ex, v) for v in z[::7].astype(np.float64)])
        assert np.max(np.abs(got[::7] - ref)) <= 4e-7
        assert np.max(np.abs(ref - np.exp(-z[::7].astype(np.float64)))) <= ex.eps * 1.01 + 1e-7
    P = np.concatenate([np.logspace(-8, 0, 50001), np.linspace(0, 0.5, 50001)]).astype(np.float32)
    for spec, en in [(("minimax", 6), oracle.ent_approx("rangered", 6)),
                     (("paper", 4), oracle.ent_approx("rational")), (("exact", 0), oracle.ent_approx("exact"))]:
        got = vf.eval_function("evmf", torch.from_numpy(P).cuda(), vf.Approx(*spec)).cpu().numpy()
        ref = np.array([oracle.eval_ent(en, v) for v in P[::9].astype(np.float64)])
        assert np.max(np.abs(got[::9] - ref)) <= 2e-6


# ---------------------------------------------------------------- full size

@pytest.mark.parametrize("filt,window,spec,config", [
    ("vdf", 3, ("chord", 11), 1), ("vdf", 5, ("chord", 11), 1), ("vdf", 3, ("exact", 0), 1),
    ("ddf", 5, ("split", 9), 1), ("vdf", 5, ("split", 7), 1), ("vdf", 7, ("chord", 11), 1),
    ("ddf", 5, ("chord", 11), 1), ("amnfe", 5, ("minimax", 6), 2), ("evmf", 5, ("minimax", 6), 2),
    ("amnfe", 5, ("rational", 4), 2), ("evmf", 5, ("paper", 4), 2), ("amnfg", 5, ("minimax", 5), 2),
    ("amnfe", 5, ("ratfit", 2), 2), ("amnfg", 7, ("ratfit", 2), 2), ("evmf", 7, ("minimax", 7), 2)])
def test_parity_full_size_sampled(vf, filt, window, spec, config):
    """4096 x 4096 workloads (headline; mixed noise for AMNFE / EVMF), in the
    launch configuration the benchmark times, checked on sampled pixels (all
    borders and corners included)."""
    clean, img = synth.workload_image(config)
    ap = vf.Approx(*spec)
    got = gpu_run(vf, img, filt, window, ap)
    pix = sample_pixels(*img.shape[:2], 6000, 11)
    want = oracle.run_filter(img, filt, window, pixels=pix, **oracle_approx(filt, ap, window))
    g = got[pix[:, 0], pix[:, 1]]
    assert (g == want).all(-1).mean() >= 0.999
    check_valid(img, filt, window, ap, None, g, want, pixels=pix)
    if filt in ("amnfe", "amnfg"):
        return   # a weighted mean, not a member
    # whole-image property at any size: every output is a member of its window
    H, W = img.shape[:2]
    pad = np.pad(img, ((window // 2,) * 2, (window // 2,) * 2, (0, 0)), mode="edge")
    member = np.zeros((H, W), bool)
    for dy in range(window):
        for dx in range(window):
            member |= (pad[dy:dy + H, dx:dx + W] == got).all(-1)
    assert member.all()


@pytest.mark.parametrize("filt,window,spec,extra,config", [
    ("vdf", 5, ("chord", 11), dict(precision="fp16x2"), 1), ("vdf", 3, ("chord", 9), dict(precision="fp16x2"), 1),
    ("ddf", 5, ("chord", 11), dict(precision="fp16x2"), 1), ("vdf", 5, ("chord", 11), dict(scheme="estrin"), 1),
    ("amnfe", 5, ("minimax", 6), dict(precision="fp16x2"), 2), ("evmf", 5, ("minimax", 6), dict(precision="fp16x2"), 2),
    ("amnfg", 5, ("minimax", 5), dict(precision="fp16x2"), 2)])
def test_variants_full_size_sampled(vf, filt, window, spec, extra, config):
    """The evaluation variants (packed FP16 corrections, Estrin's scheme) on
    the full 4096 x 4096 workloads, checked on sampled pixels with borders."""
    clean, img = synth.workload_image(config)
    ap = vf.Approx(*spec, **extra)
    got = gpu_run(vf, img, filt, window, ap)
    pix = sample_pixels(*img.shape[:2], 4000, 17)
    want = oracle.run_filter(img, filt, window, pixels=pix, **oracle_approx(filt, ap, window))
    g = got[pix[:, 0], pix[:, 1]]
    assert (g == want).all(-1).mean() >= 0.999
    check_valid(img, filt, window, ap, None, g, want, pixels=pix)


@pytest.mark.parametrize("filt", ["amnfe", "amnfg"])
@pytest.mark.parametrize("window", [3, 5, 7])
@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
@pytest.mark.parametrize("spec", [("minimax", 6), ("exact", 0), ("rational", 4), ("ratfit", 2)])
def test_amnfe_streaming_equals_per_window(vf, filt, window, dtype, spec):
    """The streaming AMNF kernels form the same exact integer L1 sums and then
    the same FP32 weights as the per-window kernels (both kernel functions):
    outputs agree bit for bit (before any re-check, which is switched off here)."""
    if filt == "amnfg" and spec == ("minimax", 6):
        spec = ("minimax", 5)      # (degree 6 is below FP32 resolution on the Gaussian range)
    clean, img = synth.workload_image(2, height=150, width=190)
    img = img.astype(dtype) * (257 if dtype == np.uint16 else 1)
    a = gpu_run(vf, img, filt, window, vf.Approx(*spec, recheck=False))
    b = gpu_run(vf, img, filt, window, vf.Approx(*spec, recheck=False, direct=True))
    assert np.array_equal(a, b)


@pytest.mark.parametrize("filt", ["amnfe", "amnfg"])
@pytest.mark.parametrize("window", [3, 7])
@pytest.mark.parametrize("spec", [("exact", 0), ("paper", 4), ("minimax", 6), ("rational", 4), ("ratfit", 3)])
@pytest.mark.parametrize("direct", [False, True])
def test_amnf_large_kappa_reaches_the_cutoff(vf, filt, window, spec, direct):
    """kappa = 4: the EXP argument reaches past the cutoff T = 10 (n^(4/3) =
    18.7 at 3x3), where K jumps from about e^-10 to 0; members whose FP32
    argument lies within its error of T are decided in FP64, so the outputs
    match the oracle's."""
    clean, img = synth.workload_image(2, height=60, width=131)
    ap = vf.Approx(*spec, direct=direct)
    got = gpu_run(vf, img, filt, window, ap, 4.0)
    want = oracle.run_filter(img, filt, window, param=4.0, **oracle_approx(filt, ap, window, kappa=4.0))
    assert (got == want).all(-1).mean() >= 0.999
    check_valid(img, filt, window, ap, 4.0, got, want)


def test_fuzzy_exp_rejects_unknown_kernel(vf):
    img = torch.zeros((8, 8, 3), dtype=torch.uint8, device="cuda")
    out = torch.full_like(img, 5)
    im, a = vf._image(img, out), vf.Approx("exact").struct()
    import ctypes as C
    st = vf.lib().vf_filter_fuzzy_exp(vf.context(0), C.byref(im), 3, 0.33, 2, C.byref(a), vf._stream())
    assert st == vf.VF_EINVAL
    torch.cuda.synchronize()
    assert int((out != 5).sum()) == 0


@pytest.mark.parametrize("filt,window,spec", [("evmf", 3, ("minimax", 6)), ("evmf", 5, ("exact", 0)),
                                              ("evmf", 7, ("paper", 4)), ("ddf", 5, ("chord", 11)),
                                              ("vdf", 7, ("chord", 11)), ("ddf", 7, ("chord", 11)),
                                              ("vdf", 7, ("exact", 0)), ("ddf", 7, ("exact", 0)),
                                              ("ddf", 7, ("split", 9)), ("ddf", 7, ("paper", 4)),
                                              ("vdf", 5, ("exact", 0))])
def test_streaming_equals_per_window_after_recheck(vf, filt, window, spec):
    """Streaming and per-window kernels sum in different orders; after the FP64
    re-check of near ties both give the oracle's decision everywhere."""
    clean, img = synth.workload_image(2, height=150, width=190)
    a = gpu_run(vf, img, filt, window, vf.Approx(*spec))
    b = gpu_run(vf, img, filt, window, vf.Approx(*spec, direct=True))
    assert (a == b).all(-1).mean() >= 0.999
    want = oracle.run_filter(img, filt, window, **oracle_approx(filt, vf.Approx(*spec), window))
    check_valid(img, filt, window, vf.Approx(*spec), None, a, want)


@pytest.mark.parametrize("shape", [(70, 133), (9, 300), (130, 61)])
@pytest.mark.parametrize("p", [0.5, 0.25])
def test_ddf7_parity_u16(vf, shape, p):
    """7x7 DDF with the chord approximant (one-pass selection): 16-bit images,
    ragged shapes, both criterion forms, against the oracle."""
    clean, img = synth.workload_image(4, height=shape[0], width=shape[1])
    ap = vf.Approx("chord", 11)
    got = gpu_run(vf, img, "ddf", 7, ap, p)
    want = oracle.run_filter(img, "ddf", 7, param=p, **oracle_approx("ddf", ap, 7))
    assert (got == want).all(-1).mean() >= 0.999
    check_valid(img, "ddf", 7, ap, p, got, want)


def test_deferred_recheck_matches(vf):
    clean, img = synth.workload_image(1, height=300, width=257)
    t = torch.from_numpy(img).cuda()
    for filt, ap in [("vdf", ("chord", 11)), ("vdf", ("exact", 0)), ("ddf", ("split", 9)),
                     ("amnfe", ("minimax", 6)), ("evmf", ("minimax", 6))]:
        a = vf.run(filt, t, 5, vf.Approx(*ap))
        b = vf.run(filt, t, 5, vf.Approx(*ap, defer=True))
        vf.recheck_pending()
        vf.recheck_pending()     # nothing pending: no-op
        torch.cuda.synchronize()
        assert torch.equal(a, b)
    # without the deferred re-check the near-tie windows keep their FP32 choice
    st_before = vf.get_stats()
    assert st_before["windows"] == 300 * 257


# ---------------------------------------------------------------- evaluation variants

VARIANT_CASES = [("vdf", 3, 11), ("vdf", 5, 11), ("vdf", 5, 7), ("ddf", 3, 9), ("ddf", 5, 11),
                 ("vdf", 7, 13)]


@pytest.mark.parametrize("filt,window,degree", VARIANT_CASES)
@pytest.mark.parametrize("variant", [dict(scheme="estrin"), dict(precision="fp16x2")])
@pytest.mark.parametrize("config", [0, 1])
def test_parity_variants(vf, filt, window, degree, variant, config):
    """Estrin's scheme and the packed-FP16 correction term against the oracle
    evaluating the same polynomial (for FP16: the coefficients after the first
    rounded to half precision) in FP64."""
    clean, img = synth.workload_image(config, height=37, width=131)
    ap = vf.Approx("chord", degree, **variant)
    got = gpu_run(vf, img, filt, window, ap)
    want = oracle.run_filter(img, filt, window, **oracle_approx(filt, ap, window))
    assert (got == want).all(-1).mean() >= 0.999
    check_valid(img, filt, window, ap, None, got, want)


FE_F16_CASES = [("amnfe", 3, 6), ("amnfe", 5, 6), ("amnfe", 7, 5), ("evmf", 3, 6), ("evmf", 5, 6),
                ("evmf", 7, 7), ("amnfg", 5, 5), ("amnfg", 7, 4)]


@pytest.mark.parametrize("filt,window,degree", FE_F16_CASES)
@pytest.mark.parametrize("config", [0, 1, 2])
def test_parity_fe_f16(vf, filt, window, degree, config):
    """AMNFE / EVMF with the packed-FP16 exp / ln1p correction against the
    oracle evaluating the same polynomial (c_1.. rounded to half precision) in
    FP64."""
    clean, img = synth.workload_image(config, height=37, width=131)
    ap = vf.Approx("minimax", degree, precision="fp16x2")
    got = gpu_run(vf, img, filt, window, ap)
    want = oracle.run_filter(img, filt, window, **oracle_approx(filt, ap, window))
    assert (got == want).all(-1).mean() >= 0.999
    check_valid(img, filt, window, ap, None, got, want)


def _f16_correction_bound(c, xmax):
    """Absolute bound of the FP16 correction sum_{k>=1} c_k x^k on [0, xmax]
    from the error analysis (argument rounding, FMA Horner gamma_{m-1} with
    u = 2^-11, subnormal steps), written out here from that analysis."""
    c = np.asarray(c, dtype=np.float64)
    m = len(c)
    u, sub = 2.0 ** -11, 2.0 ** -25
    gam = (m - 1) * u / (1 - (m - 1) * u)
    x = np.linspace(0.0, xmax, 4097)
    dmax = np.abs(sum(k * c[k] * x ** (k - 1) for k in range(1, m))).max()
    a = sum(np.abs(c[k]) * x ** k for k in range(1, m))
    carry = sum(max(1.0, xmax) ** k for k in range(m))
    return float((dmax * (u * x + sub) + gam * a + (m - 1) * sub * carry).max() * 1.1)


@pytest.mark.parametrize("filt,degree", [("amnfe", 4), ("amnfe", 5), ("amnfe", 6), ("evmf", 4), ("evmf", 6),
                                         ("evmf", 7)])
def test_fe_f16_function_error_within_bound(vf, filt, degree):
    """The device's packed-FP16 exp / ENT against the same rounded polynomial
    in FP64 on a dense grid: within the correction bound (plus the FP32 steps
    around it), which the flagging bound relies on."""
    window = 5
    ap = vf.Approx("minimax", degree, precision="fp16x2")
    if filt == "amnfe":
        c = oracle.exp_approx("poly", degree, window=window, precision="fp16x2").coeffs
        xmax = oracle.amnfe_range(window)
        x = np.linspace(0.0, xmax, 1 << 20)
        out = vf.eval_function("amnfe", torch.from_numpy(x.astype(np.float32)).cuda(), ap, window=window)
        xf = x.astype(np.float32).astype(np.float64)
        ref = np.polyval(c[::-1], xf)
        bound = _f16_correction_bound(c, xmax) + 4 * 2.0 ** -24 * np.abs(ref)
    else:
        c = oracle.ent_approx("rangered", degree, precision="fp16x2").p
        P = np.linspace(0.0, 0.5, 1 << 20)[1:]
        out = vf.eval_function("evmf", torch.from_numpy(P.astype(np.float32)).cuda(), ap, window=window)
        Pf = P.astype(np.float32).astype(np.float64)
        m, e = np.frexp(Pf)
        ln = (e - 1) * math.log(2.0) + np.polyval(c[::-1], 2 * m - 1)
        ref = Pf * ln
        bound = Pf * (_f16_correction_bound(c, 1.0) + 8 * 2.0 ** -24 * (np.abs(ln) + 1.0))
    got = out.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - ref) <= bound), np.max(np.abs(got - ref) - bound)


def test_fe_f16_flags_more(vf):
    """The FP16 variants' wider bounds show up as more flagged windows."""
    clean, img = synth.workload_image(2, height=256, width=512)
    t = torch.from_numpy(img).cuda()
    for filt in ("amnfe", "evmf"):
        vf.run(filt, t, 5, vf.Approx("minimax", 6))
        f32 = vf.get_stats()["flagged"]
        vf.run(filt, t, 5, vf.Approx("minimax", 6, precision="fp16x2"))
        f16 = vf.get_stats()["flagged"]
        assert f16 >= f32, filt


def test_variants_rejected_where_not_implemented(vf):
    img = torch.zeros((8, 8, 3), dtype=torch.uint8, device="cuda")
    for ap in (vf.Approx("chord", 11, scheme="estrin", direct=True),
               vf.Approx("split", 7, precision="fp16x2"),
               vf.Approx("split", 7, scheme="estrin"),
               vf.Approx("chord", 11, scheme="estrin", precision="fp16x2")):
        with pytest.raises(vf.VfError):
            vf.filter_vdf(img, 3, ap)
    with pytest.raises(vf.VfError):
        vf.filter_batch([(img, "vdf", 3, None, vf.Approx("chord", 11, scheme="estrin"))])


def test_variant_stats_report_flags(vf):
    """The FP16 variant's wider bound shows up as more flagged windows."""
    clean, img = synth.workload_image(1, height=256, width=512)
    t = torch.from_numpy(img).cuda()
    vf.filter_vdf(t, 5, vf.Approx("chord", 11))
    f32 = vf.get_stats()["flagged"]
    vf.filter_vdf(t, 5, vf.Approx("chord", 11, precision="fp16x2"))
    f16 = vf.get_stats()["flagged"]
    assert f16 >= f32
