"""GPU parity at the workload configurations' own sizes and recipes, the FP64
precision mode, and the decision cases the FP32 bounds have to catch.

* The 256 x 256 uint8 anchor (10% salt-and-pepper, VDF 3x3, exact arccos)
  evaluated in FP64 on the GPU must equal the FP64 oracle pixel for pixel; the
  FP32 exact kernel must reach the 99.9% bar with every differing pixel valid.
* The 8192 x 8192 uint16 7x7 workload (Gaussian sigma 400 + 25% correlated
  impulses), VDF and DDF with the chord approximant, in the launch
  configuration the benchmark times, checked on every border tile and seeded
  interior tiles, plus window membership over the whole image.
* EVMF with the Table 4 rational (Section 3.3): windows built so that some P_j
  equals the cutoff T = 0.05 exactly and the switching decision depends on
  which side of T the computed P_j falls.
"""
import numpy as np
import pytest

import oracle
from paper_1009_0959_amd import synth
from parity_util import check_valid, cut_image, gpu_run, member_of_window, oracle_approx, tile_sample

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1009_0959_amd import vf as V
    V.lib()
    return V


# ---------------------------------------------------------------- FP64 precision

def test_config0_fp64_whole_image_equals_oracle(vf):
    """The 256^2 anchor, VDF 3x3 with the exact arccos, every window in FP64 on
    the GPU: bit-identical to the FP64 oracle over the whole image."""
    clean, img = synth.workload_image(0)
    assert img.shape == (256, 256, 3) and img.dtype == np.uint8
    ap = vf.Approx("exact", precision="fp64")
    got = gpu_run(vf, img, "vdf", 3, ap)
    want = oracle.run_filter(img, "vdf", 3, angle=oracle.angle_approx("exact"))
    assert np.array_equal(got, want)
    st = vf.get_stats()
    assert st["windows"] == 256 * 256 and st["flagged"] == 0


@pytest.mark.parametrize("direct", [False, True])
def test_config0_fp32_exact_whole_image(vf, direct):
    """The same anchor through the FP32 kernels (acosf, FP64 re-check of near
    ties): the 99.9% bar over the whole image, every differing pixel valid."""
    clean, img = synth.workload_image(0)
    ap = vf.Approx("exact", direct=direct)
    got = gpu_run(vf, img, "vdf", 3, ap)
    want = oracle.run_filter(img, "vdf", 3, angle=oracle.angle_approx("exact"))
    assert (got == want).all(-1).mean() >= 0.999
    check_valid(img, "vdf", 3, ap, None, got, want)


FP64_CASES = [("vdf", 3, ("paper", 4)), ("vdf", 5, ("chord", 11)), ("vdf", 7, ("split", 7)),
              ("ddf", 3, ("exact", 0)), ("ddf", 5, ("split", 9)), ("ddf", 7, ("chord", 11)),
              ("amnfe", 3, ("exact", 0)), ("amnfe", 5, ("minimax", 6)), ("amnfe", 7, ("rational", 4)),
              ("amnfe", 5, ("paper", 3)), ("evmf", 3, ("paper", 4)), ("evmf", 5, ("exact", 0)),
              ("evmf", 7, ("minimax", 6))]


@pytest.mark.parametrize("filt,window,spec", FP64_CASES)
@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_fp64_precision_bit_exact(vf, filt, window, spec, dtype):
    """FP64 precision evaluates every window from its definition with the same
    constants, in the oracle's order: equal to the oracle everywhere, on a
    ragged image of the mixed-noise recipe, 8- and 16-bit."""
    clean, img = synth.workload_image(2, height=41, width=77)
    if dtype == np.uint16:
        img = img.astype(np.uint16) * 257 + np.uint16(3)
    ap = vf.Approx(*spec, precision="fp64")
    got = gpu_run(vf, img, filt, window, ap)
    want = oracle.run_filter(img, filt, window, **oracle_approx(filt, ap, window))
    assert np.array_equal(got, want)


def test_fp64_rejected_where_not_defined(vf):
    img = torch.zeros((8, 8, 3), dtype=torch.uint8, device="cuda")
    with pytest.raises(vf.VfError):
        vf.filter_vdf(img, 3, vf.Approx("chord", 11, precision="fp64", scheme="estrin"))
    with pytest.raises(vf.VfError):
        vf.filter_batch([(img, "vdf", 3, None, vf.Approx("chord", 11, precision="fp64"))])
    with pytest.raises(vf.VfError):
        vf.eval_function("vdf", torch.zeros(4, device="cuda"), vf.Approx("chord", 11, precision="fp64"))


# ---------------------------------------------------------------- 16-bit 7x7

@pytest.mark.parametrize("shape", [(70, 133), (9, 300), (130, 61), (3, 2)])
@pytest.mark.parametrize("spec", [("chord", 11), ("split", 9), ("exact", 0)])
def test_vdf7_parity_u16(vf, shape, spec):
    """7x7 VDF on 16-bit images of the 8192^2 workload's recipe, ragged shapes
    (several strips and a partial one, fewer rows than the window)."""
    clean, img = synth.workload_image(4, height=shape[0], width=shape[1])
    ap = vf.Approx(*spec)
    got = gpu_run(vf, img, "vdf", 7, ap)
    want = oracle.run_filter(img, "vdf", 7, **oracle_approx("vdf", ap, 7))
    assert (got == want).all(-1).mean() >= 0.999
    check_valid(img, "vdf", 7, ap, None, got, want)


@pytest.fixture(scope="module")
def config4():
    return synth.workload_image(4)


@pytest.mark.parametrize("filt", ["vdf", "ddf"])
def test_config4_full_size_sampled(vf, config4, filt):
    """8192 x 8192 uint16, 7x7, chord degree 11, one call as the benchmark makes
    it: on every 64 x 64 border tile and seeded interior tiles (1/32 of the
    image) the outputs match the oracle, differing pixels valid; over the whole
    image every output is a member of its window."""
    clean, img = config4
    assert img.shape == (8192, 8192, 3) and img.dtype == np.uint16
    ap = vf.Approx("chord", 11)
    t = torch.from_numpy(img).cuda()
    out = vf.run(filt, t, 7, ap)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    del t, out
    pix = tile_sample(8192, 8192, seed=[4, 7, 1], fraction=32)
    want = oracle.run_filter(img, filt, 7, pixels=pix, **oracle_approx(filt, ap, 7))
    g = got[pix[:, 0], pix[:, 1]]
    assert (g == want).all(-1).mean() >= 0.999
    check_valid(img, filt, 7, ap, None, g, want, pixels=pix)
    assert member_of_window(img, got, 7).all()


# ---------------------------------------------------------------- EVMF at the ENT cutoff

@pytest.mark.parametrize("window", [3, 5, 7])
@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_evmf_paper_cutoff_band(vf, window, dtype):
    """EVMF with the Table 4 rational on windows whose P_j sits exactly at the
    cutoff: the FP32 kernels must flag them (the computed P_j may fall on
    either side of T) and the FP64 re-check must reproduce the oracle, in the
    streaming and the per-window kernels."""
    imgs = []
    for k, (base, u) in enumerate([((40, 60, 80), (3, 2, 1)), ((10, 200, 5), (1, -3, 4)),
                                   ((120, 20, 30), (2, 2, 5))]):
        im = cut_image(window, 45, 131, base, u, seed=[window, k])
        if dtype == np.uint16:
            im = im * 257 + 11
        imgs.append(im.astype(dtype))
    for img in imgs:
        assert img.min() >= 0
        for direct in (False, True):
            ap = vf.Approx("paper", 4, direct=direct)
            got = gpu_run(vf, img, "evmf", window, ap)
            want = oracle.run_filter(img, "evmf", window, ent=oracle.ent_approx("rational"))
            assert np.array_equal(got, want), (window, direct, (got != want).any(-1).sum())


# ---------------------------------------------------------------- deferred re-check

def test_pending_recheck_refuses_new_calls(vf):
    """While a deferred re-check is pending, a new filter or batch call on the
    context is refused without writing; after vf_recheck_pending a call on a
    smaller image filters it correctly (its re-check reads only its own list)."""
    clean, big = synth.workload_image(1, height=300, width=257)
    t = torch.from_numpy(big).cuda()
    a = vf.run("vdf", t, 5, vf.Approx("exact", defer=True))
    clean, small = synth.workload_image(1, height=40, width=70)
    ts = torch.from_numpy(small).cuda()
    out = torch.full_like(ts, 7)
    with pytest.raises(vf.VfError) as e:
        vf.run("vdf", ts, 5, vf.Approx("exact"), out=out)
    assert e.value.status == vf.VF_EINVAL
    with pytest.raises(vf.VfError):
        vf.filter_batch([(ts, "vdf", 5, None, vf.Approx("exact"))], [out])
    torch.cuda.synchronize()
    assert int((out != 7).sum()) == 0
    vf.recheck_pending()
    want_big = oracle.run_filter(big, "vdf", 5, angle=oracle.angle_approx("exact"))
    got_big = a.cpu().numpy()
    assert (got_big == want_big).all(-1).mean() >= 0.999
    check_valid(big, "vdf", 5, vf.Approx("exact"), None, got_big, want_big)
    got = gpu_run(vf, small, "vdf", 5, vf.Approx("exact"))
    want = oracle.run_filter(small, "vdf", 5, angle=oracle.angle_approx("exact"))
    assert (got == want).all(-1).mean() >= 0.999
    check_valid(small, "vdf", 5, vf.Approx("exact"), None, got, want)
