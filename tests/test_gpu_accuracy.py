"""Accuracy of the approximants at full size, against the exact FP64 oracle.

The method's accuracy target: the minimax-polynomial filters change the image
quality by at most 0.01 dB of PSNR (against the clean image) relative to the
exact-function filter, and the exact GPU kernel agrees with the exact oracle.
Computed on the whole 4096 x 4096 headline image (VDF 3x3 / 5x5, DDF 5x5) and on
a 1024-row band of the mixed-noise image (AMNFE, EVMF 5x5).
"""
import numpy as np
import pytest

import oracle
import oracle.quality as OQ
from paper_1009_0959_amd import synth
from parity_util import oracle_approx

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1009_0959_amd import vf
    vf.lib()
    return vf


@pytest.fixture(scope="module")
def headline():
    return synth.workload_image(1)


@pytest.fixture(scope="module")
def mixed_band():
    clean, noisy = synth.workload_image(2)
    return clean[:1024].copy(), noisy[:1024].copy()


def run_gpu(vf, img, filt, window, ap):
    t = torch.from_numpy(img).cuda()
    out = vf.run(filt, t, window, ap)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("filt,window,spec", [("vdf", 3, ("chord", 11)), ("vdf", 5, ("chord", 11)),
                                              ("ddf", 5, ("chord", 11))])
def test_delta_psnr_headline(vf, headline, filt, window, spec):
    clean, noisy = headline
    exact = oracle.run_filter(noisy, filt, window, angle=oracle.angle_approx("exact"))
    approx_gpu = run_gpu(vf, noisy, filt, window, vf.Approx(*spec))
    d = OQ.psnr(clean, approx_gpu) - OQ.psnr(clean, exact)
    assert abs(d) <= 0.01, d
    # and the exact GPU kernel against the exact oracle, whole image
    exact_gpu = run_gpu(vf, noisy, filt, window, vf.Approx("exact"))
    assert (exact_gpu == exact).all(-1).mean() >= 0.999


@pytest.mark.parametrize("filt,spec", [("amnfe", ("minimax", 6)), ("evmf", ("minimax", 6))])
def test_delta_psnr_mixed_noise(vf, mixed_band, filt, spec):
    clean, noisy = mixed_band
    exact = oracle.run_filter(noisy, filt, 5, **oracle_approx(filt, vf.Approx("exact"), 5))
    approx_gpu = run_gpu(vf, noisy, filt, 5, vf.Approx(*spec))
    d = OQ.psnr(clean, approx_gpu) - OQ.psnr(clean, exact)
    assert abs(d) <= 0.01, d
    exact_gpu = run_gpu(vf, noisy, filt, 5, vf.Approx("exact"))
    assert (exact_gpu == exact).all(-1).mean() >= 0.999
