"""Every output is the exact FP64 decision of its window, so it cannot depend
on how the streaming kernels cut the image into strips: contexts created
with VF_STRIP_ROWS = 1, 2, 7, 64 and 300 rows per strip give the same bytes
as the per-call sized strips, for every filter (the member sums restart at
each strip's first row, where the state is built from padding rows)."""
import ctypes as C

import numpy as np
import pytest

from paper_1009_0959_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1009_0959_amd import vf
    vf.lib()
    return vf


def call(vf, ctx, filt, img, out, window, ap, param):
    L, im, a, s = vf.lib(), vf._image(img, out), ap.struct(), vf._stream()
    p = vf.default_param(filt, ap) if param is None else param
    if filt == "vdf":
        return L.vf_filter_vdf(ctx, C.byref(im), window, C.byref(a), s)
    if filt == "ddf":
        return L.vf_filter_ddf(ctx, C.byref(im), window, p, C.byref(a), s)
    if filt in ("amnfe", "amnfg"):
        return L.vf_filter_fuzzy_exp(ctx, C.byref(im), window, p, 1 if filt == "amnfg" else 0, C.byref(a), s)
    return L.vf_filter_log(ctx, C.byref(im), window, p, C.byref(a), s)


CASES = [("vdf", 3, ("chord", 11), None), ("vdf", 5, ("chord", 11), None), ("vdf", 7, ("chord", 11), None),
         ("vdf", 7, ("exact", 0), None), ("vdf", 5, ("exact", 0), None), ("ddf", 5, ("chord", 11), None),
         ("ddf", 7, ("chord", 11), None), ("ddf", 7, ("split", 9), None), ("amnfe", 5, ("minimax", 6), None),
         ("amnfg", 7, ("minimax", 5), None), ("evmf", 5, ("minimax", 6), None), ("evmf", 3, ("paper", 4), 0.05),
         ("vdf", 5, ("chord", 11, ), "fp16")]


@pytest.mark.parametrize("filt,window,spec,param", CASES)
def test_strip_height_does_not_change_outputs(vf, monkeypatch, filt, window, spec, param):
    extra = {}
    if param == "fp16":
        extra, param = dict(precision="fp16x2"), None
    cfg = 2 if filt in ("amnfe", "amnfg", "evmf") else 1
    clean, img_np = synth.workload_image(cfg, height=157, width=250)
    img = torch.from_numpy(img_np).cuda()
    ap = vf.Approx(*spec, **extra)
    want = vf.run(filt, img, window, ap, param if filt == "evmf" else None)
    torch.cuda.synchronize()
    for rows in ("1", "2", "7", "64", "300"):
        monkeypatch.setenv("VF_STRIP_ROWS", rows)
        ctx = C.c_void_p()
        assert vf.lib().vf_create(0, C.byref(ctx)) == vf.VF_OK
        try:
            out = torch.empty_like(img)
            assert call(vf, ctx, filt, img, out, window, ap, param) == vf.VF_OK
            torch.cuda.synchronize()
            bad = (out != want).any(-1).nonzero()
            assert bad.shape[0] == 0, (rows, bad.shape[0], bad[:4].tolist())
        finally:
            vf.lib().vf_destroy(ctx)
