"""The no-allocation VDF entry point (vf_filter_vdf_noalloc) through the C ABI
against the context entry point (vf_filter_vdf) and the FP64 oracle: two calls
in a row on one GPU (the second on a smaller image, so stale list entries and
counts of the first would show), plus its refusals."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_1009_0959_amd import synth
from parity_util import check_valid, oracle_approx

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1009_0959_amd import vf as V
    V.lib()
    return V


def _noalloc(vf, t, out, window, ap):
    im, a = vf._image(t, out), ap.struct()
    return vf.lib().vf_filter_vdf_noalloc(t.device.index, C.byref(im), window, C.byref(a), vf._stream())


@pytest.mark.parametrize("window,spec", [(3, ("chord", 11)), (5, ("chord", 11)), (5, ("exact", 0)),
                                         (7, ("split", 9))])
def test_noalloc_equals_context_entry_point(vf, window, spec):
    ap = vf.Approx(*spec)
    for shape in ((700, 1200), (130, 257)):       # 840000 pixels, then a smaller image
        clean, img = synth.workload_image(1, height=shape[0], width=shape[1])
        t = torch.from_numpy(img).cuda()
        ref = vf.filter_vdf(t, window, ap)
        out = torch.full_like(t, 3)
        assert _noalloc(vf, t, out, window, ap) == vf.VF_OK
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got, ref.cpu().numpy()), (shape, int((got != ref.cpu().numpy()).any(-1).sum()))
        want = oracle.run_filter(img, "vdf", window, **oracle_approx("vdf", ap, window))
        assert (got == want).all(-1).mean() >= 0.999
        check_valid(img, "vdf", window, ap, None, got, want)


def test_noalloc_refusals(vf):
    big = torch.zeros((1025, 1024, 3), dtype=torch.uint8, device="cuda")    # 2^20 + 1024 pixels
    out = torch.full_like(big, 9)
    assert _noalloc(vf, big, out, 3, vf.Approx("chord", 11)) == vf.VF_EINVAL
    small = torch.zeros((16, 16, 3), dtype=torch.uint8, device="cuda")
    out2 = torch.full_like(small, 9)
    assert _noalloc(vf, small, out2, 3, vf.Approx("chord", 11, defer=True)) == vf.VF_EINVAL
    assert _noalloc(vf, small, out2, 3, vf.Approx("chord", 11, tuned=True)) == vf.VF_EINVAL
    assert _noalloc(vf, small, out2, 9, vf.Approx("chord", 11)) == vf.VF_EUNSUPPORTED
    torch.cuda.synchronize()
    assert int((out != 9).sum()) == 0 and int((out2 != 9).sum()) == 0
    # the largest accepted image
    clean, img = synth.workload_image(1, height=1024, width=1024)
    t = torch.from_numpy(img).cuda()
    o = torch.empty_like(t)
    assert _noalloc(vf, t, o, 5, vf.Approx("chord", 11)) == vf.VF_OK
    assert torch.equal(o, vf.filter_vdf(t, 5, vf.Approx("chord", 11)))
