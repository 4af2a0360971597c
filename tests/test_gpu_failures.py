"""Failure handling forced from the host (no kernel faults): launch failures
injected through VF_INJECT_HIP_ERROR must surface as VF_EHIP with the launch
named in vf_last_error, and the context must stay usable, its next calls
exact again (the re-check counters of the failed call are re-zeroed)."""
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
    from paper_1009_0959_amd import vf
    vf.lib()
    return vf


def run_checked(vf, img, filt, window, ap):
    out = vf.run(filt, torch.from_numpy(img).cuda(), window, ap)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    want = oracle.run_filter(img, filt, window, **oracle_approx(filt, ap, window))
    assert (got == want).all(-1).mean() >= 0.999
    check_valid(img, filt, window, ap, None, got, want)


@pytest.mark.parametrize("site", ["window", "recheck"])
@pytest.mark.parametrize("filt,window,spec", [("vdf", 5, ("chord", 11)), ("evmf", 3, ("minimax", 6)),
                                              ("ddf", 7, ("chord", 11))])
def test_injected_launch_failure_then_exact_again(vf, monkeypatch, site, filt, window, spec):
    ap = vf.Approx(*spec)
    clean, img = synth.workload_image(1, height=70, width=150)
    t = torch.from_numpy(img).cuda()
    monkeypatch.setenv("VF_INJECT_HIP_ERROR", site)
    with pytest.raises(vf.VfError) as e:
        vf.run(filt, t, window, ap)
        torch.cuda.synchronize()
    assert e.value.status == vf.VF_EHIP
    assert ("re-check" if site == "recheck" else "window kernel") in str(e.value)
    monkeypatch.delenv("VF_INJECT_HIP_ERROR")
    # the context recovers: a larger image, then the same one, both exact
    clean2, img2 = synth.workload_image(0, height=130, width=201)
    run_checked(vf, img2, filt, window, ap)
    run_checked(vf, img, filt, window, ap)


def test_injected_batch_failure_then_batch_again(vf, monkeypatch):
    imgs = [synth.workload_image(1, image=k, height=40 + 9 * k, width=90)[1] for k in range(3)]
    items = [(torch.from_numpy(i).cuda(), f, w, None, vf.Approx(*s))
             for i, (f, w, s) in zip(imgs, [("vdf", 3, ("chord", 11)), ("amnfe", 5, ("minimax", 6)),
                                            ("evmf", 3, ("paper", 4))])]
    monkeypatch.setenv("VF_INJECT_HIP_ERROR", "batch")
    with pytest.raises(vf.VfError) as e:
        vf.filter_batch(items)
    assert e.value.status == vf.VF_EHIP
    monkeypatch.delenv("VF_INJECT_HIP_ERROR")
    outs = vf.filter_batch(items)
    torch.cuda.synchronize()
    for (t, f, w, p, ap), o in zip(items, outs):
        want = vf.run(f, t, w, ap)
        torch.cuda.synchronize()
        assert torch.equal(o, want)
