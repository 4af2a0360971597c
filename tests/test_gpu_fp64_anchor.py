"""Whole-image check of every FP32 flagging bound: VF_PREC_FP64 evaluates
every window in FP64 with the same window function as the re-check (the
oracle's arithmetic, Section 3's equations), so the FP32 path (FP32 criteria,
flags, FP64 re-check of the flagged windows) must give the same bytes on
every pixel. A window that escapes its bound while its FP32 decision differs
from the FP64 one shows up here at any image size, not only on sampled
pixels."""
import zlib

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


def image(kind):
    if kind == "impulse":
        return synth.workload_image(1, height=400, width=517)[1]
    if kind == "mixed":
        return synth.workload_image(2, height=400, width=517)[1]
    if kind == "u16":
        return synth.workload_image(4, height=300, width=413)[1]
    # three colours a unit apart with 3% impulses: exact ties between distinct vectors
    rng = np.random.default_rng(zlib.crc32(b"anchor-palette"))
    pal = np.array([[203, 179, 157], [202, 180, 157], [202, 179, 157]])
    img = pal[rng.choice(3, size=(200, 333), p=[0.45, 0.45, 0.1])]
    hit = rng.random((200, 333)) < 0.03
    img[hit] = rng.integers(0, 256, (int(hit.sum()), 3))
    return img.astype(np.uint8)


CASES = []
for w in (3, 5, 7):
    for spec in (("chord", 11), ("split", 9), ("paper", 4), ("exact", 0)):
        CASES.append(("vdf", w, spec, None))
    for spec in (("chord", 11), ("split", 7), ("exact", 0)):
        CASES.append(("ddf", w, spec, None))
    for filt in ("amnfe", "amnfg"):
        for spec in (("minimax", 5), ("rational", 4), ("ratfit", 2), ("exact", 0)):
            CASES.append((filt, w, spec, None))
    CASES.append(("amnfe", w, ("paper", 4), None))
    for spec, t in ((("minimax", 6), 0.0), (("minimax", 6), 0.05), (("paper", 4), 0.05), (("exact", 0), 0.0),
                    (("exact", 0), 0.05)):
        CASES.append(("evmf", w, spec, t))


@pytest.mark.parametrize("kind", ["impulse", "mixed", "u16", "palette"])
@pytest.mark.parametrize("filt,window,spec,param", CASES)
def test_fp32_path_equals_fp64_every_window(vf, kind, filt, window, spec, param):
    img = torch.from_numpy(image(kind)).cuda()
    direct_too = window == 5
    want = vf.run(filt, img, window, vf.Approx(*spec, precision="fp64"), param)
    for direct in ((False, True) if direct_too else (False,)):
        got = vf.run(filt, img, window, vf.Approx(*spec, direct=direct), param)
        torch.cuda.synchronize()
        bad = (got != want).any(-1).nonzero()
        assert bad.shape[0] == 0, (direct, bad.shape[0], bad[:4].tolist(),
                                   got[tuple(bad[0].tolist())].tolist(), want[tuple(bad[0].tolist())].tolist())
