"""GPU tests of the autotuner: the chosen configuration meets the error target,
calls with the tuned flag equal explicit calls with the chosen configuration,
tuned batches equal tuned single calls, and tune files round-trip."""
import os

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
    vf.tune_clear()
    yield vf
    vf.tune_clear()


def explicit(vf, res, eval_kind):
    return vf.Approx(eval_kind, res["degree"], direct=res["direct"], scheme=res["scheme"],
                     precision=res["precision"])


@pytest.mark.parametrize("filt,window,eval_kind,target", [("vdf", 5, "chord", 1e-6), ("vdf", 3, "chord", 1e-5),
                                                          ("ddf", 5, "chord", 1e-6), ("amnfe", 5, "minimax", 1e-6),
                                                          ("evmf", 5, "minimax", 1e-5)])
def test_autotune_choice_and_tuned_calls(vf, filt, window, eval_kind, target):
    clean, img = synth.workload_image(1, height=512, width=512)
    t = torch.from_numpy(img).cuda()
    res = vf.autotune(filt, t, window, vf.Approx(eval_kind), max_func_err=target)
    assert res["func_err"] <= target and res["candidates"] >= 1 and res["ms"] > 0
    if res["direct"]:
        assert res["strip_rows"] == 0
    tuned = vf.run(filt, t, window, vf.Approx(eval_kind, tuned=True))
    torch.cuda.synchronize()
    # the same configuration requested explicitly (tile height via the tuned call only)
    ex = vf.run(filt, t, window, explicit(vf, res, eval_kind))
    torch.cuda.synchronize()
    got = tuned.cpu().numpy()
    assert np.array_equal(got, ex.cpu().numpy())
    ap = explicit(vf, res, eval_kind)
    pix = np.stack(np.meshgrid(np.arange(0, 512, 7), np.arange(0, 512, 5), indexing="ij"), -1).reshape(-1, 2)
    pix = pix.astype(np.int32)
    want = oracle.run_filter(img, filt, window, pixels=pix, **oracle_approx(filt, ap, window))
    g = got[pix[:, 0], pix[:, 1]]
    assert (g == want).all(-1).mean() >= 0.999
    check_valid(img, filt, window, ap, None, g, want, pixels=pix)


def test_tuned_batch_equals_tuned_calls(vf):
    """Batch items with the tuned flag take the tuned degree and kernel
    (Horner, FP32; strips sized per class); every output still equals the single tuned call's
    (both are exact against the oracle's decision for their polynomial) and the
    oracle on sampled pixels."""
    vf.tune_clear()
    clean, img = synth.workload_image(1, height=256, width=256)
    t = torch.from_numpy(img).cuda()
    r5 = vf.autotune("vdf", t, 5, vf.Approx("chord"), max_func_err=1e-6)
    r3 = vf.autotune("amnfe", t, 3, vf.Approx("minimax"), max_func_err=1e-6)
    arrs = [synth.workload_image(3, i, height=200 + 37 * i, width=300 - 21 * i)[1] for i in range(4)]
    imgs = [torch.from_numpy(a).cuda() for a in arrs]
    items = [(imgs[0], "vdf", 5, None, vf.Approx("chord", tuned=True)),
             (imgs[1], "amnfe", 3, None, vf.Approx("minimax", tuned=True)),
             (imgs[2], "vdf", 5, None, vf.Approx("chord", tuned=True)),
             (imgs[3], "vdf", 3, None, vf.Approx("chord", 11, tuned=True))]   # no entry: as given
    outs = vf.filter_batch(items)
    torch.cuda.synchronize()
    used = [vf.Approx("chord", r5["degree"], direct=r5["direct"]),
            vf.Approx("minimax", r3["degree"], direct=r3["direct"]),
            vf.Approx("chord", r5["degree"], direct=r5["direct"]),
            vf.Approx("chord", 11)]
    plain = [r5["precision"] == "fp32" and r5["scheme"] == "horner",
             r3["precision"] == "fp32" and r3["scheme"] == "horner", None, True]
    plain[2] = plain[0]
    for k, ((im, f, w, p, a), o) in enumerate(zip(items, outs)):
        got = o.cpu().numpy()
        # the FP32 Horner form of the tuned configuration, and the tuned call
        # itself where the tuner chose FP32 Horner (a batch evaluates no other)
        ref = vf.run(f, im, w, used[k], p)
        torch.cuda.synchronize()
        assert np.array_equal(got, ref.cpu().numpy()), k
        if plain[k]:
            single = vf.run(f, im, w, a, p)
            torch.cuda.synchronize()
            assert np.array_equal(got, single.cpu().numpy()), k
        H, W = arrs[k].shape[:2]
        pix = np.stack(np.meshgrid(np.arange(0, H, 4), np.arange(0, W, 4), indexing="ij"), -1).reshape(-1, 2)
        pix = pix.astype(np.int32)
        want = oracle.run_filter(arrs[k], f, w, pixels=pix, **oracle_approx(f, used[k], w))
        g = got[pix[:, 0], pix[:, 1]]
        assert (g == want).all(-1).mean() >= 0.999, k
        check_valid(arrs[k], f, w, used[k], None, g, want, pixels=pix)


def test_tune_file_round_trip(vf, tmp_path):
    vf.tune_clear()
    clean, img = synth.workload_image(1, height=256, width=256)
    t = torch.from_numpy(img).cuda()
    res = vf.autotune("vdf", t, 3, vf.Approx("chord"), max_func_err=1e-6)
    a = vf.run("vdf", t, 3, vf.Approx("chord", tuned=True))
    path = str(tmp_path / "tune.txt")
    vf.tune_save(path)
    vf.tune_clear()
    b = vf.run("vdf", t, 3, vf.Approx("chord", 7, tuned=True))      # no entry: degree 7 as given
    vf.tune_load(path)
    c = vf.run("vdf", t, 3, vf.Approx("chord", 7, tuned=True))      # entry restored
    torch.cuda.synchronize()
    assert torch.equal(a, c)
    with open(path) as f:
        lines = [l for l in f if not l.startswith("#")]
    assert len(lines) == 1 and int(lines[0].split()[6]) == res["degree"]
    bad = str(tmp_path / "bad.txt")
    with open(bad, "w") as f:
        f.write("0 3 1 3 0 64 8 0 0 1.0 0.0\n")   # chord degree 8 does not exist
    with pytest.raises(vf.VfError):
        vf.tune_load(bad)
