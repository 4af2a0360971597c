"""Benchmark of the vector-filter hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-configs]
    python bench.py --profile NAME [--steps K]      (one kernel, for rocprofv3)

Workload of the metric (the headline configuration): one 4096 x 4096 RGB uint8
synthetic image (smooth gradients + Gaussian blobs, 20% correlated impulse
noise with uniform replacement values), resident in HBM. One step filters it
with the vector directional filter at 3x3 and at 5x5 using the minimax arccos
approximant (chord degree 11, FP32, with the FP64 re-check of near-tie
windows). The value is filtered pixels per second over the step (2 x 4096^2
pixels per step), in Mpixel/s.

Also in the same JSON line:
  * roofline: the dominant kernel (streaming VDF 5x5) -- algorithmic FLOP per
    launch over its event-timed duration, against the published FP32 vector
    peak (157.3 TFLOP/s); the issue ceiling without packed FP32 math (78.6)
    under its own key; HBM traffic from the committed counter summary while
    the kernel's sources are unchanged;
  * cpu_baseline: the FP64 CPU oracle on the same step (whole image, both
    windows, host threads), with the GPU's agreement with it;
  * configs: every other workload configuration, each with its time,
    Mpixel/s, flagged fraction, the oracle's agreement on a stated sample and
    its dominant kernel's roofline fraction: the 256^2 anchor (FP64 and FP32
    exact), the approximant sweep of the headline image (VDF and DDF), the
    mixed-noise 5x5 AMNFE / AMNFG / EVMF study (FP32, packed FP16, the paper's
    rationals), the uneven 256-image batch, and the 8192^2 16-bit 7x7 VDF / DDF.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpixel/s VDF 3x3 & 5x5, minimax vs exact acosf, at ≥99.9% oracle selection match"
HEADLINE = ("chord", 11)           # approximant of the timed step
PEAK_FP32 = 157.3                  # TFLOP/s: published MI355X FP32 vector peak (counts packed FMA)
PEAK_FP32_NONPACKED = 78.6         # TFLOP/s: 256 CU x 64 lanes x 2 flop x 2.4 GHz, one FMA per lane-cycle


# Sources that define the dominant kernel; the counter summary under profiles/
# records their hash, and its HBM traffic figure is reported only while the
# kernel is unchanged.
KERNEL_SOURCES = ["include/vf.h", "paper_1009_0959_amd/csrc/vf_internal.h",
                  "paper_1009_0959_amd/csrc/kern_common.h", "paper_1009_0959_amd/csrc/kern_stream.h",
                  "paper_1009_0959_amd/csrc/batch.h", "paper_1009_0959_amd/csrc/recheck_dev.h",
                  "paper_1009_0959_amd/csrc/kern_angle_w5.hip"]
COUNTER_SUMMARY = "profiles/vdf5_stream_chord11_4096_counters.md"


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read() + b"\0")
    return h.hexdigest()


def profiled_traffic():
    """(bytes per launch, summary file) from the counter summary if it was taken
    on the current kernel sources, else (None, reason)."""
    path = os.path.join(ROOT, COUNTER_SUMMARY)
    if not os.path.exists(path):
        return None, "no counter summary"
    fields = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].strip().split(": ", 1)
                fields[k.strip("`")] = v.strip().strip("`")
    if fields.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None, "kernel changed since the counters were taken"
    return int(fields["traffic_bytes_per_launch"]), COUNTER_SUMMARY


# ------------------------------------------------------------------ algorithmic work

def pair_flops(eval_kind: str, degree: int) -> int:
    """Algorithmic FLOP per unordered window pair of the VDF kernel (FMA = 2):
    chord difference 3, squared norm 5, polynomial in s^2 2(m - 1) with m
    coefficients, times s 1, two accumulations 2 (the square root is not a
    FLOP). Exact mode: difference 3, norm 5, cosine 2, accumulation 2 (acosf
    itself is not counted)."""
    if eval_kind == "exact":
        return 12
    m = (degree + 1) // 2
    if eval_kind == "chord":
        return 3 + 5 + 2 * (m - 1) + 1 + 2
    if eval_kind == "split":
        return 3 + 5 + (2 * (m - 1) + 1) + (2 + 1 + 2 * (m - 1) + 2) + 2
    return 3 + 5 + 1 + 8 + 2 + 8 + 2    # paper two-piece, degree 4


def direct_flops_per_pixel(w: int, spec) -> int:
    """Per-window VDF kernel: every unordered pair of the n = w^2 members."""
    n = w * w
    return n * (n - 1) // 2 * pair_flops(*spec)


def sliding_sum_flops(w: int) -> int:
    """Per output pixel and summed quantity, the streaming kernels' sliding
    member sums: subtract the leaving row (w(w-1)), add the new row's pair
    values to both members (2 w^2 (w-1)) and the new row's own pairs (w(w-1))."""
    return w * (w - 1) + 2 * w * w * (w - 1) + w * (w - 1)


def stream_flops_per_pixel(filt: str, w: int, spec) -> int:
    """Algorithmic FLOP per output pixel of the streaming kernels (FMA = 2;
    square roots, reciprocals and the exact acosf / expf / logf are not
    counted). Each of the 2w(w-1) unique pixel pairs per pixel is scored once:
      VDF   : the angle (pair_flops - 2) + the sliding sums;
      DDF   : the angle + the L2 distance (difference 3, norm 5), two sliding
              sums, the criterion product per member;
      AMNFE/AMNFG : the exact L1 distance (one v_sad, counted 1) + its sliding
              sum; per member the EXP argument (L1 r k: 2; Gaussian: r k 1,
              squared deviation 5, 0.5 q t^2 3), the exp polynomial 2 deg
              (rational 4 deg + 1), r^3 2, weight 1, deviations 3, the
              weighted sums 12, the denominator 1;
      EVMF  : the L2 distance 8 + its sliding sum; per member the deviation
              from the mean 11, D 1, P 1, ENT (range reduced: 5 + 2 deg; exact
              1; the Table 4 rational: two Horner sums 4 deg, + 1) and H 1."""
    n = w * w
    pairs = 2 * w * (w - 1)
    kind, deg = spec
    if filt == "vdf":
        return pairs * (pair_flops(kind, deg) - 2) + sliding_sum_flops(w)
    if filt == "ddf":
        return pairs * (pair_flops(kind, deg) - 2 + 8) + 2 * sliding_sum_flops(w) + n
    if filt in ("amnfe", "amnfg"):
        kev = {"exact": 0, "minimax": 2 * deg, "paper": 2 * deg, "rational": 4 * deg + 1,
               "ratfit": 4 * deg + 1}[kind]
        zarg = 2 if filt == "amnfe" else 9
        return pairs * 1 + sliding_sum_flops(w) + n * (zarg + kev + 2 + 1 + 3 + 12 + 1)
    ent = {"exact": 1, "minimax": 5 + 2 * deg, "paper": 4 * deg + 1}[kind]
    return pairs * 8 + sliding_sum_flops(w) + n * (11 + 1 + 1 + ent + 1)


# ------------------------------------------------------------------ helpers

def oracle_approx(filt, spec, window, kappa=0.33):
    """The oracle's approximant for a library approximant (eval, degree)."""
    import oracle
    kind, deg = spec
    if filt in ("vdf", "ddf"):
        if kind == "exact":
            return dict(angle=oracle.angle_approx("exact"))
        if kind == "paper":
            return dict(angle=oracle.angle_approx("paper2", source="paper"))
        return dict(angle=oracle.angle_approx(kind, deg))
    if filt in ("amnfe", "amnfg"):
        if kind == "exact":
            return dict(expap=oracle.exp_approx("exact"))
        if kind == "paper":
            return dict(expap=oracle.exp_approx("poly", deg, source="paper"))
        if kind == "rational":
            return dict(expap=oracle.exp_approx("rational"))
        if kind == "ratfit":
            return dict(expap=oracle.exp_approx("ratfit", deg, window=window, kappa=kappa,
                                                kernel="gauss" if filt == "amnfg" else "exp"))
        return dict(expap=oracle.exp_approx("poly", deg, window=window, kappa=kappa,
                                            kernel="gauss" if filt == "amnfg" else "exp"))
    if kind == "exact":
        return dict(ent=oracle.ent_approx("exact"))
    if kind == "paper":
        return dict(ent=oracle.ent_approx("rational"))
    return dict(ent=oracle.ent_approx("rangered", deg))


def sample_pixels(H, W, k, seed, band=4):
    """k seeded pixels plus every pixel of a band of `band` rows / columns
    along each border (K x 2 array of (y, x))."""
    rng = np.random.default_rng(seed)
    pts = [np.stack([rng.integers(0, H, k), rng.integers(0, W, k)], 1)]
    b = min(band, H, W)
    ys, xs = np.mgrid[0:b, 0:W]
    pts += [np.stack([ys.ravel(), xs.ravel()], 1), np.stack([H - 1 - ys.ravel(), xs.ravel()], 1)]
    ys, xs = np.mgrid[0:H, 0:b]
    pts += [np.stack([ys.ravel(), xs.ravel()], 1), np.stack([ys.ravel(), W - 1 - xs.ravel()], 1)]
    return np.unique(np.concatenate(pts), axis=0).astype(np.int32)


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


class Gpu:
    """Timing helpers on torch's current stream (the stream the library's
    calls are issued on)."""

    def __init__(self):
        import torch
        from paper_1009_0959_amd import vf
        self.torch, self.vf = torch, vf

    def quality(self, clean_t, img):
        """Section 4's criteria on the GPU (vf_quality) of a filtered image
        (tensor or array) against the original."""
        t = img if isinstance(img, self.torch.Tensor) else self.torch.from_numpy(img).cuda()
        return self.vf.quality(clean_t, t)

    def psnr(self, clean_t, img):
        mse = self.quality(clean_t, img)["mse"]
        maxv = 65535.0 if clean_t.dtype == self.torch.uint16 else 255.0
        return float("inf") if mse == 0 else 10.0 * math.log10(maxv * maxv / mse)

    def timed(self, fn, steps, warmup):
        torch = self.torch
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps   # ms

    def kernel_only(self, filt, img, w, spec, param, out, steps, **extra):
        """The window kernel alone, exactly as a call runs it: the call lists
        its near ties (deferred re-check); events bracket only the window
        kernel, on the stream it is launched on."""
        torch, vf = self.torch, self.vf
        a_def = vf.Approx(*spec, defer=True, **extra)
        total = 0.0
        for i in range(steps + 2):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            vf.run(filt, img, w, a_def, param, out=out)
            e1.record()
            vf.recheck_pending()
            torch.cuda.synchronize()
            if i >= 2:
                total += e0.elapsed_time(e1)
        return total / steps

    def measure(self, filt, img, w, spec, out, steps, param=None, kernel=True, **extra):
        """(call ms, window-kernel ms or None, flagged fraction, output array)."""
        vf = self.vf
        a = vf.Approx(*spec, **extra)
        ms = self.timed(lambda: vf.run(filt, img, w, a, param, out=out), steps, 2)
        k_ms = self.kernel_only(filt, img, w, spec, param, out, max(3, steps // 2), **extra) if kernel else None
        vf.run(filt, img, w, a, param, out=out)
        st = vf.get_stats()
        return ms, k_ms, st["flagged"] / max(1, st["windows"]), out.cpu().numpy()


def frac_of(flops, ms):
    tf = flops / (ms * 1e-3) / 1e12
    return round(tf, 3), round(tf / PEAK_FP32, 4)


# ------------------------------------------------------------------ further configurations

def config0(g, images, nthreads):
    """256 x 256 uint8, 10% salt-and-pepper, VDF 3x3 with the exact arccos:
    every window in FP64 on the GPU (the correctness anchor) and the FP32
    acosf kernel, both against the FP64 oracle on the whole image."""
    import oracle
    torch, vf = g.torch, g.vf
    clean, img = images["c0"]
    t = torch.from_numpy(img).cuda()
    out = torch.empty_like(t)
    res = {"workload": "256x256 RGB uint8, 10% uncorrelated salt-and-pepper; VDF 3x3, exact arccos"}
    t1 = time.time()
    want = oracle.run_filter(img, "vdf", 3, angle=oracle.angle_approx("exact"), nthreads=nthreads)
    t_cpu = time.time() - t1
    for key, extra in (("fp64", dict(precision="fp64")), ("fp32_acosf", {})):
        ms, _, fl, got = g.measure("vdf", t, 3, ("exact", 0), out, 10, kernel=False, **extra)
        res[key] = {"ms": round(ms, 4), "mpix_s": round(256 * 256 / (ms * 1e-3) / 1e6, 1),
                    "flagged_frac": round(fl, 6), "oracle_agreement": float((got == want).all(-1).mean()),
                    "oracle_sample": "the whole image"}
    res["oracle_mpix_s"] = round(256 * 256 / t_cpu / 1e6, 3)
    log(f"config 0: fp64 {res['fp64']['ms']} ms agreement {res['fp64']['oracle_agreement']}")
    return res


SWEEP = [("vdf", ("exact", 0)), ("vdf", ("paper", 4)), ("vdf", ("split", 3)), ("vdf", ("split", 5)),
         ("vdf", ("split", 7)), ("vdf", ("split", 9)), ("vdf", ("chord", 7)), ("vdf", ("chord", 9)),
         ("vdf", ("chord", 11)), ("vdf", ("chord", 13)), ("ddf", ("exact", 0)), ("ddf", ("split", 9)),
         ("ddf", ("chord", 11))]


def config1_sweep(g, images, nthreads, steps):
    """The headline image: every approximant of the VDF and DDF at 3x3 and
    5x5, each timed (call and window kernel), its flagged fraction, its
    agreement with the FP64 oracle (same approximant) on a sample, and its
    PSNR change against the exact-acosf kernel's output."""
    import oracle
    from paper_1009_0959_amd import synth
    torch = g.torch
    clean, img = images["c1"]
    H, W = img.shape[:2]
    t = torch.from_numpy(img).cuda()
    clean_t = torch.from_numpy(clean).cuda()
    out = torch.empty_like(t)
    pix = sample_pixels(H, W, 30000, [1, 5])
    res, exact_out = {}, {}
    for filt, spec in SWEEP:
        for w in (3, 5):
            ms, k_ms, fl, got = g.measure(filt, t, w, spec, out, steps)
            want = oracle.run_filter(img, filt, w, pixels=pix, nthreads=nthreads, **oracle_approx(filt, spec, w))
            gs = got[pix[:, 0], pix[:, 1]]
            if spec[0] == "exact":
                exact_out[(filt, w)] = got
            ref = exact_out[(filt, w)]
            flops = H * W * stream_flops_per_pixel(filt, w, spec)
            tf, fr = frac_of(flops, k_ms)
            res[f"{filt}{w}_{spec[0]}{spec[1] or ''}"] = {
                "ms": round(ms, 4), "mpix_s": round(H * W / (ms * 1e-3) / 1e6, 1), "kernel_ms": round(k_ms, 4),
                "kernel_tflops": tf, "kernel_frac": fr, "flagged_frac": round(fl, 6),
                "oracle_agreement": round(float((gs == want).all(-1).mean()), 7),
                "agree_with_exact": round(float((got == ref).all(-1).mean()), 6),
                "dpsnr_vs_exact_db": round(g.psnr(clean_t, got) - g.psnr(clean_t, ref), 5),
                "dncd_vs_exact": round(g.quality(clean_t, got)["ncd"] - g.quality(clean_t, ref)["ncd"], 8)}
            log(f"sweep {filt}{w} {spec}: {ms:.3f} ms, kernel {k_ms:.3f} ms")
    return {"workload": "the headline 4096x4096 image; VDF and DDF, 3x3 and 5x5, every approximant",
            "oracle_sample": f"{len(pix)} pixels: 30000 seeded + 4-pixel border bands", "runs": res}


def config2(g, images, nthreads, steps):
    """Mixed noise 4096^2, 5x5: AMNFE and EVMF with minimax exp / ln (FP32 and
    packed FP16), the paper's Table 3 / Table 4 rationals and the exact
    functions; AMNFG (Gaussian kernel) with its minimax exp."""
    import oracle
    from paper_1009_0959_amd import synth
    torch = g.torch
    clean, img = images["c2"]
    H, W = img.shape[:2]
    t = torch.from_numpy(img).cuda()
    clean_t = torch.from_numpy(clean).cuda()
    out = torch.empty_like(t)
    pix = sample_pixels(H, W, 60000, [2, 5])
    runs = [("amnfe", ("minimax", 6), {}), ("amnfe", ("minimax", 6), {"precision": "fp16x2"}),
            ("amnfe", ("rational", 4), {}), ("amnfe", ("exact", 0), {}),
            ("evmf", ("minimax", 6), {}), ("evmf", ("minimax", 6), {"precision": "fp16x2"}),
            ("evmf", ("paper", 4), {}), ("evmf", ("exact", 0), {}),
            ("amnfg", ("minimax", 5), {}), ("amnfg", ("exact", 0), {}),
            ("amnfe", ("ratfit", 2), {}), ("amnfg", ("ratfit", 2), {})]
    res, exact_out, total_ms = {}, {}, 0.0
    for filt, spec, extra in runs:
        ms, k_ms, fl, got = g.measure(filt, t, 5, spec, out, steps, **extra)
        want = oracle.run_filter(img, filt, 5, pixels=pix, nthreads=nthreads, **oracle_approx(filt, spec, 5))
        gs = got[pix[:, 0], pix[:, 1]]
        tag = "".join(f"_{v}" for v in extra.values())
        if spec[0] == "exact":
            exact_out[filt] = got
        d = {"ms": round(ms, 4), "mpix_s": round(H * W / (ms * 1e-3) / 1e6, 1), "kernel_ms": round(k_ms, 4),
             "flagged_frac": round(fl, 6), "oracle_agreement": round(float((gs == want).all(-1).mean()), 7)}
        if not extra:
            tf, fr = frac_of(H * W * stream_flops_per_pixel(filt, 5, spec), k_ms)
            d["kernel_tflops"], d["kernel_frac"] = tf, fr
        if spec[0] == "minimax" and not extra:     # the FP32 minimax polynomial runs make the config's figure
            total_ms += ms
        res[f"{filt}5_{spec[0]}{spec[1] or ''}{tag}"] = d
        log(f"config 2 {filt} {spec}{tag}: {ms:.3f} ms")
    for filt, ref in exact_out.items():
        res[f"{filt}5_exact"]["psnr_db"] = round(g.psnr(clean_t, ref), 4)
    return {"workload": "4096x4096 RGB uint8, Gaussian sigma 10 + 10% correlated impulses; AMNFE, EVMF, AMNFG 5x5",
            "oracle_sample": f"{len(pix)} pixels: 60000 seeded + 4-pixel border bands (same approximant)",
            "mpix_s_amnfe_evmf_amnfg_minimax": round(3 * H * W / (total_ms * 1e-3) / 1e6, 1), "runs": res}


BATCH_APPROX = {"vdf": ("chord", 11), "ddf": ("chord", 11), "amnfe": ("minimax", 6),
                "evmf": ("minimax", 6)}


def _batch_image(i: int):
    from paper_1009_0959_amd import synth
    return synth.workload_image(3, i)[1]


def batch_images(count=256):
    import concurrent.futures as cf
    with cf.ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(_batch_image, range(count), chunksize=4))


def config3(g, images, nthreads, steps):
    """The uneven batch: 256 uint8 images of log-uniform area 320x240 ..
    4000x3000, each with its own filter and window, one vf_filter_batch call
    (a captured graph of persistent kernels), against one call per image; the
    oracle on 300 seeded pixels of every image (corners included)."""
    import oracle
    from paper_1009_0959_amd import synth
    torch, vf = g.torch, g.vf
    imgs = images["c3"]
    assign = synth.batch_assignments(len(imgs))
    tens = [torch.from_numpy(i).cuda() for i in imgs]
    outs = [torch.empty_like(t) for t in tens]
    items = [(t, f, w, None, vf.Approx(*BATCH_APPROX[f])) for t, (f, w) in zip(tens, assign)]
    pixels = sum(int(i.shape[0]) * int(i.shape[1]) for i in imgs)
    t1 = time.time()
    vf.filter_batch(items, outs)
    torch.cuda.synchronize()
    build_s = time.time() - t1
    ms = g.timed(lambda: vf.filter_batch(items, outs), steps, 1)
    st = vf.get_stats()

    def one_by_one():
        for (t, f, w, p, a), o in zip(items, outs):
            vf.run(f, t, w, a, p, out=o)

    ms_single = g.timed(one_by_one, 2, 1)
    vf.filter_batch(items, outs)
    torch.cuda.synchronize()
    agree, n_s, t_cpu = 0, 0, 0.0
    flops = 0
    for k, ((f, w), img) in enumerate(zip(assign, imgs)):
        H, W = img.shape[:2]
        rng = np.random.default_rng([3, k, 9])
        pix = np.concatenate([np.stack([rng.integers(0, H, 300), rng.integers(0, W, 300)], 1),
                              np.array([[0, 0], [0, W - 1], [H - 1, 0], [H - 1, W - 1]])]).astype(np.int32)
        t1 = time.time()
        want = oracle.run_filter(img, f, w, pixels=pix, nthreads=nthreads, **oracle_approx(f, BATCH_APPROX[f], w))
        t_cpu += time.time() - t1
        got = outs[k][torch.from_numpy(pix[:, 0]).long().cuda(), torch.from_numpy(pix[:, 1]).long().cuda()].cpu().numpy()
        agree += int((got == want).all(-1).sum())
        n_s += len(pix)
        flops += H * W * stream_flops_per_pixel(f, w, BATCH_APPROX[f])
    tf, fr = frac_of(flops, ms)
    log(f"config 3: batch {ms:.2f} ms, one call per image {ms_single:.2f} ms")
    return {"workload": "256 RGB uint8 images, area log-uniform 320x240..4000x3000, aspect 1/2..2, 15% "
                        "correlated impulses, random filter (VDF/DDF/AMNFE/EVMF) and window (3/5/7), minimax",
            "images": len(imgs), "pixels": pixels, "ms": round(ms, 3),
            "mpix_s": round(pixels / (ms * 1e-3) / 1e6, 1), "one_call_per_image_ms": round(ms_single, 3),
            "speedup_vs_one_call_per_image": round(ms_single / ms, 3), "graph_build_s": round(build_s, 3),
            "flagged_frac": round(st["flagged"] / max(1, st["windows"]), 6),
            "whole_batch_tflops": tf, "whole_batch_frac": fr,
            "oracle_agreement": round(agree / n_s, 7),
            "oracle_sample": f"{n_s} pixels: 300 seeded + 4 corners of every image"}


def config_quality(g, images, steps):
    """Section 4's comparison in the manner of Table 5: for each noise model
    at 10% (uncorrelated impulses, correlated impulses, Gaussian sigma 10 +
    correlated impulses), 8 seeded 512x512 uint8 images filtered 3x3 with the
    exact evaluation and with the paper's approximants (BVDF: Table 1's
    arccos polynomial; AMNFE: Table 3's rational; EVMF: Table 4's rational,
    both EVMF versions with the ENT cutoff T = 0.05 and AMNFE's with T = 10);
    mean and standard deviation over the set of the MAE / MSE / NCD
    percentages and of 100 T_exact / T_approx; the criteria kernel itself
    timed on the headline image."""
    from paper_1009_0959_amd import quality as Qd
    from paper_1009_0959_amd import synth
    torch, vf = g.torch, g.vf
    table = {}
    for model in synth.NOISE_MODELS:
        pairs = [(torch.from_numpy(c).cuda(), torch.from_numpy(n).cuda())
                 for c, n in synth.quality_set(model, 0.10, count=8)]
        for filt, spec, param in (("vdf", ("paper", 4), None), ("amnfe", ("rational", 4), None),
                                  ("evmf", ("paper", 4), 0.05)):
            row = Qd.compare(pairs, filt, 3, vf.Approx(*spec), param=param, repeats=3)["row"]
            table[f"{model}/{filt}"] = {k: [round(v[0], 4), round(v[1], 4)] for k, v in row.items()}
        log(f"quality table: {model} done")
    clean, img = images["c1"]
    H, W = img.shape[:2]
    clean_t = torch.from_numpy(clean).cuda()
    out = vf.filter_vdf(torch.from_numpy(img).cuda(), 5, vf.Approx(*HEADLINE))
    ms = g.timed(lambda: vf.quality(clean_t, out), steps, 1)
    q = vf.quality(clean_t, out)
    gbs = 6.0 * H * W / (ms * 1e-3) / 1e9
    return {"workload": "Table 5 layout: 3 noise models at 10%, 8 seeded 512x512 uint8 images each, 3x3 windows; "
                        "cells [mean %, sample std %] of 100 (E_exact - E_approx) / E_exact and 100 T_exact / T_approx",
            "table": table,
            "criteria_kernel": {"image": [H, W], "ms_per_call": round(ms, 4), "hbm_gb_s": round(gbs, 1),
                                "hbm_frac": round(gbs / 8000.0, 4), "mae": round(q["mae"], 6),
                                "mse": round(q["mse"], 6), "ncd": round(q["ncd"], 8),
                                "note": "one call includes the result copy and a stream synchronization"}}


def config4(g, images, nthreads, steps):
    """8192^2 uint16 (Gaussian sigma 400 + 25% correlated impulses), VDF and
    DDF 7x7 with the chord approximant against the exact-acosf kernels; the
    oracle on 4-pixel border bands and seeded interior pixels."""
    import oracle
    from paper_1009_0959_amd import synth
    torch = g.torch
    clean, img = images["c4"]
    H, W = img.shape[:2]
    t = torch.from_numpy(img).cuda()
    out = torch.empty_like(t)
    pix = sample_pixels(H, W, 40000, [4, 5])
    res, total_ms = {}, 0.0
    for filt in ("vdf", "ddf"):
        for spec, st in ((HEADLINE, steps), (("exact", 0), 2)):
            ms, k_ms, fl, got = g.measure(filt, t, 7, spec, out, st)
            want = oracle.run_filter(img, filt, 7, pixels=pix, nthreads=nthreads, **oracle_approx(filt, spec, 7))
            gs = got[pix[:, 0], pix[:, 1]]
            tf, fr = frac_of(H * W * stream_flops_per_pixel(filt, 7, spec), k_ms)
            res[f"{filt}7_{spec[0]}{spec[1] or ''}"] = {
                "ms": round(ms, 3), "mpix_s": round(H * W / (ms * 1e-3) / 1e6, 1), "kernel_ms": round(k_ms, 3),
                "kernel_tflops": tf, "kernel_frac": fr, "flagged_frac": round(fl, 6),
                "oracle_agreement": round(float((gs == want).all(-1).mean()), 7)}
            if spec == HEADLINE:
                total_ms += ms
            log(f"config 4 {filt} {spec}: {ms:.2f} ms (kernel {k_ms:.2f})")
    for filt in ("vdf", "ddf"):
        res[f"{filt}7_speedup_vs_exact"] = round(res[f"{filt}7_exact"]["ms"] / res[f"{filt}7_chord11"]["ms"], 3)
    return {"workload": "8192x8192 RGB uint16, Gaussian sigma 400 + 25% correlated impulses; VDF and DDF 7x7",
            "mpix_s_vdf_ddf_chord11": round(2 * H * W / (total_ms * 1e-3) / 1e6, 1),
            "oracle_sample": f"{len(pix)} pixels: 40000 seeded + 4-pixel border bands (same approximant)",
            "runs": res}


# ------------------------------------------------------------------ profile mode

PROFILES = {
    # name: (config image, filter, window, approximant)
    "vdf5": (1, "vdf", 5, HEADLINE), "vdf3": (1, "vdf", 3, HEADLINE),
    "vdf7u16": (4, "vdf", 7, HEADLINE), "ddf7u16": (4, "ddf", 7, HEADLINE),
    "ddf5": (1, "ddf", 5, HEADLINE),
    "amnfe5": (2, "amnfe", 5, ("minimax", 6)), "evmf5": (2, "evmf", 5, ("minimax", 6)),
    "amnfg5": (2, "amnfg", 5, ("minimax", 5)),
}


def profile(args) -> int:
    """Only one window kernel, --steps launches (re-check deferred and run
    separately), then a 256 MiB device-to-device copy that calibrates the HBM
    byte counters."""
    import torch
    from paper_1009_0959_amd import synth, vf
    cfg, filt, w, spec = PROFILES[args.profile]
    clean, noisy = synth.workload_image(cfg)
    H, W = noisy.shape[:2]
    img = torch.from_numpy(noisy).cuda()
    out = torch.empty_like(img)
    a_def = vf.Approx(*spec, defer=True)
    for _ in range(args.steps):
        vf.run(filt, img, w, a_def, out=out)
        vf.recheck_pending()
    torch.cuda.synchronize()
    st = vf.get_stats()
    src = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    es = noisy.itemsize
    print(json.dumps({"profile": args.profile, "steps": args.steps, "image": [H, W], "dtype": str(noisy.dtype),
                      "filter": filt, "window": w, "approximant": list(spec),
                      "strip_rows": st["tile_h"], "strip_cols": st["tile_w"], "workgroups": st["workgroups"],
                      "kernel_sources_sha256": kernel_sources_sha256(),
                      "algorithmic_flop_per_launch": H * W * stream_flops_per_pixel(filt, w, spec),
                      "input_bytes": H * W * 3 * es, "output_bytes": H * W * 3 * es,
                      "calibration_copy_bytes": 256 << 20}), flush=True)
    return 0


# ------------------------------------------------------------------ main

def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline and agreement checks")
    ap.add_argument("--no-configs", action="store_true", help="only the headline step")
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--profile", choices=sorted(PROFILES), default=None,
                    help="only one window kernel --steps times (re-check deferred), then a 256 MiB device "
                         "copy for counter calibration")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(pixels are independent given a (w-1)/2-row halo: an image would be split into row bands, one per GPU)",
              file=sys.stderr)
        return 2
    if args.profile:
        return profile(args)

    from paper_1009_0959_amd import synth
    H = W = args.size
    t0 = time.time()
    images = {"c1": synth.workload_image(1, height=H, width=W)}
    configs_on = not args.no_configs and not args.no_cpu
    if configs_on:
        # every workload is generated on the host before the GPU is touched
        # (the batch's images by worker processes)
        images["c0"] = synth.workload_image(0)
        images["c2"] = synth.workload_image(2)
        images["c4"] = synth.workload_image(4)
        images["c3"] = batch_images()
    log(f"generated the workloads in {time.time() - t0:.1f}s")
    clean, noisy = images["c1"]

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    g = Gpu()
    vf = g.vf
    img = torch.from_numpy(noisy).cuda()
    out3 = torch.empty_like(img)
    out5 = torch.empty_like(img)
    torch.cuda.synchronize()

    def step(spec):
        a = vf.Approx(*spec)
        vf.filter_vdf(img, 3, a, out=out3)
        vf.filter_vdf(img, 5, a, out=out5)

    # ---- the timed step (headline approximant)
    ms = g.timed(lambda: step(HEADLINE), args.steps, args.warmup)
    pixels = 2 * H * W
    value = pixels / (ms * 1e-3) / 1e6
    log(f"headline {HEADLINE}: {ms:.3f} ms/step, {value:.0f} Mpixel/s")

    # ---- the step's windows with the exact-acosf comparator, and the window kernels alone
    detail = {}
    for spec in (("exact", 0), HEADLINE):
        for w in (3, 5):
            t_ms, k_ms, fl, _ = g.measure("vdf", img, w, spec, out3, max(5, args.steps // 2))
            flops = H * W * stream_flops_per_pixel("vdf", w, spec)
            tf, fr = frac_of(flops, k_ms)
            detail[f"vdf{w}_{spec[0]}{spec[1] or ''}"] = {
                "mpix_s": round(H * W / (t_ms * 1e-3) / 1e6, 1), "ms": round(t_ms, 4), "kernel_ms": round(k_ms, 4),
                "kernel_tflops": tf, "kernel_frac": fr, "flagged_frac": round(fl, 6)}
    hk = f"{HEADLINE[0]}{HEADLINE[1]}"
    speedup = {f"{w}x{w}": round(detail[f"vdf{w}_exact"]["ms"] / detail[f"vdf{w}_{hk}"]["ms"], 3) for w in (3, 5)}

    # ---- roofline of the dominant kernel (streaming VDF 5x5), timed live with
    #      events around the window kernel alone (re-check deferred)
    dom_ms = detail[f"vdf5_{hk}"]["kernel_ms"]
    dom_flops = H * W * stream_flops_per_pixel("vdf", 5, HEADLINE)
    achieved = dom_flops / (dom_ms * 1e-3) / 1e12
    traffic, traffic_src = profiled_traffic() if (H, W) == (4096, 4096) else (None, "profiled at 4096x4096 only")
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32, 4), "traffic": traffic, "traffic_source": traffic_src,
                "algorithmic_bytes": 6 * H * W, "kernel": f"streaming VDF 5x5 {HEADLINE[0]}-{HEADLINE[1]}",
                "flop_per_launch": dom_flops, "kernel_ms": dom_ms,
                "frac_of_nonpacked_issue_peak": round(achieved / PEAK_FP32_NONPACKED, 4),
                "nonpacked_issue_peak": PEAK_FP32_NONPACKED}

    # ---- CPU oracle on the same step: the whole image at 3x3 and at 5x5 with
    #      the same approximant (about 5-20 s on 16 host threads)
    cpu = None
    nthreads = min(16, os.cpu_count() or 1)
    if not args.no_cpu:
        import oracle
        ap_o = oracle.angle_approx(*HEADLINE)
        t_cpu, px_cpu = 0.0, 0
        agree = []
        for w in (3, 5):
            t1 = time.time()
            o = oracle.run_filter(noisy, "vdf", w, angle=ap_o, nthreads=nthreads)
            t_cpu += time.time() - t1
            px_cpu += H * W
            vf.filter_vdf(img, w, vf.Approx(*HEADLINE), out=out3)
            torch.cuda.synchronize()
            agree.append(float((out3.cpu().numpy() == o).all(-1).mean()))
            log(f"oracle {w}x{w}: {t_cpu:.1f}s so far")
        cpu = {"value": round(px_cpu / t_cpu / 1e6, 4), "unit": "Mpixel/s", "cores": nthreads,
               "kind": "oracle",
               "sample": f"the whole {H}x{W} image at 3x3 and at 5x5 (one step), same approximant, FP64, "
                         f"{nthreads} OpenMP threads",
               "seconds": round(t_cpu, 2),
               "gpu_agreement_on_sample": [round(a, 7) for a in agree]}

    configs = None
    if configs_on:
        configs = {}
        steps = max(3, args.steps // 4)
        configs["c0_256_u8_vdf3_exact"] = config0(g, images, nthreads)
        configs["c1_approximant_sweep"] = config1_sweep(g, images, nthreads, steps)
        configs["f4_quality_table"] = config_quality(g, images, steps)
        del img, out3, out5
        configs["c2_mixed_noise_5x5"] = config2(g, images, nthreads, steps)
        configs["c4_8192_u16_7x7"] = config4(g, images, nthreads, steps)
        torch.cuda.empty_cache()
        configs["c3_uneven_batch"] = config3(g, images, nthreads, steps)

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "Mpixel/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{H}x{W} RGB uint8, 20% correlated impulse noise; VDF 3x3 + 5x5, "
                               f"minimax {HEADLINE[0]} degree {HEADLINE[1]} FP32 + FP64 near-tie re-check",
                   "image": [H, W], "windows": [3, 5], "approximant": list(HEADLINE)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "speedup_vs_exact_acosf": speedup,
        "detail": detail,
        "configs": configs,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
