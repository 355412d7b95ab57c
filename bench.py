#!/usr/bin/env python3
"""Benchmark: neural vs footprint-filtered analytic shading of a 1080p,
8-fabric synthetic G-buffer on one MI355X, with error against the FP64 oracle.

One timed step is one full frame (2,073,600 pixels) through the neural
shading path: G-buffer ingest, per-fabric staging, spatial encoding, the four
MFMA dense layers and albedo composition, in one kernel launch.  The
analytic footprint filter (256 samples per pixel) is timed the same way on the
same frame.  Before timing, the network is trained on GPU-generated batches
and targets (not timed).  Inputs are seeded and synthetic (see
fabric_inputs.py); they stand in for the paper's scenes.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
# Algorithmic work of one neural pixel: per-pixel multiply-adds of the four
# dense layers once the latent is folded into the first-layer bias:
# 40*64 + 64*64 + 69*64 + 64*4 = 11,328 MAC = 22,656 FLOP.
FLOP_PER_PIXEL = 2 * (40 * 64 + 64 * 64 + 69 * 64 + 64 * 4)
# G-buffer bytes per pixel in (fabric id u16 + 9 float32) and RGB out (3 float32).
BYTES_PER_PIXEL = 2 + 9 * 4 + 3 * 4


SHADE_SOURCES = ["common.hpp", "model.hpp", "mlp_tile.hpp", "mlp_tile32.hpp", "shade.hpp", "decode.hip"]
PROFILE = os.path.join(ROOT, "profiles", "decode32_bf16_fabric8_1080p.md")


def recorded_traffic():
    """HBM bytes per shading launch from the committed rocprofv3 record, if
    the shading kernel's sources are still the ones the counters measured."""
    import hashlib
    import re
    try:
        text = open(PROFILE).read()
    except OSError:
        return None, "no profile record"
    m = re.search(r"traffic-record: kernel=\S+ sources_sha256=([0-9a-f]+) fetch_kib=([0-9.]+) "
                  r"write_kib=([0-9.]+) fetch_scale=([0-9.]+) write_scale=([0-9.]+)", text)
    if not m:
        return None, "no traffic record"
    h = hashlib.sha256()
    for f in SHADE_SOURCES:
        with open(os.path.join(ROOT, "paper_2406_17782_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != m.group(1):
        return None, "kernel changed since the counters were taken"
    fetch = float(m.group(2)) * float(m.group(4)) * 1024
    write = float(m.group(3)) * float(m.group(5)) * 1024
    return fetch + write, "rocprofv3 FETCH_SIZE x %s + WRITE_SIZE x %s" % (m.group(4), m.group(5))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def time_launches(torch, fn, iters):
    """Average milliseconds per call of fn over `iters` calls, by HIP events
    on the current stream (the stream every library call is enqueued on)."""
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(iters):
        fn()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / iters


def rmse_stats(pred, ref):
    d = np.asarray(pred, np.float64) - np.asarray(ref, np.float64)
    return {"rmse": float(np.sqrt(np.mean(d * d))), "max_abs": float(np.abs(d).max())}


def cpu_baseline(orc, mats, g, params, budget_s):
    """The FP64 oracle's decoder forward and footprint filter on growing
    subsets of the frame until each leg has run about budget_s seconds."""
    import fabric_inputs as fi
    z = orc.encoder(params[fi.N_DECODER_PARAMS:].astype(np.float64), mats)
    P = params[: fi.N_DECODER_PARAMS].astype(np.float64)
    out = {}
    for leg in ("decoder", "filter256"):
        n = 2048 if leg == "decoder" else 128
        while True:
            idx = fi.subset_indices(g.n, n / g.n, 4321)
            sub = g.subset(idx)
            t0 = time.perf_counter()
            if leg == "decoder":
                orc.decoder_gbuffer(P, z, mats, sub)
            else:
                orc.filter_gbuffer(mats, sub, 256, 1, same_sample=False, pixel_index=idx)
            dt = time.perf_counter() - t0
            if dt >= budget_s or n >= g.n:
                out[leg] = (len(idx), dt)
                break
            n = min(g.n, int(n * max(2.0, 1.2 * budget_s / max(dt, 1e-3))))
    # One host thread: the decoder on a fixed 4,096-pixel subset.
    threads = orc.num_threads()
    orc.set_num_threads(1)
    try:
        idx = fi.subset_indices(g.n, 4096 / g.n, 4322)
        t0 = time.perf_counter()
        orc.decoder_gbuffer(P, z, mats, g.subset(idx))
        out["decoder_1thread"] = (len(idx), time.perf_counter() - t0)
    finally:
        orc.set_num_threads(threads)
    return out


def oracle_errors(args, torch, pkg, fi, fab, d, mats, g, rgb, gt_rgb):
    """RMSE and max abs of every result against the FP64 oracle's footprint
    filter (256 samples, same samples as the GPU) on a seeded pixel subset."""
    import oracle
    idx = fi.subset_indices(g.n, args.rmse_frac, 99)
    sub = g.subset(idx)
    t0 = time.perf_counter()
    o_comp, o_rgb, _, _ = oracle.filter_gbuffer(mats, sub, args.gt_samples, 4242, same_sample=True,
                                                pixel_index=idx)
    log(f"oracle reference on {len(idx)} px in {time.perf_counter() - t0:.1f}s")
    err = {f"neural_{k}": rmse_stats(v[:, idx], o_rgb) for k, v in rgb.items()}
    err["analytic_gpu_same_samples"] = rmse_stats(gt_rgb[:, idx], o_rgb)
    # The method without the network: one jittered footprint sample per pixel.
    one = torch.empty((3, g.n), dtype=torch.float32, device="cuda")
    pkg.fabric_gt_filtered(fab.ctx, d, 1, 777, one, None)
    err["analytic_1spp"] = rmse_stats(one.cpu().numpy()[:, idx], o_rgb)
    # The method without the network at the network's frame time: the
    # largest square sample count whose filter frame is no slower than the
    # BF16 decoder's (informational, as the paper's equal-time comparison).
    eqo = torch.empty_like(one)
    eq = {}
    for m in range(1, 8):
        ms_m = time_launches(torch, lambda: pkg.fabric_gt_filtered(fab.ctx, d, m * m, 778, eqo, None), 5)
        eq[m * m] = ms_m
    neural_ms = args.neural_ms
    n_eq = max([k for k, t in eq.items() if t <= neural_ms] or [1])
    pkg.fabric_gt_filtered(fab.ctx, d, n_eq, 778, eqo, None)
    err["analytic_equal_time"] = dict(rmse_stats(eqo.cpu().numpy()[:, idx], o_rgb), samples=n_eq,
                                      ms_per_frame=eq[n_eq], neural_bf16_ms=neural_ms,
                                      within_neural_time=eq[n_eq] <= neural_ms,
                                      filter_ms_by_samples=eq)
    # Monte-Carlo noise floor of the 256-sample reference (truth mode, N = 128^2).
    nf_idx = idx[:: max(1, len(idx) // 256)]
    _, t_rgb, _, _ = oracle.filter_gbuffer(mats, g.subset(nf_idx), 128 * 128, 4242, same_sample=False,
                                           pixel_index=nf_idx)
    sel = np.searchsorted(idx, nf_idx)
    err["reference256_vs_truth16384"] = rmse_stats(o_rgb[:, sel], t_rgb)
    err["neural_bf16_vs_truth16384"] = rmse_stats(rgb["bf16"][:, nf_idx], t_rgb)
    ratio_bf16_fp32 = err["neural_bf16"]["rmse"] / max(err["neural_fp32"]["rmse"], 1e-30)
    # Error by footprint radius (cells): filtering matters once the footprint
    # covers a sizeable part of a weave cell; below that one sample already
    # lands close to the footprint average.
    edges = [1e-3, 0.01, 0.05, 0.15, 0.3, 0.5]
    rad = sub.radius
    by_r = {}
    for lo, hi in zip(edges[:-1], edges[1:]):
        m = (rad >= lo) & (rad < hi)
        key = f"[{lo},{hi})"
        by_r[key] = {"pixels": int(m.sum())}
        for name, pred in (("neural_bf16", rgb["bf16"][:, idx]), ("neural_fp32", rgb["fp32"][:, idx]),
                           ("analytic_1spp", one.cpu().numpy()[:, idx])):
            by_r[key][name] = float(np.sqrt(np.mean((pred[:, m] - o_rgb[:, m]) ** 2)))
    # What the network gains over the method without it (one analytic sample
    # per pixel), over every pixel of the subset; the footprint bands above
    # are the breakdown.  The paper-size network's figures join in main().
    gain = {"pixels": int(len(idx)), "over": "every pixel of the seeded 1 % subset",
            "config_bf16_rmse": err["neural_bf16"]["rmse"],
            "analytic_1spp_rmse": err["analytic_1spp"]["rmse"]}
    gain["config_bf16_beats_1spp"] = gain["config_bf16_rmse"] < gain["analytic_1spp_rmse"]
    log(f"rmse bf16 {err['neural_bf16']['rmse']:.4g}, fp32 {err['neural_fp32']['rmse']:.4g}, "
        f"1spp {err['analytic_1spp']['rmse']:.4g}")

    return {"err": err, "by_r": by_r, "gain": gain, "ratio": ratio_bf16_fp32}


def precision_row_4k(args, torch, pkg, fi, fab, params):
    """3840x2160 G-buffer with 64 fabrics (patterns up to 16x16, radii
    log-uniform in [1e-4, 2] cells): shading throughput per precision, and
    each precision's error against the FP64 oracle's decoder with the same
    (trained) parameters on a seeded 0.25 % pixel subset."""
    import oracle
    wl = fi.WORKLOADS["fabric64_4k"]
    mats, g = wl.materials(), wl.gbuffer()
    fab.encode(mats)
    d = pkg.DeviceGBuffer.from_host(g)
    out = torch.empty((3, g.n), dtype=torch.float32, device="cuda")
    idx = fi.subset_indices(g.n, 0.0025, 77)
    z = oracle.encoder(params[fi.N_DECODER_PARAMS:].astype(np.float64), mats)
    _, o_rgb = oracle.decoder_gbuffer(params[: fi.N_DECODER_PARAMS], z, mats, g.subset(idx))
    row = {"pixels": g.n, "fabrics": len(mats), "subset_pixels": len(idx),
           "reference": "FP64 oracle decoder forward, same parameters"}
    for prec in ("bf16", "fp8", "fp32"):
        fn = lambda: pkg.fabric_shade_gbuffer(fab.ctx, d, pkg.PREC[prec], 0, 0, out)
        for _ in range(200 if prec != "fp32" else 20):   # clocks settle, as for the headline
            fn()
        t = time_launches(torch, fn, 100 if prec != "fp32" else 10)
        pred = out.cpu().numpy()[:, idx]
        row[prec] = {"ms_per_frame": t, "mpix_per_s": g.n / (t * 1e-3) / 1e6,
                     "hbm_gbs": BYTES_PER_PIXEL * g.n / (t * 1e-3) / 1e9, **rmse_stats(pred, o_rgb)}
        log(f"4k 64 fabrics {prec}: {t * 1e3:.1f} us/frame, rmse {row[prec]['rmse']:.4g}")
    del d, out
    return row


def c1_row(args, torch, pkg, fi):
    """The small plain-method case: a 128x128 G-buffer of the plain weave
    (seeded yarn parameters), the decoder with seeded weights in FP32 and
    BF16, and the analytic filter at 64 stratified samples; the decoders'
    largest error against the FP64 oracle's forward of the same weights over
    every pixel."""
    import oracle
    wl = fi.WORKLOADS["plain128"]
    mats, g = wl.materials(), wl.gbuffer()
    params = fi.init_params(5, bias_scale=0.05)
    fab = pkg.Fabric(0, seed=wl.seed())
    try:
        fab.set_params(params)
        fab.encode(mats)
        d = pkg.DeviceGBuffer.from_host(g)
        out = torch.empty((3, g.n), dtype=torch.float32, device="cuda")
        z = oracle.encoder(params[fi.N_DECODER_PARAMS:].astype(np.float64), mats)
        _, o_rgb = oracle.decoder_gbuffer(params[: fi.N_DECODER_PARAMS], z, mats, g)
        row = {"pixels": g.n, "fabrics": 1, "weights": "seeded"}
        for prec in ("fp32", "bf16"):
            fn = lambda: pkg.fabric_shade_gbuffer(fab.ctx, d, pkg.PREC[prec], 0, 0, out)
            for _ in range(200):
                fn()
            t = time_launches(torch, fn, 200)
            rgb = out.cpu().numpy()
            row[prec] = {"us_per_frame": t * 1e3, "mpix_per_s": g.n / (t * 1e-3) / 1e6,
                         "max_abs_vs_fp64_oracle": float(np.abs(rgb - o_rgb).max())}
        a = torch.empty((3, g.n), dtype=torch.float32, device="cuda")
        filt = lambda: pkg.fabric_gt_filtered(fab.ctx, d, 64, 4242, a, None)
        for _ in range(20):
            filt()
        t = time_launches(torch, filt, 50)
        row["analytic_64"] = {"us_per_frame": t * 1e3, "mpix_per_s": g.n / (t * 1e-3) / 1e6}
        log(f"c1 128x128: fp32 {row['fp32']['us_per_frame']:.1f} us, bf16 "
            f"{row['bf16']['us_per_frame']:.1f} us, filter 64 {row['analytic_64']['us_per_frame']:.1f} us")
        return row
    finally:
        fab.close()


def hybrid_class_errors(args, torch, pkg, fi, fab, mats, hg):
    """Per-class error of the first hybrid frame against the FP64 oracle's
    filter (256 samples, seeded like the frame's fallback) on a seeded 1 %
    of its pixels: the decoder's pixels and the filter's pixels apart."""
    import oracle
    g0 = fi.jitter_gbuffer(hg, 50_000)
    d0 = pkg.DeviceGBuffer.from_host(g0)
    out = torch.empty((3, g0.n), dtype=torch.float32, device="cuda")
    pkg.fabric_shade_gbuffer(fab.ctx, d0, pkg.FABRIC_BF16, args.gt_samples, 0, out)
    rgb = out.cpu().numpy()
    idx = fi.subset_indices(g0.n, 0.01, 98)
    _, o_rgb, _, _ = oracle.filter_gbuffer(mats, g0.subset(idx), args.gt_samples, 0,
                                           same_sample=True, pixel_index=idx)
    oor = (g0.radius[idx] > np.float32(1.0)) | (g0.wo_z[idx] < np.float32(0.05))
    res = {"subset_pixels": int(idx.size), "reference": "FP64 oracle filter, 256 same samples"}
    for name, m in (("decoder_bf16", ~oor), ("filter_fallback", oor)):
        res[name] = dict(rmse_stats(rgb[:, idx][:, m], o_rgb[:, m]), pixels=int(m.sum()))
    log(f"hybrid rmse: decoder {res['decoder_bf16']['rmse']:.4g}, "
        f"fallback {res['filter_fallback']['rmse']:.3g}")
    return res


def train_row_2p20(args, torch, pkg, fab):
    """Training steps at the training workload's batch of 2^20 generated
    samples (targets from the filter at 256 samples, BF16 decoder), timed by
    events after warmup; the trained state is restored afterwards."""
    blob = pkg.fabric_save(fab.ctx)
    step = lambda s: fab.train_step(seed=3_000_000 + s, batch=1 << 20, gt_samples=args.gt_samples,
                                    prec=pkg.FABRIC_BF16, lr=1e-4, want_loss=False)
    for s in range(5):
        step(s)
    torch.cuda.synchronize()
    k = [0]

    def one():
        step(5 + k[0])
        k[0] += 1
    ms = time_launches(torch, one, 20)
    pkg.fabric_load(fab.ctx, blob)
    log(f"train step 2^20: {ms:.2f} ms")
    return {"ms_per_step": ms, "batch": 1 << 20, "gt_samples": args.gt_samples,
            "samples_per_s": (1 << 20) / (ms * 1e-3), "prec": "bf16 decoder, FP32 masters, FP64 Adam"}


def visibility_row(args, torch, pkg, fi, wl, mats, g, d, neural_ms):
    """The analytic model with inter-yarn visibility (V of Eq. (3)-(4)): the
    filter's cost on the 1080p frame, a network trained on visibility
    targets (same schedule as the main one), and the errors of that network
    and of one analytic sample against the FP64 oracle's filter with V on
    the seeded 1 % subset."""
    import oracle
    fab = pkg.Fabric(0, seed=wl.seed())
    try:
        fab.encode(mats)
        fab.set_visibility(True)
        steps = args.train_steps
        loss = None
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record()
        for s in range(steps):
            lr = args.train_lr * 0.5 * (1.0 + math.cos(math.pi * s / max(1, steps)))
            loss = fab.train_step(seed=1_000_000 + s, batch=args.train_batch,
                                  gt_samples=args.gt_samples, prec=pkg.FABRIC_BF16, lr=lr,
                                  want_loss=(s == steps - 1))
        ev1.record()
        torch.cuda.synchronize()
        train_ms = ev0.elapsed_time(ev1) / max(1, steps)
        fab.encode(mats)
        out = torch.empty((3, g.n), dtype=torch.float32, device="cuda")
        pkg.fabric_shade_gbuffer(fab.ctx, d, pkg.PREC["bf16"], 0, 0, out)
        rgb = out.cpu().numpy()
        filt = lambda: pkg.fabric_gt_filtered(fab.ctx, d, args.gt_samples, 4242, out, None)
        filt()
        f_ms = time_launches(torch, filt, args.analytic_steps)
        gt = out.cpu().numpy()
        pkg.fabric_gt_filtered(fab.ctx, d, 1, 777, out, None)
        one = out.cpu().numpy()
        res = {"filter_ms_per_frame": f_ms, "filter_mpix_per_s": g.n / (f_ms * 1e-3) / 1e6,
               "neural_bf16_over_filter": f_ms / neural_ms, "train_ms_per_step": train_ms,
               "train_steps": steps, "loss_last": loss,
               "definition": "height texels 16/cell from the yarn slopes, 32-step march (2 cells)"}
        if not args.no_rmse:
            idx = fi.subset_indices(g.n, args.rmse_frac, 99)
            sub = g.subset(idx)
            _, o_rgb, _, _ = oracle.filter_gbuffer(mats, sub, args.gt_samples, 4242,
                                                   same_sample=True, pixel_index=idx,
                                                   visibility=True)
            res["rmse_vs_fp64_oracle"] = {
                "neural_bf16": rmse_stats(rgb[:, idx], o_rgb),
                "analytic_gpu_same_samples": rmse_stats(gt[:, idx], o_rgb),
                "analytic_1spp": rmse_stats(one[:, idx], o_rgb)}
            big = sub.radius >= 0.15
            res["radius_ge_0.15"] = {
                "pixels": int(big.sum()),
                "neural_bf16_rmse": float(np.sqrt(np.mean((rgb[:, idx][:, big] - o_rgb[:, big]) ** 2))),
                "analytic_1spp_rmse": float(np.sqrt(np.mean((one[:, idx][:, big] - o_rgb[:, big]) ** 2)))}
        log(f"visibility: filter {f_ms:.2f} ms/frame, train {train_ms:.2f} ms/step" +
            ("" if args.no_rmse else
             f", rmse bf16 {res['rmse_vs_fp64_oracle']['neural_bf16']['rmse']:.4g}, "
             f"1spp {res['rmse_vs_fp64_oracle']['analytic_1spp']['rmse']:.4g}"))
        return res
    finally:
        fab.close()


def btdf_row(args, torch, pkg, fi):
    """Transmission (light below the fabric, Sec. 4.2's BTDF queries): a
    network trained like the main one on batches with half the samples lit
    from below (targets with k = 1000), shaded on the 1080p frame whose
    pixels are half lit from below; the decoder's and the filter's cost on
    that frame, and RMSE against the FP64 oracle's filter on a seeded 1 %,
    for the pixels lit from above and from below apart."""
    import oracle
    wl = fi.WORKLOADS["btdf_1080p"]
    mats, g = wl.materials(), wl.gbuffer()
    d = pkg.DeviceGBuffer.from_host(g)
    fab = pkg.Fabric(0, seed=wl.seed())
    try:
        fab.encode(mats)
        steps = args.train_steps
        loss = None
        for s in range(steps):
            lr = args.train_lr * 0.5 * (1.0 + math.cos(math.pi * s / max(1, steps)))
            loss = fab.train_step(seed=5_000_000 + s, batch=args.train_batch,
                                  gt_samples=args.gt_samples, prec=pkg.FABRIC_BF16, lr=lr,
                                  btdf_frac=0.5, want_loss=(s == steps - 1))
        fab.encode(mats)
        out = torch.empty((3, g.n), dtype=torch.float32, device="cuda")
        shade = lambda: pkg.fabric_shade_gbuffer(fab.ctx, d, pkg.PREC["bf16"], 0, 0, out)
        for _ in range(args.warmup // 2):
            shade()
        s_ms = time_launches(torch, shade, args.steps // 2)
        rgb = out.cpu().numpy()
        filt = lambda: pkg.fabric_gt_filtered(fab.ctx, d, args.gt_samples, 4242, out, None)
        filt()
        f_ms = time_launches(torch, filt, args.analytic_steps)
        pkg.fabric_gt_filtered(fab.ctx, d, 1, 777, out, None)
        one = out.cpu().numpy()
        res = {"workload": "btdf_1080p", "below_frac": float((g.wi_z < 0).mean()),
               "train_steps": steps, "train_btdf_frac": 0.5, "loss_last": loss,
               "bf16_ms_per_frame": s_ms, "bf16_mpix_per_s": g.n / (s_ms * 1e-3) / 1e6,
               "filter_ms_per_frame": f_ms, "neural_bf16_over_filter": f_ms / s_ms}
        if not args.no_rmse:
            idx = fi.subset_indices(g.n, args.rmse_frac, 99)
            _, o_rgb, _, _ = oracle.filter_gbuffer(mats, g.subset(idx), args.gt_samples, 4242,
                                                   same_sample=True, pixel_index=idx)
            below = g.wi_z[idx] < 0
            res["rmse_vs_fp64_oracle"] = {}
            for name, m in (("lit_from_above", ~below), ("lit_from_below", below)):
                res["rmse_vs_fp64_oracle"][name] = {
                    "pixels": int(m.sum()),
                    "neural_bf16": rmse_stats(rgb[:, idx][:, m], o_rgb[:, m]),
                    "analytic_1spp": rmse_stats(one[:, idx][:, m], o_rgb[:, m])}
            e = res["rmse_vs_fp64_oracle"]
            log(f"btdf: bf16 {s_ms * 1e3:.1f} us/frame, filter {f_ms:.2f} ms; rmse above "
                f"{e['lit_from_above']['neural_bf16']['rmse']:.4g} (1spp "
                f"{e['lit_from_above']['analytic_1spp']['rmse']:.4g}), below "
                f"{e['lit_from_below']['neural_bf16']['rmse']:.4g} (1spp "
                f"{e['lit_from_below']['analytic_1spp']['rmse']:.4g})")
        return res
    finally:
        fab.close()


PAPER_FLOP_PER_PIXEL = 2 * (24 * 64 + 64 * 64 + 69 * 64 + 3 * 64 * 64 + 64 * 4)   # 45,184
# Training of the paper-size decoder per sample: forward 26,688 MAC (latent
# columns included), input gradients 20,736 MAC, weight gradients 22,592 MAC.
PAPER_TRAIN_FLOP_PER_SAMPLE = 2 * (26688 + 20736 + 22592)
FP32_UNPACKED_PEAK_TFLOPS = 78.6   # half of 157.3, which counts packed FP32 FMAs


def paper_decoder_row(args, torch, pkg, fi, mats, g, d):
    """The decoder at the paper's own form (latent 64, one-blob 24, 2 + 5
    layers of width 64 with a residual skip, leaky ReLU), BF16 on the 1080p
    frame with seeded weights and latents (the training row trains its own);
    its error against the FP64 oracle's forward of the same weights on a
    seeded 1 %."""
    fab = pkg.Fabric(0, seed=7)
    try:
        fab.encode(mats)
        params = fi.init_paper_params(4500, bias_scale=0.05)
        z = fi.random_latents(len(mats), 4501, dim=64)
        pkg.fabric_paper_prepare(fab.ctx, torch.from_numpy(params).cuda(), torch.from_numpy(z).cuda())
        out = torch.empty((3, g.n), dtype=torch.float32, device="cuda")
        fp16 = lambda: pkg.fabric_paper_shade(fab.ctx, d, out, "fp16")
        for _ in range(args.warmup // 2):
            fp16()
        ms16 = time_launches(torch, fp16, args.steps // 2)
        rgb16 = out.cpu().numpy()
        shade = lambda: pkg.fabric_paper_shade(fab.ctx, d, out, "bf16")
        for _ in range(args.warmup // 4):
            shade()
        ms = time_launches(torch, shade, args.steps // 2)
        tflops = PAPER_FLOP_PER_PIXEL * g.n / (ms * 1e-3) / 1e12
        res = {"ms_per_frame": ms, "mpix_per_s": g.n / (ms * 1e-3) / 1e6,
               "algorithmic_flop_per_pixel": PAPER_FLOP_PER_PIXEL, "tflops": tflops,
               "mfma_frac": tflops / BF16_PEAK_TFLOPS, "weights": "seeded",
               "fp16_ms_per_frame": ms16,
               "fp16_mfma_frac": PAPER_FLOP_PER_PIXEL * g.n / (ms16 * 1e-3) / 1e12 / BF16_PEAK_TFLOPS,
               "paper_rtx3090_decoder_ms_per_1080p_frame": [13.6, 14.4]}
        if not args.no_rmse:
            import oracle
            idx = fi.subset_indices(g.n, args.rmse_frac, 98)
            _, o_rgb = oracle.paper_decoder_gbuffer(params, z, mats, g.subset(idx))
            rgb = out.cpu().numpy()[:, idx]
            res["rel_l2_vs_fp64_oracle"] = float(np.linalg.norm(rgb - o_rgb) / np.linalg.norm(o_rgb))
            res["rmse_vs_fp64_oracle"] = rmse_stats(rgb, o_rgb)
            r16 = rgb16[:, idx]
            res["fp16_rel_l2_vs_fp64_oracle"] = float(np.linalg.norm(r16 - o_rgb) / np.linalg.norm(o_rgb))
        log(f"paper-size decoder: bf16 {ms * 1e3:.1f} us/frame, {tflops:.0f} TFLOP/s "
            f"({100 * tflops / BF16_PEAK_TFLOPS:.1f} % of bf16 peak); fp16 {ms16 * 1e3:.1f} us")
        return res
    finally:
        fab.close()


def train_paper_network(args, torch, pkg, fi, mats, steps, one_blob=True, fused=True,
                        encoder=False):
    """A paper-size decoder trained on `mats` (one latent of 64 per fabric
    trained as a parameter, or with encoder=True the paper-size encoder
    trained beside it; forward and backward in the precision
    --paper-train-prec names (BF16 operands on the matrix cores, or FP32 on
    the vector units), FP32 weight gradients and masters; generated batches
    of 2^16 samples with 256-sample targets; Adam with the main network's
    cosine-decayed rate).  Returns the open context and the training record."""
    fab = pkg.Fabric(0, seed=4600)
    fab.encode(mats)
    params = fi.init_paper_params(5, bias_scale=0.0)
    if encoder:
        enc = fi.init_paper_encoder_params(6, bias_scale=0.0)
        pkg.fabric_paper_prepare_encoder(fab.ctx, torch.from_numpy(params).cuda(),
                                         torch.from_numpy(enc).cuda())
    else:
        z = fi.random_latents(len(mats), 6, scale=0.1, dim=64)
        pkg.fabric_paper_prepare(fab.ctx, torch.from_numpy(params).cuda(),
                                 torch.from_numpy(z).cuda())
    pkg.fabric_paper_set_footprint_encoding(fab.ctx, one_blob)
    pkg.fabric_paper_set_spatial_fusion(fab.ctx, fused)
    batch = 1 << 16
    prec = pkg.PREC[args.paper_train_prec]
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        lr = args.train_lr * 0.5 * (1.0 + math.cos(math.pi * s / max(1, steps)))
        want = s == 0 or s == steps - 1
        l = pkg.fabric_paper_train_step(fab.ctx, None, None,
                                        dict(batch=batch, gt_samples=args.gt_samples,
                                             seed=3_000_000 + s, lr=lr, prec=prec),
                                        want_loss=want)
        if want:
            losses.append(l)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    ms = train_s / max(1, steps) * 1e3
    tflops = PAPER_TRAIN_FLOP_PER_SAMPLE * batch / (ms * 1e-3) / 1e12 if steps else None
    rec = {"train_steps": steps, "train_batch": batch, "train_prec": args.paper_train_prec,
           "train_ms_per_step": ms, "train_s": train_s,
           # The whole step (batch, 256-sample targets, forward, backward,
           # weight gradients, Adam) against the training's algorithmic FLOPs;
           # for FP32 training against the peak of unpacked FP32 FMAs (the
           # library uses no packed FP32 instructions).
           "algorithmic_flop_per_sample": PAPER_TRAIN_FLOP_PER_SAMPLE,
           "step_tflops": tflops,
           "step_frac_of_unpacked_fp32": (tflops / FP32_UNPACKED_PEAK_TFLOPS
                                          if steps and args.paper_train_prec == "fp32" else None),
           "loss_first": losses[0] if losses else None, "loss_last": losses[-1] if losses else None,
           "footprint_encoding": "one-blob" if one_blob else "none", "spatial_fusion": fused,
           "latents": "paper-size encoder" if encoder else "one per fabric, trained as parameters"}
    return fab, rec


def subset_reference(args, fi, mats, g):
    """The main section's seeded 1 % and the oracle's filter on it."""
    import oracle
    idx = fi.subset_indices(g.n, args.rmse_frac, 99)
    sub = g.subset(idx)
    _, o_rgb, _, _ = oracle.filter_gbuffer(mats, sub, args.gt_samples, 4242, same_sample=True,
                                           pixel_index=idx)
    return idx, sub, o_rgb


def errors_by_radius(preds, o_rgb, radius):
    edges = [1e-3, 0.01, 0.05, 0.15, 0.3, 0.5]
    by_r = {}
    for lo, hi in zip(edges[:-1], edges[1:]):
        m = (radius >= lo) & (radius < hi)
        by_r[f"[{lo},{hi})"] = dict(
            pixels=int(m.sum()),
            **{k: float(np.sqrt(np.mean((v[:, m] - o_rgb[:, m]) ** 2))) for k, v in preds.items()})
    return by_r


def paper_training_row(args, torch, pkg, fi, mats, g, d, config_rgb):
    """The paper-size decoder trained on the 1080p workload's fabrics; its
    FP16 and BF16 frames against the oracle's filter on the main section's
    seeded 1 %, by footprint radius, beside the config-size network and one
    analytic sample."""
    fab, res = train_paper_network(args, torch, pkg, fi, mats, args.paper_train_steps)
    try:
        out = torch.empty((3, g.n), dtype=torch.float32, device="cuda")
        fp16 = lambda: pkg.fabric_paper_shade(fab.ctx, d, out, "fp16")
        for _ in range(100):
            fp16()
        res["fp16_ms_per_frame"] = time_launches(torch, fp16, 100)
        rgb16 = out.cpu().numpy()
        pkg.fabric_paper_shade(fab.ctx, d, out, "bf16")
        rgb_bf = out.cpu().numpy()
        log(f"paper-size training: {res['train_steps']} steps in {res['train_s']:.1f}s, loss "
            f"{res['loss_first']} -> {res['loss_last']}")
        if not args.no_rmse and res["train_steps"] > 0:
            idx, sub, o_rgb = subset_reference(args, fi, mats, g)
            one = torch.empty((3, g.n), dtype=torch.float32, device="cuda")
            pkg.fabric_gt_filtered(fab.ctx, d, 1, 777, one, None)
            preds = {"paper_fp16": rgb16[:, idx], "paper_bf16": rgb_bf[:, idx],
                     "config_bf16": config_rgb[:, idx], "analytic_1spp": one.cpu().numpy()[:, idx]}
            res["rmse_vs_fp64_oracle"] = {k: rmse_stats(v, o_rgb) for k, v in preds.items()}
            res["rmse_by_footprint_radius"] = errors_by_radius(preds, o_rgb, sub.radius)
            e = res["rmse_vs_fp64_oracle"]
            res["paper_fp16_beats_1spp"] = e["paper_fp16"]["rmse"] < e["analytic_1spp"]["rmse"]
            log(f"paper-size network rmse fp16 {e['paper_fp16']['rmse']:.4g}, bf16 "
                f"{e['paper_bf16']['rmse']:.4g}; config bf16 {e['config_bf16']['rmse']:.4g}, "
                f"1spp {e['analytic_1spp']['rmse']:.4g}")
        return res
    finally:
        fab.close()


def ablation_row(args, torch, pkg, fi, mats, g, d):
    """Sec. 5 "Ablation study": three paper-size networks trained alike -
    the paper's, one without the one-blob footprint encoding ("Encoding of
    footprint") and one without the spatial fusion stage ("Spatial
    fusion"); their FP16 frames against the oracle's filter on the main
    section's seeded 1 %, overall and by footprint radius."""
    steps = args.ablation_train_steps
    res = {"train_steps": steps, "train_batch": 1 << 16}
    ref = None if args.no_rmse or steps == 0 else subset_reference(args, fi, mats, g)
    preds = {}
    for name, one_blob, fused in (("paper", True, True), ("unencoded", False, True),
                                  ("unfused", True, False)):
        fab, rec = train_paper_network(args, torch, pkg, fi, mats, steps, one_blob, fused)
        try:
            out = torch.empty((3, g.n), dtype=torch.float32, device="cuda")
            pkg.fabric_paper_shade(fab.ctx, d, out, "fp16")
            res[name] = {"loss_last": rec["loss_last"], "train_s": rec["train_s"]}
            if ref is not None:
                preds[name] = out.cpu().numpy()[:, ref[0]]
                res[name]["rmse"] = rmse_stats(preds[name], ref[2])
        finally:
            fab.close()
    if ref is not None:
        res["rmse_by_footprint_radius"] = errors_by_radius(preds, ref[2], ref[1].radius)
        e = {k: res[k]["rmse"]["rmse"] for k in preds}
        res["encoding_lowers_rmse"] = e["paper"] < e["unencoded"]
        res["fusion_lowers_rmse"] = e["paper"] < e["unfused"]
        log(f"ablations: paper {e['paper']:.4g}, without one-blob {e['unencoded']:.4g}, "
            f"without spatial fusion {e['unfused']:.4g}")
    return res


def slot_frame(torch, d, slot):
    """The G-buffer `d` with every pixel showing fabric `slot`."""
    import dataclasses
    fid = torch.from_numpy(np.full(d.n, slot, dtype=np.int16)).to("cuda").view(torch.uint16)
    return dataclasses.replace(d, fabric_id=fid)


def paper_encoder_row(args, torch, pkg, fi, d):
    """The paper-size network with its encoder (Sec. 4.2 "Encoder"), encoder
    and decoder trained together on the interpolation row's 64 twill
    variants; then 8 of those variants and 8 new draws of the same family,
    encoded by one call and each shaded (FP16) over a 1080p frame showing it
    alone, against the 256-sample filter: the encoder lets fabrics it never
    saw be shaded from their parameters."""
    train = fi.sweep_training_set(64, 4400)
    fab, rec = train_paper_network(args, torch, pkg, fi, train, args.paper_encoder_train_steps,
                                   encoder=True)
    try:
        seen = train[:8]
        unseen = fi.sweep_training_set(8, 4400, variant_seed=4499)
        fab.encode(seen + unseen)
        pkg.fabric_paper_encode(fab.ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(100):
            pkg.fabric_paper_encode(fab.ctx)
        torch.cuda.synchronize()
        encode_ms = (time.perf_counter() - t0) / 100 * 1e3
        out = torch.empty((3, d.n), dtype=torch.float32, device="cuda")
        rel = lambda x, y: float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-30))
        errs = []
        for k in range(16):
            f = slot_frame(torch, d, k)
            pkg.fabric_paper_shade(fab.ctx, f, out, "fp16")
            nn = out.cpu().numpy().astype(np.float64)
            pkg.fabric_gt_filtered(fab.ctx, f, args.gt_samples, 4242, out, None)
            errs.append(rel(nn, out.cpu().numpy().astype(np.float64)))
        rec["generalisation"] = {
            "seen_mean": float(np.mean(errs[:8])), "seen_max": float(np.max(errs[:8])),
            "unseen_mean": float(np.mean(errs[8:])), "unseen_max": float(np.max(errs[8:])),
            "metric": "relative L2 of the FP16 frame against the 256-sample filter"}
        rec["training_table"] = "64 twill variants"
        rec["encode_16_fabrics_ms"] = encode_ms
        log(f"paper-size encoder: loss {rec['loss_first']} -> {rec['loss_last']}; seen "
            f"{rec['generalisation']['seen_mean']:.4f}, unseen {rec['generalisation']['unseen_mean']:.4f}")
        return rec
    finally:
        fab.close()


def interp_row(args, torch, pkg, fi, g, d):
    """Latent interpolation study (Sec. 5 "Interpolation") on the 1080p
    frame's geometry: a second network trained on variants of one twill whose
    roughness and height-field scale span [0.15, 0.95]; latents encoded at
    0.2 and 0.8, blended on the GPU at 0.3 and 0.6 and extrapolated to 0.9.
    Every pixel of a frame shows one slot; each blended frame is compared with
    the directly encoded one and with the analytic filter at 256 samples."""
    fab = pkg.Fabric(0, seed=4343)
    try:
        fab.encode(fi.sweep_training_set(64, 4400))
        steps = args.interp_train_steps
        for s in range(steps):
            lr = args.train_lr * 0.5 * (1.0 + math.cos(math.pi * s / max(1, steps)))
            fab.train_step(seed=2_000_000 + s, batch=1 << 17, gt_samples=args.gt_samples,
                           prec=pkg.FABRIC_BF16, lr=lr, want_loss=(s == steps - 1))
        pts = fi.INTERP_ENDPOINTS + fi.INTERP_POINTS
        # The trained twill itself, the other parameter held at 0.5 (inside
        # the training range).
        table = (fi.parameter_sweep("alpha", pts, 4400, other=0.5) +
                 fi.parameter_sweep("beta", pts, 4400, other=0.5))
        fab.encode(table)
        p0, p1 = fi.INTERP_ENDPOINTS
        dst, a, b, t = [], [], [], []
        for base in (0, 5):
            for k, p in enumerate(fi.INTERP_POINTS):
                dst.append(base + 2 + k)
                a.append(base)
                b.append(base + 1)
                t.append((p - p0) / (p1 - p0))

        def frame(slot):
            return slot_frame(torch, d, slot)

        frames = [frame(k) for k in range(len(table))]
        out = torch.empty((3, g.n), dtype=torch.float32, device="cuda")

        def shade_all(slots):
            res = {}
            for k in slots:
                pkg.fabric_shade_gbuffer(fab.ctx, frames[k], pkg.PREC["bf16"], 0, 0, out)
                res[k] = out.cpu().numpy().astype(np.float64)
            return res

        direct = shade_all(range(len(table)))
        gt = {}
        for k in dst:
            pkg.fabric_gt_filtered(fab.ctx, frames[k], args.gt_samples, 4242, out, None)
            gt[k] = out.cpu().numpy().astype(np.float64)
        # The blend call (host arrays in, one copy, blend + refold launches).
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(100):
            fab.lerp_latents(dst, a, b, t)
        torch.cuda.synchronize()
        lerp_ms = (time.perf_counter() - t0) / 100 * 1e3
        blended = shade_all(dst)
        shade = lambda: pkg.fabric_shade_gbuffer(fab.ctx, frames[dst[0]], pkg.PREC["bf16"], 0, 0, out)
        for _ in range(300):
            shade()
        shade_ms = time_launches(torch, shade, 200)
        rel = lambda x, y: float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-30))
        points = {}
        for k, field in enumerate(("alpha", "beta")):
            for j, p in enumerate(fi.INTERP_POINTS):
                slot = 5 * k + 2 + j
                near = 5 * k + (0 if abs(p - p0) < abs(p - p1) else 1)
                points[f"{field}={p}"] = {
                    "t": t[3 * k + j],
                    "blend_vs_direct": rel(blended[slot], direct[slot]),
                    "nearest_endpoint_vs_direct": rel(direct[near], direct[slot]),
                    "direct_vs_analytic": rel(direct[slot], gt[slot]),
                    "blend_vs_analytic": rel(blended[slot], gt[slot]),
                }
        log("interpolation: " + ", ".join(f"{k} {v['blend_vs_direct']:.4f}" for k, v in points.items()))
        # Unseen parameters: 8 variants from the training table and 8 new
        # draws of the same family, each shaded over the frame and compared
        # with the analytic filter.
        seen = fi.sweep_training_set(64, 4400)[:8]
        unseen = fi.sweep_training_set(8, 4400, variant_seed=4499)
        fab.encode(seen + unseen)
        frames = [frame(k) for k in range(16)]
        errs = []
        for k in range(16):
            pkg.fabric_shade_gbuffer(fab.ctx, frames[k], pkg.PREC["bf16"], 0, 0, out)
            nn = out.cpu().numpy().astype(np.float64)
            pkg.fabric_gt_filtered(fab.ctx, frames[k], args.gt_samples, 4242, out, None)
            errs.append(rel(nn, out.cpu().numpy().astype(np.float64)))
        general = {"seen_mean": float(np.mean(errs[:8])), "seen_max": float(np.max(errs[:8])),
                   "unseen_mean": float(np.mean(errs[8:])), "unseen_max": float(np.max(errs[8:])),
                   "metric": "relative L2 of the BF16 frame against the 256-sample filter"}
        log(f"generalisation: seen {general['seen_mean']:.4f}, unseen {general['unseen_mean']:.4f}")
        return {"train_steps": steps, "train_batch": 1 << 17, "training_table": "64 twill variants",
                "generalisation": general,
                "lerp_call_ms": lerp_ms, "blends_per_call": len(dst),
                "bf16_ms_per_frame_after_edit": shade_ms,
                "metric": "relative L2 over a 1080p frame showing one slot",
                "points": points}
    finally:
        fab.close()


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    # The GPU's clocks settle only after several hundred back-to-back frames
    # (about 50 ms of shading); fewer warmup frames under-report throughput.
    ap.add_argument("--warmup", type=int, default=1500)
    ap.add_argument("--train-steps", type=int, default=6000)
    ap.add_argument("--train-batch", type=int, default=1 << 18)
    ap.add_argument("--train-lr", type=float, default=1e-2)
    ap.add_argument("--gt-samples", type=int, default=256)
    ap.add_argument("--interp-train-steps", type=int, default=12000,
                    help="training steps of the latent interpolation row's network")
    ap.add_argument("--paper-train-steps", type=int, default=96000,
                    help="training steps (2^16 samples each) of the paper-size decoder's row")
    ap.add_argument("--paper-encoder-train-steps", type=int, default=24000,
                    help="training steps (2^16 samples each) of the paper-size encoder's row")
    ap.add_argument("--paper-train-prec", choices=("bf16", "fp32"), default="bf16",
                    help="forward/backward precision of the paper-size network's training")
    ap.add_argument("--ablation-train-steps", type=int, default=12000,
                    help="training steps of each network of the ablation row")
    ap.add_argument("--analytic-steps", type=int, default=10)
    ap.add_argument("--rmse-frac", type=float, default=0.01)
    ap.add_argument("--cpu-budget", type=float, default=8.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-rows", action="store_true", help="skip the secondary rows")
    ap.add_argument("--rows", default="all",
                    help="comma-separated secondary rows to run (default: all)")
    ap.add_argument("--no-rmse", action="store_true", help="skip the oracle error section")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 512 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the shading path has no "
              "cross-GPU exchange and every box in this setup has a single MI355X.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import fabric_inputs as fi
    import paper_2406_17782_amd as pkg

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    wl = fi.WORKLOADS["fabric8_1080p"]
    mats = wl.materials()
    g = wl.gbuffer()
    log(f"workload {wl.name}: {g.n} px, {len(mats)} fabrics")
    d = pkg.DeviceGBuffer.from_host(g)
    fab = pkg.Fabric(0, seed=wl.seed())
    fab.encode(mats)

    # ---- training on GPU-generated batches and analytic targets (untimed) ----
    rows = {}
    lr0 = args.train_lr
    t0 = time.perf_counter()
    losses = []
    torch.cuda.synchronize()
    tr_start = torch.cuda.Event(enable_timing=True)
    tr_stop = torch.cuda.Event(enable_timing=True)
    tr_start.record()
    for s in range(args.train_steps):
        # Adam, cosine-decayed learning rate
        lr = lr0 * 0.5 * (1.0 + math.cos(math.pi * s / max(1, args.train_steps)))
        want = (s % 500 == 0) or s == args.train_steps - 1
        l = fab.train_step(seed=1_000_000 + s, batch=args.train_batch, gt_samples=args.gt_samples,
                           prec=pkg.FABRIC_BF16, lr=lr, want_loss=want)
        if want:
            losses.append((s, l))
            log(f"train step {s}: loss {l:.5f}")
    tr_stop.record()
    torch.cuda.synchronize()
    train_ms = tr_start.elapsed_time(tr_stop) / max(1, args.train_steps)
    rows["train_step"] = {"ms_per_step": train_ms, "batch": args.train_batch,
                          "gt_samples": args.gt_samples,
                          "samples_per_s": args.train_batch / (train_ms * 1e-3),
                          "loss_first": losses[0][1] if losses else None,
                          "loss_last": losses[-1][1] if losses else None}
    log(f"trained {args.train_steps} steps in {time.perf_counter() - t0:.1f}s ({train_ms:.2f} ms/step)")
    fab.encode(mats)
    params = fab.params()

    # ---- timed neural shading (BF16) ----
    out = torch.empty((3, g.n), dtype=torch.float32, device="cuda")
    shade = lambda prec: pkg.fabric_shade_gbuffer(fab.ctx, d, pkg.PREC[prec], 0, 0, out)
    for _ in range(args.warmup):
        shade("bf16")
    torch.cuda.synchronize()
    ms = time_launches(torch, lambda: shade("bf16"), args.steps)
    mpix = g.n / (ms * 1e-3) / 1e6
    log(f"neural bf16: {ms * 1e3:.1f} us/frame, {mpix:.0f} Mpix/s")
    rgb_bf16 = out.cpu().numpy()

    # ---- analytic footprint filter on the same frame ----
    a_rgb = torch.empty((3, g.n), dtype=torch.float32, device="cuda")
    a_comp = torch.empty((4, g.n), dtype=torch.float32, device="cuda")
    filt = lambda: pkg.fabric_gt_filtered(fab.ctx, d, args.gt_samples, 4242, a_rgb, a_comp)
    filt()
    a_ms = time_launches(torch, filt, args.analytic_steps)
    a_mpix = g.n / (a_ms * 1e-3) / 1e6
    log(f"analytic {args.gt_samples} samples: {a_ms:.2f} ms/frame, {a_mpix:.1f} Mpix/s")
    gt_rgb = a_rgb.cpu().numpy()

    if args.copy_calibration:
        src = torch.ones(128 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 512 MiB read + 512 MiB written")
        del src, dst

    # ---- other precisions and rows ----
    rgb = {"bf16": rgb_bf16}
    for prec in ("fp32", "fp16", "fp8"):
        for _ in range(max(5, args.warmup // (10 if prec == "fp32" else 2))):
            shade(prec)
        t = time_launches(torch, lambda: shade(prec), max(5, args.steps // 10))
        rows[f"neural_{prec}"] = {"ms_per_frame": t, "mpix_per_s": g.n / (t * 1e-3) / 1e6}
        rgb[prec] = out.cpu().numpy()
        log(f"neural {prec}: {t * 1e3:.1f} us/frame")
    def want(name):
        return not args.no_rows and (args.rows == "all" or name in args.rows.split(","))

    if want("c1_plain128"):
        rows["c1_plain128"] = c1_row(args, torch, pkg, fi)
    if want("hybrid_frame"):
        # Hybrid frame: 20 % out-of-range pixels routed to the analytic filter.
        # The hybrid G-buffer (20 % out of range) over the trained fabric
        # table, so that the decoder's class is judged on fabrics it learnt.
        hw = fi.WORKLOADS["hybrid_1080p"]
        hg = hw.gbuffer()
        hout = torch.empty((3, hg.n), dtype=torch.float32, device="cuda")
        # 60 jittered frames, all resident first (as a renderer's G-buffers
        # would be), shaded back to back after 10 warmup frames; each frame
        # is timed by its own pair of events.
        frames = [pkg.DeviceGBuffer.from_host(fi.jitter_gbuffer(hg, 50_000 + f)) for f in range(60)]
        hybrid = lambda f: pkg.fabric_shade_gbuffer(fab.ctx, frames[f], pkg.FABRIC_BF16,
                                                     args.gt_samples, f, hout)
        for f in range(10):
            hybrid(f)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in frames]
        torch.cuda.synchronize()
        for f in range(60):
            ev[f][0].record()
            hybrid(f)
            ev[f][1].record()
        torch.cuda.synchronize()
        frame_ms = [a.elapsed_time(b) for a, b in ev]
        del frames
        rows["hybrid_frame"] = {"frames": 60, "p50_ms": float(np.percentile(frame_ms, 50)),
                                "p99_ms": float(np.percentile(frame_ms, 99)),
                                "fps_p50": 1e3 / float(np.percentile(frame_ms, 50)),
                                "out_of_range_frac": hw.out_of_range_frac}
        if not args.no_rmse:
            rows["hybrid_frame"]["rmse_by_class"] = hybrid_class_errors(args, torch, pkg, fi, fab,
                                                                        mats, hg)
        log(f"hybrid frame p50 {rows['hybrid_frame']['p50_ms']:.3f} ms")
        fab.encode(mats)
    if want("encode_8_fabrics"):
        # Encoder: one (re-)encode of 8 fabrics (an edit).
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(20):
            fab.encode(mats)
        torch.cuda.synchronize()
        rows["encode_8_fabrics"] = {"ms": (time.perf_counter() - t0) / 20 * 1e3,
                                    "note": "host call incl. table upload"}
    if want("fabric64_4k"):
        rows["fabric64_4k"] = precision_row_4k(args, torch, pkg, fi, fab, params)
        fab.encode(mats)
    if want("train_step_2p20"):
        rows["train_step_2p20"] = train_row_2p20(args, torch, pkg, fab)
        fab.encode(mats)
    if want("latent_interpolation"):
        rows["latent_interpolation"] = interp_row(args, torch, pkg, fi, g, d)
    if want("visibility"):
        rows["visibility"] = visibility_row(args, torch, pkg, fi, wl, mats, g, d, ms)
    if want("transmission"):
        rows["transmission"] = btdf_row(args, torch, pkg, fi)
    if want("paper_decoder"):
        rows["paper_decoder"] = paper_decoder_row(args, torch, pkg, fi, mats, g, d)
    if want("paper_training"):
        rows["paper_training"] = paper_training_row(args, torch, pkg, fi, mats, g, d, rgb["bf16"])
    if want("ablations"):
        rows["ablations"] = ablation_row(args, torch, pkg, fi, mats, g, d)
    if want("paper_encoder"):
        rows["paper_encoder"] = paper_encoder_row(args, torch, pkg, fi, d)

    # ---- error against the FP64 oracle on a seeded pixel subset ----
    args.neural_ms = ms
    errs = None if args.no_rmse else oracle_errors(args, torch, pkg, fi, fab, d, mats, g, rgb, gt_rgb)
    paper = rows.get("paper_training", {}).get("rmse_vs_fp64_oracle")
    if errs and paper:
        gain = errs["gain"]
        gain["paper_size_bf16_rmse"] = paper["paper_bf16"]["rmse"]
        gain["paper_size_fp16_rmse"] = paper["paper_fp16"]["rmse"]
        gain["paper_size_bf16_beats_1spp"] = gain["paper_size_bf16_rmse"] < gain["analytic_1spp_rmse"]

    # ---- CPU baseline: the oracle on the host cores ----
    cpu = None
    if not args.no_cpu:
        import oracle
        threads = oracle.num_threads()
        res = cpu_baseline(oracle, mats, g, params, args.cpu_budget)
        n_dec, t_dec = res["decoder"]
        n_fil, t_fil = res["filter256"]
        n_1t, t_1t = res["decoder_1thread"]
        cpu = {"value": n_dec / t_dec / 1e6, "unit": "Mpixels/s", "cores": threads, "kind": "oracle",
               "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
               "decoder_1thread_mpix_per_s": n_1t / t_1t / 1e6,
               "sample": f"FP64 oracle decoder forward on a seeded {n_dec}-pixel subset of the frame "
                         f"({t_dec:.1f} s); footprint filter at 256 samples on {n_fil} pixels "
                         f"({t_fil:.1f} s) = {n_fil / t_fil / 1e6:.4f} Mpixels/s",
               "filter256_mpix_per_s": n_fil / t_fil / 1e6}
        log(f"cpu oracle: decoder {cpu['value']:.3f} Mpix/s, filter {cpu['filter256_mpix_per_s']:.5f} "
            f"Mpix/s on {threads} threads")

    achieved_tflops = FLOP_PER_PIXEL * g.n / (ms * 1e-3) / 1e12
    traffic, traffic_note = recorded_traffic()
    result = {
        "metric": "Mpixels/s neural vs filtered-analytic shading at 1080p; RMSE vs FP64 oracle",
        "value": mpix,
        "unit": "Mpixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "fabric8_1080p", "width": 1920, "height": 1080, "fabrics": 8,
                   "decoder": "latent 32, Fourier uv 8 freq + one-blob size, 3x64 ReLU, 4 outputs",
                   "analytic_samples": args.gt_samples},
        "fps": 1e3 / ms,
        "analytic_mpix_per_s": a_mpix,
        "analytic_ms_per_frame": a_ms,
        "neural_over_analytic": mpix / a_mpix,
        "rmse_vs_fp64_oracle": errs and errs["err"],
        "rmse_by_footprint_radius": errs and errs["by_r"],
        "gain_over_method_without_network": errs and errs["gain"],
        "bf16_over_fp32_rmse": errs and errs["ratio"],
        "roofline": {"bound": "mfma", "achieved": achieved_tflops, "peak": BF16_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved_tflops / BF16_PEAK_TFLOPS, "traffic": traffic,
                     "traffic_note": traffic_note,
                     "algorithmic_bytes": BYTES_PER_PIXEL * g.n,
                     "kernel": "decode32_kernel<bf16>",
                     "hbm_gbs": BYTES_PER_PIXEL * g.n / (ms * 1e-3) / 1e9},
        "cpu_baseline": cpu,
        "rows": rows,
        "paper_context": {"decoder_ms_per_1080p_frame": [13.6, 14.4], "hardware": "RTX 3090, TensorRT",
                          "network": "latent 64, 2+5 FC layers", "derived_mpix_per_s": [144.0, 152.5]},
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
