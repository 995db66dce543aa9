#!/usr/bin/env python
"""Throughput of the exact Gaussian ray renderer on one MI355X.

One step = one full forward (preprocess + PBF, association sort, render) of a
synthetic scene shaped like the forward-only workload: 100,000 Gaussians
with SH degree 3 in a 20 m box around the camera, an equidistant 180-degree
fisheye, a 1024 x 1024 BEAP ray grid, 16 x 16 tiles.  Inputs are resident in
HBM before the timed region; outputs are preallocated.

Printed (one JSON line on stdout):
  value          rays rendered per second (Mrays/s, whole job)
  roofline       the render kernel (dominant) against the FP32 vector peak,
                 its duration from HIP events recorded on its stream inside
                 the library; frame_roofline: the frame's algorithmic time
                 against the measured one
  cpu_baseline   the FP64 oracle on a bounded sample of the same rays, on the
                 host cores (and on one core), with the GPU's rays checked
                 against it on that sample
  fwd_bwd        forward + L1 loss + backward of 500,000 Gaussians (SH 3)
                 through a Kannala-Brandt 190-degree fisheye at 1280 x 960
                 against a target rendered from perturbed parameters, with
                 its own roofline (the backward replay kernel) and oracle leg
  train_batched  one captured training step (per view: forward, L1, backward)
                 of 3M Gaussians (SH 3) over 8 views of 1920 x 1080, four
                 pinhole 90-degree and four equidistant 180-degree, with its
                 roofline and oracle leg
  serving        render requests (pinhole 640 x 480, equidistant 1024 x 1024,
                 KB 200-degree 1920 x 1080) over a resident 1M-Gaussian scene:
                 saturated throughput (closed loop), then Poisson arrivals at
                 70% and 90% of it; p50/p99 latency to device completion,
                 req/s, Mrays/s, mean batch, device overlap
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mrays/s fwd and fwd+bwd vs plain, p50/p99 frame latency, RGB err vs FP64"
# MI355X published peaks: FP32 vector 157.3 TFLOP/s (the figure counts packed
# FP32, two lanes' FMAs per instruction; this build keeps packed FP32 off, so
# 78.6 TFLOP/s is the most its scalar-FP32 code can issue, reported beside
# it), HBM3E 8 TB/s.
PEAK_TFLOPS = 157.3
UNPACKED_TFLOPS = 78.6
HBM_BPS = 8.0e12
# Algorithmic work of one evaluated (ray, Gaussian) pair of the render:
# whitened direction (9 FMA), cross product (9), the two squared norms (5 + 5),
# closest approach (5), contribution test, alpha, blend and transmittance
# (~10): 48 FLOP, plus one exp and one reciprocal.  The backward replay does
# about 2.5 times that per pair (recovering T, the colour behind, and the
# 16 partial derivatives of App. C).
FLOP_FWD_PAIR = 48
FLOP_BWD_PAIR = 120


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Sources the render kernel is compiled from (its own file and the headers
# holding its device code).
RENDER_SOURCES = ("render.hip", "geer_device.h", "geer_common.h")


def source_hash(paths):
    h = hashlib.sha256()
    for path in paths:
        h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


def traffic_record(csrc_dir):
    """HBM bytes per render launch from the committed rocprofv3 PMC summary,
    or None when the kernel's sources changed since the counters were taken."""
    p = os.path.join(ROOT, "profiles", "render_fisheye100k_pmc.json")
    if not os.path.exists(p):
        return None
    rec = json.load(open(p))
    if rec.get("render_src_sha") != source_hash([os.path.join(csrc_dir, f) for f in RENDER_SOURCES]):
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    threads = len(os.sched_getaffinity(0))
    if os.environ.get("OMP_NUM_THREADS"):
        threads = min(threads, int(os.environ["OMP_NUM_THREADS"]))
    return threads


# ----------------------------------------------------- algorithmic time --

def t_forward(gaussians, views, sh_degree, visible, entries, evaluated, rays):
    """Algorithmic time (s) of one forward at the MI355X peaks, by term:
    preprocess reads the scene once (44 + 12K B per Gaussian) and writes an
    80-B item per (Gaussian, view); the association moves ~44 B per list entry
    (expansion write, two tile passes, the render's read) and 32 B per
    visible item (four depth passes); the render does 48 FLOP per evaluated
    pair and writes 24 B per ray."""
    K = (sh_degree + 1) ** 2
    return {"preprocess": (gaussians * (44 + 12 * K) + gaussians * views * 80) / HBM_BPS,
            "association": (entries * 44 + visible * 32) / HBM_BPS,
            "render": evaluated * FLOP_FWD_PAIR / (PEAK_TFLOPS * 1e12) + rays * 24 / HBM_BPS}


def t_backward(gaussians, sh_degree, visible, evaluated_bwd, rays):
    """Algorithmic time (s) of the L1 loss and the backward: the loss reads
    RGB, target and mask and writes dL/dRGB (37 B per ray); the replay does
    120 FLOP per replayed pair and reads dL/dRGB, T_final and the last index
    (20 B per ray); the Gaussian-wise stage reads the parameters and the
    64-B accumulator of each visible item and writes the gradients."""
    K = (sh_degree + 1) ** 2
    return {"l1": rays * 37 / HBM_BPS,
            "replay": evaluated_bwd * FLOP_BWD_PAIR / (PEAK_TFLOPS * 1e12) + rays * 20 / HBM_BPS,
            "gaussian_wise": (2 * gaussians * (44 + 12 * K) + visible * 64) / HBM_BPS}


def frame_roofline(terms_s, measured_ms):
    t = sum(terms_s.values())
    return {"t_roof_ms": round(t * 1e3, 4), "t_measured_ms": round(measured_ms, 4),
            "frac": round(t * 1e3 / measured_ms, 4) if measured_ms > 0 else None,
            "terms_ms": {k: round(v * 1e3, 4) for k, v in terms_s.items()}}


def kernel_roofline(kernel, flop_per_pair, pairs, ms, traffic=None):
    """Achieved FLOP rate of one launch of `kernel`: pairs it evaluated
    times the algorithmic FLOP per pair, over its event-timed duration."""
    achieved = flop_per_pair * pairs / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    return {"kernel": kernel, "bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS, 4), "traffic": traffic,
            "launch_ms": round(ms, 4), "evaluated_pairs": int(pairs), "flop_per_pair": flop_per_pair,
            "frac_of_unpacked_78_6": round(achieved / UNPACKED_TFLOPS, 4)}


# ------------------------------------------------------------ oracle legs --

def oracle_leg(scene_np, cam, pix, threads, got, what):
    """The FP64 oracle on `pix` (all host threads), timed, and the GPU's rays
    `got` = (rgb [P,3], depth [P], trans [P]) checked against it: unflagged
    rays at the RGB/T 2e-4 and depth 1e-3 gates, flagged rays against their
    decision branches."""
    import numpy as np

    import oracle

    c0 = time.perf_counter()
    ref = oracle.render(scene_np, cam, pix=pix, nthreads=threads)
    c1 = time.perf_counter()
    rgb, depth, trans = got
    err = np.abs(rgb - ref["rgb"]).max(axis=1)
    okm = ~ref["amb"]
    terr = np.abs(trans - ref["trans"])
    derr = np.abs(depth - ref["depth"]) / (1 + np.abs(ref["depth"]))
    score = oracle.branch_scores(rgb, depth, trans, ref)
    check = {"rays": int(pix.size), "max_abs_rgb_unflagged": float(err[okm].max(initial=0)),
             "max_abs_t_unflagged": float(terr[okm].max(initial=0)),
             "max_rel_depth_unflagged": float(derr[okm].max(initial=0)),
             "flagged_frac": round(float(ref["amb"].mean()), 5),
             "flagged_match_a_branch": bool(np.all(score <= 1.0)),
             "pass": bool(err[okm].max(initial=0) <= 2e-4 and terr[okm].max(initial=0) <= 2e-4
                          and derr[okm].max(initial=0) <= 1e-3 and np.all(score <= 1.0))}
    cpu = {"value": round(pix.size / (c1 - c0) / 1e6, 6), "unit": "Mrays/s", "cores": threads, "kind": "oracle",
           "seconds": round(c1 - c0, 2), "cpu_model": cpu_model(),
           "sample": "%d seeded random rays of %s, FP64 brute force over all %d Gaussians (with the decision "
                     "branches of flagged rays)" % (pix.size, what, scene_np.n)}
    return cpu, check


def single_thread(scene_np, cam, pix):
    import oracle

    c0 = time.perf_counter()
    oracle.render(scene_np, cam, pix=pix, nthreads=1, branches=False)
    return round(pix.size / (time.perf_counter() - c0) / 1e6, 7)


def gpu_rays(rgb, depth, trans, rays, pix, dev):
    import torch

    tp = torch.as_tensor(pix, device=dev)
    g = rgb.view(3, rays).T[tp].double().cpu().numpy()
    d = depth[tp].double().cpu().numpy() if depth is not None else None
    t = trans[tp].double().cpu().numpy() if trans is not None else None
    return g, d, t


# -------------------------------------------------------------- workloads --

def bench_fwd_bwd(args, dev, threads):
    """Forward + L1 + backward steps of the 500k-Gaussian KB 190-degree frame."""
    import numpy as np
    import torch

    from paper_2505_24053_amd import _lib, renderer, synth

    scene_np, cams, target_np = synth.workload_kb_train(seed=args.seed)
    cam = cams[0]
    rays = cam["width"] * cam["height"]
    sc = renderer.scene_from_numpy(scene_np, device=dev)
    tgt_sc = renderer.scene_from_numpy(target_np, device=dev)
    target, _, _, _ = renderer.render(tgt_sc, cams)
    mask = torch.as_tensor(_lib.valid_mask(cam).reshape(-1).astype(np.uint8), device=dev)
    grads = {k: torch.empty_like(sc[k]) for k in ("mean", "scale", "quat", "opacity", "sh")}
    out = (torch.empty(3 * rays, device=dev), torch.empty(rays, device=dev), torch.empty(rays, device=dev))
    del tgt_sc
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    times = []

    def step(timed):
        if timed:
            ev[0].record()
        _, _, _, frame = renderer.render(sc, cams, out=out, keep_frame=True)
        if timed:
            ev[1].record()
        loss, dl = renderer.l1_loss(out[0], target, mask)
        if timed:
            ev[2].record()
        renderer.backward(frame, sc, dl, grads=grads)
        if timed:
            ev[3].record()
        frame.release()
        return loss

    for _ in range(args.train_warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.train_steps):
        loss = step(False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.train_steps
    # stage split: the same steps again with events between the stages, and
    # with the library's kernel events and pair counters
    renderer.set_profiling(True)
    renderer.profile_read()
    for _ in range(args.train_steps):
        step(True)
        torch.cuda.synchronize()
        times.append([ev[i].elapsed_time(ev[i + 1]) for i in range(3)])
    recs = renderer.profile_read(64)
    renderer.set_profiling(False)
    fw = [r for r in recs if r["kind"] == 0]
    bw = [r for r in recs if r["kind"] == 1]
    med = np.median(np.array(times), axis=0)
    _, _, _, frame = renderer.render(sc, cams, keep_frame=True)
    st = frame.stats()
    frame.release()
    ms_replay = statistics.mean(r["ms_render"] for r in bw)
    ms_fwd_render = statistics.mean(r["ms_render"] for r in fw)
    n_bwd = bw[-1]["n_evaluated"]
    terms = t_forward(scene_np.n, 1, scene_np.sh_degree, st["n_visible"], st["n_entries"], st["n_evaluated"], rays)
    terms.update(t_backward(scene_np.n, scene_np.sh_degree, st["n_visible"], n_bwd, rays))
    res = {"workload": "fwd_bwd_kb190_500k_sh3_1280x960_l1", "gaussians": scene_np.n, "rays": rays,
           "steps": args.train_steps, "ms_per_step": round(ms_step, 4),
           "mrays_per_s": round(rays / (ms_step * 1e-3) / 1e6, 3),
           "stages_ms": {"forward": round(float(med[0]), 4), "l1_loss": round(float(med[1]), 4),
                         "backward": round(float(med[2]), 4), "render_kernel": round(ms_fwd_render, 4),
                         "replay_kernel": round(ms_replay, 4),
                         "gaussian_wise_kernel": round(statistics.mean(r["ms_preprocess"] for r in bw), 4)},
           "loss": round(float(loss.item()), 6),
           "roofline": kernel_roofline("render_backward_kernel", FLOP_BWD_PAIR, n_bwd, ms_replay),
           "roofline_render": kernel_roofline("render_kernel", FLOP_FWD_PAIR, fw[-1]["n_evaluated"], ms_fwd_render),
           "frame_roofline": frame_roofline(terms, ms_step)}
    if args.cpu_rays > 0 and args.cpu_rays_c3 > 0:
        valid = np.nonzero(_lib.valid_mask(cam).reshape(-1))[0]
        pix = np.sort(np.random.default_rng(args.seed + 2).choice(valid, args.cpu_rays_c3, replace=False))
        got = gpu_rays(out[0], out[1], out[2], rays, pix, dev)
        res["cpu_baseline"], res["rgb_err_vs_fp64"] = oracle_leg(scene_np, cam, pix, threads, got,
                                                                 "the 1280x960 KB 190 frame's valid rays")
    return res


def bench_train_batched(args, dev, threads):
    """Captured batched training steps: 3M Gaussians SH3, 8 views of 1920x1080."""
    import numpy as np
    import torch

    from paper_2505_24053_amd import _lib, renderer, synth

    scene_np = synth.scene_box(3_000_000, seed=args.seed)
    cams = synth.workload_batched_views(seed=args.seed)
    sc = renderer.scene_from_numpy(scene_np, device=dev)
    tsc = renderer.scene_from_numpy(synth.perturb(scene_np, args.seed + 1), device=dev)
    target, _, _, _ = renderer.render(tsc, cams)
    del tsc
    mask = torch.as_tensor(np.concatenate([_lib.valid_mask(c).reshape(-1) for c in cams]).astype(np.uint8),
                           device=dev)
    pbf = 0
    for c in cams:  # the PBF pairs of the densest view size the plan's capacity
        _, _, _, fr = renderer.render(sc, [c], keep_frame=True)
        pbf = max(pbf, fr.stats()["n_candidates"])
        fr.release()
    rays = sum(c["width"] * c["height"] for c in cams)
    plan = renderer.TrainPlan(sc, cams, int(pbf * 1.25) + 1024, target, mask)
    stream = torch.cuda.current_stream()
    for _ in range(args.train_warmup):
        plan.launch(cams, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batched_steps):
        plan.launch(cams, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    E, cap, over = plan.entries()
    pst = plan.stats()
    ms = (t1 - t0) * 1e3 / args.batched_steps
    # the same per-view kernels, eagerly, with the library's kernel events and
    # pair counters: forward, L1 and backward of each view
    renderer.set_profiling(True)
    renderer.profile_read()
    grads = {k: torch.zeros_like(sc[k]) for k in ("mean", "scale", "quat", "opacity", "sh")}
    off = 0
    for c in cams:
        hw = c["width"] * c["height"]
        rgb, _, _, frame = renderer.render(sc, [c], keep_frame=True, want_depth=False, want_trans=False)
        _, dl = renderer.l1_loss(rgb, target[3 * off: 3 * (off + hw)], mask[off: off + hw])
        renderer.backward(frame, sc, dl, accumulate=True, grads=grads)
        torch.cuda.synchronize()
        frame.release()
        off += hw
    recs = renderer.profile_read(64)
    renderer.set_profiling(False)
    del grads
    bw = [r for r in recs if r["kind"] == 1]
    fw = [r for r in recs if r["kind"] == 0]
    n_bwd = sum(r["n_evaluated"] for r in bw)
    ms_replay = sum(r["ms_render"] for r in bw)
    n_fwd = sum(r["n_evaluated"] for r in fw)
    ms_render = sum(r["ms_render"] for r in fw)
    terms = t_forward(scene_np.n, len(cams), scene_np.sh_degree, pst["n_visible"], pst["n_entries"],
                      pst["n_evaluated"], rays)
    terms.update(t_backward(scene_np.n, scene_np.sh_degree, pst["n_visible"], n_bwd, rays))
    # per launch: the average view's pairs over the average launch
    roof = kernel_roofline("render_backward_kernel (one view of the step, launched eagerly)", FLOP_BWD_PAIR,
                           n_bwd / len(bw), ms_replay / len(bw))
    roof_r = kernel_roofline("render_kernel (one view of the step, launched eagerly)", FLOP_FWD_PAIR,
                             n_fwd / len(fw), ms_render / len(fw))
    out = {"workload": "train_step_3m_sh3_8x1920x1080_pinhole90_fisheye180_l1", "gaussians": scene_np.n,
           "views": len(cams), "rays": rays, "steps": args.batched_steps, "ms_per_step": round(ms, 3),
           "mrays_per_s": round(rays / (ms * 1e-3) / 1e6, 2), "loss": round(float(plan.loss.item()), 6),
           "max_pbf_pairs_per_view": int(E), "capacity": int(cap), "overflow": bool(over),
           "association": {"pbf_pairs": pst["n_candidates"], "entries": pst["n_entries"],
                           "visible": pst["n_visible"], "evaluated_pairs": pst["n_evaluated"]},
           "device_workspace_gib": round(plan.device_bytes() / 2**30, 2),
           "roofline": roof, "roofline_render": roof_r, "frame_roofline": frame_roofline(terms, ms)}
    # the optimiser step on the step's gradients: one fused Adam kernel over
    # the raw parameters, moments and statistics (HBM-bound: per Gaussian it
    # reads raw, m, v and the gradient rows, writes raw, m, v, the activated
    # scale and opacity, and updates the two statistics)
    from paper_2505_24053_amd import train

    st = train.TrainState.from_scene(scene_np, device=dev)
    for t in range(1, 3):
        st.adam_step(plan.grads, t)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for t in range(3, 3 + args.batched_steps):
        st.adam_step(plan.grads, t)
    e1.record()
    torch.cuda.synchronize()
    ms_adam = e0.elapsed_time(e1) / args.batched_steps
    nr = train.rows(scene_np.sh_degree)
    adam_bytes = scene_np.n * 4 * (4 * nr + 3 * nr + 4 + 4)
    out["adam"] = {"ms": round(ms_adam, 4), "ms_step_with_adam": round(ms + ms_adam, 3),
                   "roofline": {"kernel": "adam_kernel", "bound": "hbm",
                                "achieved": round(adam_bytes / (ms_adam * 1e-3) / 1e9, 1), "peak": HBM_BPS / 1e9,
                                "unit": "GB/s", "frac": round(adam_bytes / (ms_adam * 1e-3) / HBM_BPS, 4),
                                "traffic": None, "bytes_per_launch": adam_bytes}}
    del st
    if args.cpu_rays > 0 and args.cpu_rays_c5 > 0:
        import oracle

        per = max(args.cpu_rays_c5 // len(cams), 1)
        rng = np.random.default_rng(args.seed + 3)
        secs, checks, off = 0.0, [], 0
        for c in cams:
            hw = c["width"] * c["height"]
            pix = np.sort(rng.choice(hw, per, replace=False))
            rgb_v = plan.rgb[3 * off: 3 * (off + hw)]
            g = rgb_v.view(3, hw).T[torch.as_tensor(pix, device=dev)].double().cpu().numpy()
            c0 = time.perf_counter()
            ref = oracle.render(scene_np, c, pix=pix, nthreads=threads)
            secs += time.perf_counter() - c0
            err = np.abs(g - ref["rgb"]).max(axis=1)
            # the step keeps no depth or T: flagged rays are matched on RGB
            score = oracle.branch_scores(g, ref["depth"], ref["trans"], ref)
            checks.append((float(err[~ref["amb"]].max(initial=0)), float(ref["amb"].mean()),
                           bool(np.all(score <= 1))))
            off += hw
        out["cpu_baseline"] = {"value": round(per * len(cams) / secs / 1e6, 7), "unit": "Mrays/s",
                               "cores": threads, "kind": "oracle", "seconds": round(secs, 2),
                               "cpu_model": cpu_model(),
                               "sample": "%d seeded random rays per view of the 8 views, FP64 brute force over "
                                         "all 3M Gaussians" % per}
        out["rgb_err_vs_fp64"] = {"rays": per * len(cams), "max_abs_rgb_unflagged": max(c[0] for c in checks),
                                  "flagged_frac": round(float(np.mean([c[1] for c in checks])), 5),
                                  "flagged_match_a_branch": all(c[2] for c in checks)}
    plan.destroy()
    return out


def bench_assoc_variants(args, dev, sc, scene_np, cams, base_rgb):
    """The PBF against the projected-footprint associations (EWA and UT, square
    and snug boxes) in the same pipeline on the forward frame: frame time
    with and without the contribution-cone cull, PBF/box pairs per tile (the
    list without the cull), and how far each image is from the PBF's (pairs
    the footprint boxes lose)."""
    import numpy as np
    import torch

    from paper_2505_24053_amd import _lib, renderer

    rays = cams[0]["width"] * cams[0]["height"]
    out = (torch.empty(3 * rays, device=dev), torch.empty(rays, device=dev), torch.empty(rays, device=dev))
    res = {}
    for method in ("pbf", "ewa", "ewa_snug", "ut", "ut_snug"):
        row = {}
        for cull in (True, False):
            opts = dict(assoc=method, cone_cull=cull)
            for _ in range(2):
                renderer.render(sc, cams, opts=opts, out=out)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.variant_steps):
                renderer.render(sc, cams, opts=opts, out=out)
            torch.cuda.synchronize()
            row["ms_frame" if cull else "ms_frame_no_cull"] = round((time.perf_counter() - t0) * 1e3 /
                                                                    args.variant_steps, 4)
            if cull:
                diff = (out[0].view(3, rays) - base_rgb.view(3, rays)).abs().amax(dim=0)
                row["rgb_vs_pbf"] = {"max_abs": round(float(diff.max().item()), 6),
                                     "rays_over_2e-4": round(float((diff > 2e-4).float().mean().item()), 6)}
            else:
                _, _, _, fr = renderer.render(sc, cams, opts=opts, keep_frame=True)
                per_tile = np.diff(fr.export(_lib.BUF_RANGES).astype(np.int64))
                st = fr.stats()
                fr.release()
                row.update(pairs=int(st["n_candidates"]), per_tile_mean=round(float(per_tile.mean()), 1),
                           per_tile_std=round(float(per_tile.std()), 1), visible=int(st["n_visible"]))
        res[method] = row
        log("association %s:" % method, row)
    return res


def bench_native(args, dev):
    """Native-space output: the 1280x960 KB 190 frame (RGB, depth, T) resampled
    onto its native sensor; the kernel is HBM-bound (16 B of sampling map,
    ~4C B of image read and 4C B written per native pixel, C = 5)."""
    import torch

    from paper_2505_24053_amd import renderer, synth

    scene_np, cams, _ = synth.workload_kb_train(seed=args.seed)
    cam = cams[0]
    sc = renderer.scene_from_numpy(scene_np, device=dev)
    rgb, depth, trans, _ = renderer.render(sc, cams)
    beap = torch.cat([rgb.view(3, -1), depth.view(1, -1), trans.view(1, -1)]).contiguous()
    renderer.reproject(beap, cam)  # builds and caches the sampling map
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        nat, valid = renderer.reproject(beap, cam)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    npix = nat.shape[1] * nat.shape[2]
    C = beap.shape[0]
    nbytes = npix * (16 + 8 * C + 1)
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"workload": "reproject_kb190_1280x960_rgb_depth_t", "native_pixels": npix,
            "reached_frac": round(float(valid.float().mean().item()), 4), "channels": C, "ms": round(ms, 4),
            "roofline": {"kernel": "reproject_kernel", "bound": "hbm", "achieved": round(gbs, 1),
                         "peak": HBM_BPS / 1e9, "unit": "GB/s", "frac": round(gbs / (HBM_BPS / 1e9), 4),
                         "traffic": None, "bytes_per_launch": nbytes,
                         "note": "per launch time from events around back-to-back launches on the stream"}}


def bench_serving(args, dev):
    """Continuous batching over the resident 1M-Gaussian scene: the saturated
    throughput, then Poisson arrivals at fractions of it."""
    import numpy as np
    import torch

    from paper_2505_24053_amd import renderer, serve, synth

    scene_np = synth.scene_box(1_000_000, seed=args.seed)
    sc = renderer.scene_from_numpy(scene_np, device=dev)
    del scene_np
    # association capacity: the densest of a few sample requests, with margin
    probe = synth.workload_serving_requests(9, seed=args.seed + 100)
    per_tile, alone_ms = 0.0, {}
    for c in probe:
        renderer.render(sc, [c])  # warm the allocator
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, _, _, fr = renderer.render(sc, [c], keep_frame=True)
        torch.cuda.synchronize()
        alone_ms.setdefault(c["model"], []).append((time.perf_counter() - t) * 1e3)
        per_tile = max(per_tile, fr.stats()["n_candidates"] / serve.tiles_of((c["width"], c["height"])))
        fr.release()
    shapes = {(c["width"], c["height"]) for c in probe}
    srv = serve.Server(sc, shapes, entries_per_tile=1.5 * per_tile, slots=args.serve_slots, slot_views=2,
                       max_views=4)
    graphs = srv.prepare(shapes)
    warm = synth.workload_serving_requests(args.serve_warmup, seed=args.seed + 200)
    srv.run([serve.Request(i, c) for i, c in enumerate(warm)])

    def point(rate, j):
        srv.stats = dict(batches=0, overflows=0, stalls=0, views=0, overlapped=0)
        srv.intervals = []
        srv.evaluated = 0
        cams = synth.workload_serving_requests(args.serve_requests, seed=args.seed + 300 + 10 * j)
        arrivals = None if rate is None else serve.poisson_arrivals(len(cams), rate, seed=args.seed + 301 + 10 * j)
        done = srv.run([serve.Request(i, c) for i, c in enumerate(cams)], arrivals)
        summ = serve.latency_summary(done)
        st = dict(srv.stats)
        span = max(r.t_done for r in done) - min(r.t_arrive for r in done)
        res = {"rate_req_per_s": rate, "requests": summ["requests"], "p50_ms": round(summ["p50_ms"], 3),
               "p99_ms": round(summ["p99_ms"], 3), "mean_ms": round(summ["mean_ms"], 3),
               "max_ms": round(summ["max_ms"], 3), "req_per_s": round(float(summ["req_per_s"]), 2),
               "mrays_per_s": round(float(summ["mrays_per_s"]), 2), "batches": st["batches"],
               "mean_batch": round(st["views"] / max(st["batches"], 1), 2),
               "admitted_while_busy": st["overlapped"], "device_overlap_frac": round(srv.device_overlap(), 3),
               "overflow_batches": st["overflows"], "stalled_batches": st["stalls"],
               "render_tflops": round(FLOP_FWD_PAIR * srv.evaluated / span / 1e12, 3)}
        log("serving %s:" % ("saturated" if rate is None else "at %.0f req/s" % rate), res)
        return res

    sat = point(None, 0)
    cap = sat["req_per_s"]
    points = [point(round(f * cap, 1), j + 1) for j, f in enumerate(args.serve_loads)]
    ws_gb = srv.slot_bytes * len(srv.slots) / 2**30
    srv.close()
    out = {"workload": "serving_1m_sh3_mixed_pinhole640x480_fisheye1024_kb200_1920x1080"}
    out.update(points[0] if points else sat)
    out.update({"load_of_saturated": args.serve_loads[0] if points else 1.0, "saturated": sat,
                "slots": len(srv.slots), "workspace_gib": round(ws_gb, 2), "graphs_per_slot": graphs,
                "entries_per_tile_capacity": round(1.5 * per_tile, 1),
                "alone_ms": {k: round(float(np.median(v)), 3) for k, v in alone_ms.items()},
                "rates": points,
                "roofline": {"kernel": "render_kernel (whole-job rate over the saturated run)", "bound": "alu",
                             "achieved": sat["render_tflops"], "peak": PEAK_TFLOPS, "unit": "TFLOP/s",
                             "frac": round(sat["render_tflops"] / PEAK_TFLOPS, 4), "traffic": None,
                             "flop_per_pair": FLOP_FWD_PAIR}})
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-rays", type=int, default=16384, help="oracle sample of the 1024^2 frame (0: no oracle)")
    ap.add_argument("--cpu-rays-single", type=int, default=384, help="single-thread oracle sample")
    ap.add_argument("--cpu-rays-c3", type=int, default=2048, help="oracle sample of the fwd+bwd frame")
    ap.add_argument("--cpu-rays-c5", type=int, default=512, help="oracle sample of the 8-view step")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="after timing, copy this many MiB device-to-device once (a plain copy kernel of known "
                         "size that calibrates rocprofv3 FETCH_SIZE / WRITE_SIZE in the same run)")
    ap.add_argument("--train-steps", type=int, default=10, help="fwd+bwd steps (0: skip)")
    ap.add_argument("--train-warmup", type=int, default=3)
    ap.add_argument("--batched-steps", type=int, default=5, help="captured 8-view training steps (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=2000, help="requests per serving point (0: skip)")
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-loads", type=lambda t: [float(x) for x in t.split(",")], default=[0.7, 0.9],
                    help="Poisson arrival rates as fractions of the saturated throughput; the first is the "
                         "headline point")
    ap.add_argument("--serve-slots", type=int, default=3)
    ap.add_argument("--variant-steps", type=int, default=10, help="frames per association variant (0: skip)")
    ap.add_argument("--native", type=int, default=1, help="native-space output section (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2505_24053_amd import _lib, renderer, synth

    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__

        __graft_entry__.build()
    dev = torch.device("cuda:0")
    threads = host_threads()
    scene_np, cams = synth.workload_fisheye_forward(seed=args.seed)
    cam = cams[0]
    W, H = cam["width"], cam["height"]
    rays = W * H
    sc = renderer.scene_from_numpy(scene_np, device=dev)
    out = (torch.empty(3 * rays, device=dev), torch.empty(rays, device=dev), torch.empty(rays, device=dev))
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        renderer.render(sc, cams, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        renderer.render(sc, cams, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = rays / (ms_step * 1e-3) / 1e6
    renderer.check_errors()
    # stage split and the render kernel's launch time: the same frames again
    # with device events between the stages (outside the timed loop, since the
    # events themselves cost time)
    renderer.set_profiling(True)
    renderer.profile_read()
    for _ in range(args.steps):
        renderer.render(sc, cams, out=out)
    torch.cuda.synchronize()
    recs = [r for r in renderer.profile_read(64) if r["kind"] == 0]
    renderer.set_profiling(False)

    ms_render = statistics.mean(r["ms_render"] for r in recs)
    ms_prep = statistics.mean(r["ms_preprocess"] for r in recs)
    ms_sort = statistics.mean(r["ms_sort"] for r in recs)
    ms_total = statistics.mean(r["ms_total"] for r in recs)
    n_eval = recs[-1]["n_evaluated"]
    n_entries = recs[-1]["n_entries"]
    _, _, _, frame = renderer.render(sc, cams, keep_frame=True)
    ranges = frame.export(_lib.BUF_RANGES).astype(np.int64)
    st = frame.stats()
    frame.release()
    per_tile = np.diff(ranges)
    traffic = traffic_record(os.path.join(ROOT, "paper_2505_24053_amd", "csrc"))
    roofline = kernel_roofline("render_kernel", FLOP_FWD_PAIR, n_eval, ms_render, traffic)
    frame_roof = frame_roofline(t_forward(scene_np.n, 1, scene_np.sh_degree, st["n_visible"], n_entries, n_eval,
                                          rays), ms_step)

    if args.copy_probe > 0:
        nb = args.copy_probe << 20
        src = torch.empty(nb // 4, device=dev)
        dst = torch.empty(nb // 4, device=dev)
        src.fill_(1.0)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    cpu = None
    rgb_err = None
    if args.cpu_rays > 0:
        pix = np.sort(np.random.default_rng(args.seed + 1).choice(rays, args.cpu_rays, replace=False))
        got = gpu_rays(out[0], out[1], out[2], rays, pix, dev)
        cpu, rgb_err = oracle_leg(scene_np, cam, pix, threads, got, "the same 1024x1024 frame")
        if args.cpu_rays_single > 0:
            cpu["single_thread_value"] = single_thread(scene_np, cam, pix[: args.cpu_rays_single])
            cpu["single_thread_sample"] = "the first %d rays of the sample on one thread" % args.cpu_rays_single

    variants = None
    if args.variant_steps > 0:
        log("association variants on the forward frame")
        variants = bench_assoc_variants(args, dev, sc, scene_np, cams, out[0].clone())
    native = None
    if args.native:
        native = bench_native(args, dev)
        log("native output:", native)

    fwd_bwd = None
    if args.train_steps > 0:
        log("fwd+bwd: 500k Gaussians, KB 190 deg 1280x960")
        fwd_bwd = bench_fwd_bwd(args, dev, threads)
        log("fwd+bwd:", fwd_bwd)
    train_batched = None
    if args.batched_steps > 0:
        log("batched training step: 3M Gaussians, 8 views of 1920x1080")
        train_batched = bench_train_batched(args, dev, threads)
        log("batched:", train_batched)
    serving = None
    if args.serve_requests > 0:
        log("serving: 1M Gaussians, %d requests per point, saturated then %s of it" % (args.serve_requests,
                                                                                    args.serve_loads))
        serving = bench_serving(args, dev)
        log("serving:", serving)
    renderer.check_errors()

    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "forward_fisheye180_100k_sh3_1024x1024", "gaussians": scene_np.n, "sh_degree": 3,
                   "camera": "equidistant 180 deg", "beap_grid": [W, H], "tile": 16, "rays": rays},
        "stages_ms": {"preprocess": round(ms_prep, 4), "sort": round(ms_sort, 4), "render": round(ms_render, 4),
                      "device_total": round(ms_total, 4)},
        "association": {"entries": int(n_entries), "pbf_pairs": int(st["n_candidates"]),
                        "visible": int(st["n_visible"]),
                        "entries_per_tile_mean": round(float(per_tile.mean()), 1),
                        "entries_per_tile_std": round(float(per_tile.std()), 1)},
        "rgb_err_vs_fp64": rgb_err,
        "roofline": roofline,
        "frame_roofline": frame_roof,
        "cpu_baseline": cpu,
        "association_variants": variants,
        "native_output": native,
        "fwd_bwd": fwd_bwd,
        "train_batched": train_batched,
        "serving": serving,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
