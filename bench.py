#!/usr/bin/env python
"""Throughput of the exact Gaussian ray renderer on one MI355X.

One step = one full forward (preprocess + PBF, association sort, render) of a
synthetic scene shaped like the forward-only workload: 100,000 Gaussians
with SH degree 3 in a 20 m box around the camera, an equidistant 180-degree
fisheye, a 1024 x 1024 BEAP ray grid, 16 x 16 tiles.  Inputs are resident in
HBM before the timed region; outputs are preallocated.

Printed (one JSON line on stdout):
  value          rays rendered per second (Mrays/s, whole job)
  roofline       the render kernel (dominant) against the FP32 VALU peak,
                 timed with HIP events on its own stream inside the library
  cpu_baseline   the FP64 oracle on a bounded sample of the same rays,
                 on the host cores, with the GPU's RGB error on that sample
  fwd_bwd        forward + L1 loss + backward of 500,000 Gaussians (SH 3)
                 through a Kannala-Brandt 190-degree fisheye at 1280 x 960
                 against a target rendered from perturbed parameters
  train_batched  one captured training step (per view: forward, L1, backward)
                 of 3M Gaussians (SH 3) over 8 views of 1920 x 1080, four
                 pinhole 90-degree and four equidistant 180-degree
  serving        Poisson stream of render requests (pinhole 640 x 480,
                 equidistant 1024 x 1024, KB 200-degree 1920 x 1080) over a
                 resident 1M-Gaussian scene: p50/p99 latency, req/s, Mrays/s
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
# Render kernel work per evaluated (ray, entry) pair, in FP32 operations of its
# formulation (FMA = 2): g = G d (15), |g_perp|^2 (3), |g|^2 (2), 1/|g|^2 (1),
# q (1), exponent and exp2 (3), alpha clamp (1), T(1 - alpha) (2), weight (1),
# colour (6), depth (4).
FLOP_PER_PAIR = 39
# FP32 vector peak without packed FP32 (which the build disables): 256 CUs x
# 4 SIMD x 16 lanes x 2 FLOP (FMA) x 2.4 GHz.
PEAK_TFLOPS = 78.6432


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


def bench_fwd_bwd(args, dev):
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
    # stage split: the same steps again with events between the stages
    for _ in range(args.train_steps):
        step(True)
        torch.cuda.synchronize()
        times.append([ev[i].elapsed_time(ev[i + 1]) for i in range(3)])
    med = np.median(np.array(times), axis=0)
    return {"workload": "fwd_bwd_kb190_500k_sh3_1280x960_l1", "gaussians": scene_np.n, "rays": rays,
            "steps": args.train_steps, "ms_per_step": round(ms_step, 4),
            "mrays_per_s": round(rays / (ms_step * 1e-3) / 1e6, 3),
            "stages_ms": {"forward": round(float(med[0]), 4), "l1_loss": round(float(med[1]), 4),
                          "backward": round(float(med[2]), 4)},
            "loss": round(float(loss.item()), 6)}


def bench_train_batched(args, dev):
    """Captured batched training steps: 3M Gaussians SH3, 8 views of 1920x1080."""
    import numpy as np
    import torch

    from paper_2505_24053_amd import _lib, renderer, synth

    scene_np = synth.scene_box(3_000_000, seed=args.seed)
    cams = synth.workload_batched_views(seed=args.seed)
    sc = renderer.scene_from_numpy(scene_np, device=dev)
    tsc = renderer.scene_from_numpy(synth.perturb(scene_np, args.seed + 1), device=dev)
    del scene_np
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
    ms = (t1 - t0) * 1e3 / args.batched_steps
    out = {"workload": "train_step_3m_sh3_8x1920x1080_pinhole90_fisheye180_l1", "gaussians": sc["mean"].shape[1],
           "views": len(cams), "rays": rays, "steps": args.batched_steps, "ms_per_step": round(ms, 3),
           "mrays_per_s": round(rays / (ms * 1e-3) / 1e6, 2), "loss": round(float(plan.loss.item()), 6),
           "max_pbf_pairs_per_view": int(E), "capacity": int(cap), "overflow": bool(over),
           "device_workspace_gib": round(plan.device_bytes() / 2**30, 2)}
    plan.destroy()
    return out


def bench_serving(args, dev):
    """Continuous batching over the resident 1M-Gaussian scene at a fixed rate."""
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
    srv.run([serve.Request(i, c) for i, c in enumerate(warm)],
            serve.poisson_arrivals(len(warm), args.serve_rates[0], seed=args.seed + 201))
    points = []
    for j, rate in enumerate(args.serve_rates):
        srv.stats = dict(batches=0, overflows=0, stalls=0, views=0, overlapped=0)
        srv.intervals = []
        cams = synth.workload_serving_requests(args.serve_requests, seed=args.seed + 300 + 10 * j)
        arrivals = serve.poisson_arrivals(len(cams), rate, seed=args.seed + 301 + 10 * j)
        done = srv.run([serve.Request(i, c) for i, c in enumerate(cams)], arrivals)
        summ = serve.latency_summary(done)
        st = dict(srv.stats)
        points.append({"rate_req_per_s": rate, "requests": summ["requests"], "p50_ms": round(summ["p50_ms"], 3),
                       "p99_ms": round(summ["p99_ms"], 3), "mean_ms": round(summ["mean_ms"], 3),
                       "max_ms": round(summ["max_ms"], 3), "req_per_s": round(float(summ["req_per_s"]), 2),
                       "mrays_per_s": round(float(summ["mrays_per_s"]), 2), "batches": st["batches"],
                       "mean_batch": round(st["views"] / max(st["batches"], 1), 2),
                       "admitted_while_busy": st["overlapped"],
                       "device_overlap_frac": round(srv.device_overlap(), 3), "overflow_batches": st["overflows"]})
        log("serving at %.0f req/s:" % rate, points[-1])
    ws_gb = srv.slot_bytes * len(srv.slots) / 2**30
    srv.close()
    out = {"workload": "serving_1m_sh3_mixed_pinhole640x480_fisheye1024_kb200_1920x1080"}
    out.update(points[0])
    out.update({"slots": len(srv.slots), "workspace_gib": round(ws_gb, 2), "graphs_per_slot": graphs,
                "entries_per_tile_capacity": round(1.5 * per_tile, 1),
                "alone_ms": {k: round(float(np.median(v)), 3) for k, v in alone_ms.items()},
                "rates": points})
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-rays", type=int, default=16384, help="oracle sample size (0: skip)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="after timing, copy this many MiB device-to-device once (a plain copy kernel of known "
                         "size that calibrates rocprofv3 FETCH_SIZE / WRITE_SIZE in the same run)")
    ap.add_argument("--train-steps", type=int, default=10, help="fwd+bwd steps (0: skip)")
    ap.add_argument("--train-warmup", type=int, default=3)
    ap.add_argument("--batched-steps", type=int, default=5, help="captured 8-view training steps (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=600, help="served requests (0: skip)")
    ap.add_argument("--serve-warmup", type=int, default=60)
    ap.add_argument("--serve-rates", type=lambda t: [float(x) for x in t.split(",")], default=[200.0, 500.0],
                    help="Poisson arrival rates (requests/s), comma-separated; the first is the headline point")
    ap.add_argument("--serve-slots", type=int, default=3)
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
    # stage split and the render kernel's launch time: the same frames again
    # with device events between the stages (outside the timed loop, since the
    # events themselves cost time)
    renderer.set_profiling(True)
    renderer.profile_read()
    for _ in range(args.steps):
        renderer.render(sc, cams, out=out)
    torch.cuda.synchronize()
    recs = renderer.profile_read(max(args.steps, 1))
    renderer.set_profiling(False)

    ms_render = statistics.mean(r["ms_render"] for r in recs)
    ms_prep = statistics.mean(r["ms_preprocess"] for r in recs)
    ms_sort = statistics.mean(r["ms_sort"] for r in recs)
    ms_total = statistics.mean(r["ms_total"] for r in recs)
    n_eval = recs[-1]["n_evaluated"]
    n_entries = recs[-1]["n_entries"]
    achieved = FLOP_PER_PAIR * n_eval / (ms_render * 1e-3) / 1e12
    _, _, _, frame = renderer.render(sc, cams, keep_frame=True)
    ranges = frame.export(_lib.BUF_RANGES).astype(np.int64)
    st = frame.stats()
    frame.release()
    per_tile = np.diff(ranges)
    traffic = traffic_record(os.path.join(ROOT, "paper_2505_24053_amd", "csrc"))
    roofline = {"kernel": "render_kernel", "bound": "alu", "achieved": round(achieved, 3),
                "peak": PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS, 4),
                "traffic": traffic, "launch_ms": round(ms_render, 4), "evaluated_pairs": int(n_eval),
                "flop_per_pair": FLOP_PER_PAIR}

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
        import oracle

        threads = len(os.sched_getaffinity(0))
        if os.environ.get("OMP_NUM_THREADS"):
            threads = min(threads, int(os.environ["OMP_NUM_THREADS"]))
        pix = np.random.default_rng(args.seed + 1).choice(rays, args.cpu_rays, replace=False)
        oracle.lib()
        c0 = time.perf_counter()
        ref = oracle.render(scene_np, cam, pix=pix, nthreads=threads)
        c1 = time.perf_counter()
        cpu = {"value": round(args.cpu_rays / (c1 - c0) / 1e6, 6), "unit": "Mrays/s", "cores": threads,
               "kind": "oracle", "seconds": round(c1 - c0, 2),
               "sample": "%d seeded random rays of the same 1024x1024 frame, FP64 brute force over all %d "
                         "Gaussians" % (args.cpu_rays, scene_np.n)}
        tp = torch.as_tensor(pix, device=dev)
        got = out[0].view(3, rays).T[tp].double().cpu().numpy()
        err = np.abs(got - ref["rgb"]).max(axis=1)
        okm = ~ref["amb"]
        score = oracle.branch_scores(got, out[1][tp].double().cpu().numpy(), out[2][tp].double().cpu().numpy(), ref)
        rgb_err = {"max_abs_unflagged": float(err[okm].max()), "rays": int(args.cpu_rays),
                   "flagged_frac": round(float(ref["amb"].mean()), 5),
                   "flagged_match_a_branch": bool(np.all(score <= 1.0))}

    fwd_bwd = None
    if args.train_steps > 0:
        log("fwd+bwd: 500k Gaussians, KB 190 deg 1280x960")
        fwd_bwd = bench_fwd_bwd(args, dev)
        log("fwd+bwd:", fwd_bwd)
    train_batched = None
    if args.batched_steps > 0:
        log("batched training step: 3M Gaussians, 8 views of 1920x1080")
        train_batched = bench_train_batched(args, dev)
        log("batched:", train_batched)
    serving = None
    if args.serve_requests > 0:
        log("serving: 1M Gaussians, %d requests at %s req/s" % (args.serve_requests, args.serve_rates))
        serving = bench_serving(args, dev)
        log("serving:", serving)

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
        "cpu_baseline": cpu,
        "fwd_bwd": fwd_bwd,
        "train_batched": train_batched,
        "serving": serving,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
