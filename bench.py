#!/usr/bin/env python
"""ToF ReSTIR benchmark on one MI355X.

Workload: the dynamic glossy scene at 512x512 (about 92k triangles, eight
moving GGX spheres over a displaced Lambertian ground, 3 bounces, 256-bin
transient histogram plus a time gate, temporal + one spatial round with 5
neighbours in a 30 px radius), synthetic and seeded.  A step is one frame of
the full ToF ReSTIR pipeline: BVH build for the frame's transforms, G-buffer,
path trees + per-bin initial RIS, temporal reuse, spatial reuse (each with
the path-length-aware Newton shift and generalized balance heuristic), splat
of the gate image and the histogram.

Prints one JSON line: frames/s of ToF ReSTIR (value), the equal-RMSE
comparison against plain ToF path tracing on the same GPU, per-frame latency
percentiles, per-kernel times measured with HIP events, the roofline entry of
the dominant kernel and the CPU oracle baseline.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
# Algorithmic work model: counted events x fixed per-event costs
NODE_BYTES = 64         # one 4-wide BVH node as traversal reads it: four quantized child boxes, links, count
TRI_BYTES = 48          # one leaf: three float4 vertices
F_NODE = 125            # FP32 ops of one node visit (four slab tests, sorting network of the hits)
F_TRI = 47              # FP32 ops of one watertight ray/triangle test
F_NEWTON_ITER = 220     # one Newton iteration: length function + derivatives, step, line-search trial
F_NEWTON_SETUP = 600    # per solve: chart points, source/destination evaluation, final determinants
F_SHIFT = 300           # per shift: replayed BSDF sampling/evaluation, Jacobian and target
SPLAT_BYTES = 4 + 4 + 4 + 0.125   # per (pixel, plane): PT deposit read, two histogram writes, mask bits
REC_HEAD_BYTES = 8      # per non-empty (pixel, plane): W and phat
# k_merge per item: the item, its first task, the winner's record read and
# written, the winner's shifted fields; per task: its forward terms and its K
# MIS terms (4 B each)
REC_BYTES = 64          # one reservoir record
MERGE_ITEM_BYTES = 8 + 4 + REC_BYTES + REC_BYTES + 32
MERGE_TASK_BYTES = 16


def sources_digest():
    """sha256 over the HIP sources and the C header: identifies the kernels
    that a stored counter measurement belongs to."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2605_11536_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            h.update(name.encode())
            h.update(open(os.path.join(csrc, name), "rb").read())
    h.update(open(os.path.join(ROOT, "include", "tof.h"), "rb").read())
    return h.hexdigest()


def measured_traffic(group):
    """HBM bytes per launch of a kernel group from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE runs scaled by a plain copy's
    reading) with the frame window it was taken over, or None when the
    kernels changed since it was taken or it covers another group."""
    path = os.path.join(ROOT, "profiles", "traffic_glossy_dynamic_512.json")
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("sources_sha256") != sources_digest():
        return None
    g = t.get("groups", {}).get(group)
    if not g:
        return None
    return {"bytes_per_launch": g["hbm_bytes_per_launch"], "frames": t["frames"]}


def valu_flops(w):
    return (F_NODE * w["node_visits"] + F_TRI * w["tri_tests"] + F_NEWTON_ITER * w["newton_iters"]
            + F_NEWTON_SETUP * w["newton_attempts"] + F_SHIFT * w["shifts"])


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--width", type=int, default=512)
    ap.add_argument("--ref-calls", type=int, default=256, help="reference PT calls (x ref-trees spp each)")
    ap.add_argument("--ref-trees", type=int, default=16)
    ap.add_argument("--rmse-frames", type=str, default="10,20,30,40,50,60",
                    help="frames of the sequence at which the equal-RMSE comparison is made")
    ap.add_argument("--no-bins-sweep", action="store_true")
    ap.add_argument("--no-pairwise", action="store_true", help="skip the pairwise-MIS timing leg")
    ap.add_argument("--no-equal-rmse", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-frames", type=int, default=4, help="oracle frames timed for the CPU baseline")
    ap.add_argument("--cpu-crop", type=int, default=256, help="side of the oracle's crop for the CPU baseline")
    ap.add_argument("--no-c5", action="store_true", help="skip the near-specular stress leg")
    ap.add_argument("--c5-only", action="store_true", help="run the near-specular stress leg alone")
    ap.add_argument("--c5-width", type=int, default=1920)
    ap.add_argument("--c5-height", type=int, default=1080)
    ap.add_argument("--no-autotune", action="store_true", help="skip the tuned-launch-shape leg")
    ap.add_argument("--no-bvh", action="store_true", help="skip the tree-builder comparison leg")
    ap.add_argument("--bvh-only", action="store_true", help="run the tree-builder comparison leg alone")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-only", action="store_true", help="run the serving leg alone")
    ap.add_argument("--serve-streams", type=int, default=64)
    ap.add_argument("--serve-frames", type=int, default=4, help="frames per stream")
    ap.add_argument("--serve-rate", type=float, default=0.0,
                    help="stream arrivals per second (Poisson); 0: set from --serve-load")
    ap.add_argument("--serve-load", type=float, default=0.6,
                    help="offered load (arrival rate x frames x mean solo frame time) that sets the rate")
    ap.add_argument("--serve-period-ms", type=float, default=33.3, help="interval between a stream's frames")
    ap.add_argument("--serve-budget-gib", type=float, default=224.0, help="HBM budget of the server")
    ap.add_argument("--serve-seed", type=int, default=7)
    ap.add_argument("--serve-timeout-s", type=float, default=240.0)
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="bytes of a plain device copy run after the timed region (HBM counter calibration)")
    return ap.parse_args()


def _threads():
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, n)


def cpu_baseline(width, first, count, crop):
    """The CPU oracle, as it stands, on bounded samples of the workloads.

    Headline: frames 0..first+count-1 of the benchmark sequence rendered on a
    crop x crop window at the image centre with every host thread, the last
    `count` timed (the frames the GPU's timed window starts with), the rate
    divided by the pixel ratio.  Beside it: one thread on a 128x128 crop (one
    frame, after the same history), the tiny box configuration in full (64x64,
    4 frames) and the first 4 frames of the NLOS configuration in full (64x64
    scan, 50k-triangle torus, 1024 bins)."""
    from paper_2605_11536_amd import scenes
    from oracle import build as obuild
    if not os.path.exists(obuild.LIB):
        obuild.build()
    from oracle.oracle import Oracle
    nt = _threads()

    def run(w, threads, timed_from):
        o = Oracle(w.scene, w.sensor, num_threads=threads)
        times, shifts = [], 0
        for fr in w.frames:
            s0 = o.stats()["shifts"]
            t0 = time.perf_counter()
            o.render(fr)
            dt = time.perf_counter() - t0
            if fr.index >= timed_from:
                times.append(dt)
                shifts += o.stats()["shifts"] - s0
        o.close()
        return times, shifts

    x0 = (width - crop) // 2
    w = scenes.glossy_dynamic(width=crop, height=crop, full_width=width, full_height=width, crop_x0=x0,
                              crop_y0=x0, frames=first + count)
    times, shifts = run(w, nt, first)
    scale = (width * width) / float(crop * crop)
    c1 = (width - 128) // 2
    w1 = scenes.glossy_dynamic(width=128, height=128, full_width=width, full_height=width, crop_x0=c1, crop_y0=c1,
                               frames=first + 1)
    t1, _ = run(w1, 1, first)
    tb, _ = run(scenes.cornell_box(frames=4), nt, 0)
    tn, _ = run(scenes.nlos_confocal(scan=64, frames=4), nt, 0)
    return {"value": round(len(times) / (sum(times) * scale), 6), "unit": "frames/s", "cores": nt, "kind": "oracle",
            "sample": f"{crop}x{crop} crop at ({x0},{x0}) of the {width}x{width} sequence, frames 0..{first + count - 1} "
                      f"rendered, frames {first}..{first + count - 1} timed ({[round(t, 3) for t in times]} s), "
                      f"rate divided by the pixel ratio {scale:g}; the crop clips the 30 px spatial disk at its "
                      f"border, so it does somewhat less work per pixel than the full frame",
            "shifts_per_s": round(shifts / sum(times), 1),
            "one_thread": {"frames_per_s": round(1.0 / (t1[0] * (width * width) / 16384.0), 6),
                           "sample": f"128x128 crop at ({c1},{c1}), frame {first} timed ({round(t1[0], 3)} s), "
                                     f"rate divided by the pixel ratio"},
            "tiny_box_64x64_4_frames_s": round(sum(tb), 4),
            "nlos_64x64_1024_bins_s_per_frame": [round(t, 3) for t in tn]}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1 (sharding across GPUs "
                                   "is not built)"}))
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.serving_only:
        s0 = serving(args, torch)
        s1 = serving(args, torch, graphs=True, solo=s0.pop("_solo_s"))
        s1.pop("_solo_s")
        print(json.dumps({"serving": s0, "serving_graphs": s1}), flush=True)
        return
    if args.c5_only:
        print(json.dumps({"specular_stress": specular_stress_leg(args, torch)}), flush=True)
        return
    if args.bvh_only:
        print(json.dumps({"bvh_builders": bvh_builders(args, torch)}), flush=True)
        return
    from paper_2605_11536_amd import scenes
    from paper_2605_11536_amd.tof import Renderer

    W = args.width
    nseq = max(60, max(int(x) for x in args.rmse_frames.split(",")) + 1)
    wl = scenes.glossy_dynamic(width=W, height=W, frames=nseq)
    sensor = wl.sensor
    P, B = W * W, sensor.b_tot

    def frame_at(i):
        fr = wl.frames[i % nseq]
        return scenes.Frame(index=i, cam_pos=fr.cam_pos, cam_fwd=fr.cam_fwd, cam_up=fr.cam_up,
                            fov_y_deg=fr.fov_y_deg, ortho_half=fr.ortho_half, light_pos=fr.light_pos,
                            xforms=fr.xforms)

    # the timed region: frames warmup .. warmup+steps-1 with kernel timing off
    r = Renderer(wl.scene, sensor)
    for i in range(args.warmup):
        r.render(frame_at(i))
    torch.cuda.synchronize()
    stats0 = r.stats()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record()
        r.render(frame_at(args.warmup + k))
        ev[k][1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    stats1 = r.stats()
    frame_ms = np.array([a.elapsed_time(b) for a, b in ev])
    fps = args.steps / elapsed
    dstats = {k: stats1[k] - stats0[k] for k in stats1}
    restir_out = r.fetch()
    r.close()
    # per-kernel times and work: the same frames again in a second context,
    # with HIP events around each kernel group during the same window
    r = Renderer(wl.scene, sensor)
    for i in range(args.warmup):
        r.render(frame_at(i))
    torch.cuda.synchronize()
    r.set_kernel_timing(True)
    for k in range(args.steps):
        r.render(frame_at(args.warmup + k))
    kt = r.kernel_times()
    r.set_kernel_timing(False)
    r.close()

    result = {
        "metric": "equal-RMSE frames/s vs plain ToF PT at 512^2; p50/p99 request latency",
        "value": round(fps, 3),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"glossy_dynamic {W}x{W}: ~92k triangles (160x160-cell displaced ground + 8 "
                               f"moving GGX spheres of 64x40 cells), 3 bounces, 256 bins (t0 12, width 0.1) + "
                               f"gate (17.0, 0.1), temporal + 1 spatial round (k 5, r 30 px), Newton shift",
                   "pixels": P, "planes": B, "frames_cycled": nseq},
        "latency_ms": {"p50": round(float(np.percentile(frame_ms, 50)), 3),
                       "p99": round(float(np.percentile(frame_ms, 99)), 3)},
    }

    # per-kernel times (HIP events on the render stream, timed region only)
    groups = [k for k in kt if k != "work_items"]
    kms = {k: kt[k]["ms"] for k in groups}
    kl = {k: kt[k]["launches"] for k in groups}
    result["kernel_ms_per_frame"] = {k: round(v / max(args.steps, 1), 3) for k, v in kms.items()}
    wi = kt["work_items"]
    result["work_items_per_frame"] = {k: v // args.steps for k, v in wi.items()}
    result["shift_stats_per_frame"] = {k: dstats[k] // args.steps for k in
                                       ("shifts", "shifts_ok", "newton_attempts", "newton_converged",
                                        "newton_paths_ok", "rays", "node_visits", "tri_tests")}
    nt = max(dstats["newton_attempts"], 1)
    result["newton"] = {"iters_per_converged": round(dstats["newton_iters"] / max(dstats["newton_converged"], 1), 4),
                        "newton_sr": round(dstats["newton_converged"] / nt, 4),
                        "actual_sr": round(dstats["newton_paths_ok"] / nt, 4)}
    result["rays_per_s"] = round(dstats["rays"] / elapsed, 1)
    result["shifts_per_s"] = round(dstats["shifts"] / elapsed, 1)
    result["integrity"] = {"bvh_overflow": dstats["bvh_overflow"], "bad_records": dstats["bad_records"]}
    result["traversal"] = {"nodes_per_ray": round(dstats["node_visits"] / max(dstats["rays"], 1), 2),
                           "tri_tests_per_ray": round(dstats["tri_tests"] / max(dstats["rays"], 1), 2),
                           "bytes_per_ray": round((NODE_BYTES * dstats["node_visits"] + TRI_BYTES * dstats["tri_tests"])
                                                  / max(dstats["rays"], 1), 1)}

    # roofline of the dominant kernel group (the byte and flop models above)
    dom = max(kms, key=lambda k: kms[k])
    avg_s = kms[dom] / max(kl[dom], 1) * 1e-3
    if dom in ("splat",):
        occ = float(np.count_nonzero(restir_out["hist"])) / restir_out["hist"].size
        per_launch = P * B * (SPLAT_BYTES + REC_HEAD_BYTES * occ)
        ach = per_launch / avg_s / 1e9
        result["roofline"] = {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": None, "kernel": "k_splat",
                              "avg_launch_ms": round(avg_s * 1e3, 4)}
        mt = measured_traffic(dom)
        if mt:
            result["roofline"]["traffic"] = mt["bytes_per_launch"]
            result["roofline"]["traffic_frames"] = mt["frames"]
    else:
        w = kt[dom]["work"]
        per_launch = valu_flops(w) / max(kl[dom], 1)
        ach = per_launch / avg_s / 1e12
        kname = {"spatial_mis": "k_mis", "temporal_mis": "k_mis", "spatial_fwd": "k_fwd", "temporal_fwd": "k_fwd",
                 "spatial_vis": "k_vis", "temporal_vis": "k_vis",
                 "spatial_merge": "k_merge", "temporal_merge": "k_merge", "initial": "k_initial",
                 "gbuffer": "k_gbuffer"}.get(dom, dom)
        result["roofline"] = {"bound": "alu", "achieved": round(ach, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                              "frac": round(ach / FP32_PEAK_TFLOPS, 5),
                              "traffic": None,
                              "kernel": f"{kname} ({dom})", "avg_launch_ms": round(avg_s * 1e3, 4),
                              "flops_per_launch": per_launch}
        mt = measured_traffic(dom)
        if mt:
            result["roofline"]["traffic"] = mt["bytes_per_launch"]
            result["roofline"]["traffic_frames"] = mt["frames"]
    # the streaming passes against HBM: the splat over every (pixel, plane)
    if kl.get("splat"):
        occ = float(np.count_nonzero(restir_out["hist"])) / restir_out["hist"].size
        sp_s = kms["splat"] / kl["splat"] * 1e-3
        sp_bytes = P * B * (SPLAT_BYTES + REC_HEAD_BYTES * occ)
        result["splat_hbm"] = {"achieved_GBs": round(sp_bytes / sp_s / 1e9, 1),
                               "frac": round(sp_bytes / sp_s / 1e9 / HBM_PEAK_GBS, 4),
                               "bytes_per_launch": int(sp_bytes), "occupancy": round(occ, 5),
                               "avg_launch_ms": round(sp_s * 1e3, 4), "traffic": measured_traffic("splat")}
        if result["splat_hbm"]["traffic"]:
            # what the counters say the kernel moves (whole cache lines, not only the algorithmic bytes)
            tb = result["splat_hbm"]["traffic"]["bytes_per_launch"]
            result["splat_hbm"]["measured_GBs"] = round(tb / sp_s / 1e9, 1)
            result["splat_hbm"]["measured_frac"] = round(tb / sp_s / 1e9 / HBM_PEAK_GBS, 4)

    # ... and the resampling merge, from its algorithmic bytes per item and task
    merge = {}
    for pas, K in (("temporal", 1), ("spatial", max(int(sensor.spatial_k), 1))):
        g = pas + "_merge"
        items, tasks = wi.get(pas + "_items", 0), wi.get(pas + "_tasks", 0)
        if kms.get(g) and items:
            mb = items * MERGE_ITEM_BYTES + tasks * (MERGE_TASK_BYTES + 4 * K)
            gbs = mb / (kms[g] * 1e-3) / 1e9
            merge[pas] = {"achieved_GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                          "bytes_per_frame": int(mb / max(args.steps, 1)),
                          "ms_per_frame": round(kms[g] / max(args.steps, 1), 3), "launches": kl[g],
                          "traffic": measured_traffic(g)}
            if merge[pas]["traffic"]:
                tgbs = merge[pas]["traffic"]["bytes_per_launch"] * kl[g] / (kms[g] * 1e-3) / 1e9
                merge[pas]["measured_GBs"] = round(tgbs, 1)
                merge[pas]["measured_frac"] = round(tgbs / HBM_PEAK_GBS, 4)
    if merge:
        result["merge_hbm"] = merge

    # the same window with pairwise MIS in the spatial pass: frames/s with
    # timing off, then the kernel groups over the window in a second context
    if not args.no_pairwise:
        import dataclasses
        ps = dataclasses.replace(sensor, mis_mode=1)
        r = Renderer(wl.scene, ps)
        for i in range(args.warmup):
            r.render(frame_at(i))
        torch.cuda.synchronize()
        st0 = r.stats()
        t0 = time.perf_counter()
        for k in range(args.steps):
            r.render(frame_at(args.warmup + k))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st1 = r.stats()
        r.close()
        r = Renderer(wl.scene, ps)
        for i in range(args.warmup):
            r.render(frame_at(i))
        torch.cuda.synchronize()
        r.set_kernel_timing(True)
        for k in range(args.steps):
            r.render(frame_at(args.warmup + k))
        ktp = r.kernel_times()
        r.close()
        result["pairwise"] = {"frames_per_s": round(args.steps / el, 3), "ms_per_step": round(1e3 * el / args.steps, 3),
                              "shifts_per_frame": (st1["shifts"] - st0["shifts"]) // args.steps,
                              "rays_per_frame": (st1["rays"] - st0["rays"]) // args.steps,
                              "kernel_ms_per_frame": {k: round(v["ms"] / args.steps, 3) for k, v in ktp.items()
                                                      if k != "work_items"}}

    # the same window with the launch shape tof_autotune picks (tuned on
    # frames 0..7 of the sequence, outside the timed region)
    if not args.no_autotune:
        r = Renderer(wl.scene, sensor)
        t0 = time.perf_counter()
        cfg = r.autotune([frame_at(i) for i in range(8)])
        t_tune = time.perf_counter() - t0
        for i in range(args.warmup):
            r.render(frame_at(i))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            r.render(frame_at(args.warmup + k))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        r.close()
        result["autotuned"] = {"launch_config": cfg, "autotune_s": round(t_tune, 2),
                               "frames_per_s": round(args.steps / el, 3), "ms_per_step": round(1e3 * el / args.steps, 3)}

    # equal RMSE against plain ToF PT on the same GPU, over the sequence
    if not args.no_equal_rmse:
        import dataclasses
        result["equal_rmse"] = equal_rmse_seq(
            wl, frame_at, [("gbh", sensor), ("pairwise", dataclasses.replace(sensor, mis_mode=1))], args, torch,
            Renderer)
        result["equal_rmse_gate_only"] = gate_only(wl, frame_at, args, torch, Renderer)
    if not args.no_bins_sweep:
        result["cost_vs_bins"] = bins_sweep(wl, frame_at, args, torch, Renderer)
    if not args.no_serving:
        result["serving"] = serving(args, torch)
        # the same arrivals with every frame recorded into a graph and
        # launched as one (tof_server_set_graphs)
        sg = serving(args, torch, graphs=True, solo=result["serving"].pop("_solo_s"))
        result["serving_graphs"] = {k: sg[k] for k in ("latency_ms", "service_ms", "queueing_ms", "latency_ms_p50_by_kind",
                                                       "latency_ms_p99_by_kind", "frames_per_s", "wall_s")}
    if not args.no_bvh:
        result["bvh_builders"] = bvh_builders(args, torch)
    if not args.no_c5:
        result["specular_stress"] = specular_stress_leg(args, torch)
    if args.copy_probe:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters give
        # the scale from counter units to bytes for the traffic figure
        n = args.copy_probe // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_probe_bytes"] = 4 * n
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(W, args.warmup, args.cpu_frames, args.cpu_crop)
    print(json.dumps(result), flush=True)


SERVE_RES = (128, 256, 512, 1024)
SERVE_BINS = (1, 64, 256)
SERVE_NLOS_SCAN = (32, 64)
SERVE_NLOS_BINS = (256, 1024)


def serving(args, torch, graphs=False, solo=None):
    """Batched serving: streams arrive as a Poisson process.  Three in four are
    render streams: a box scene of the tiny-workload generator with its own
    seed, a resolution drawn from SERVE_RES, a gate width from U[0.01, 0.2]
    and a bin count from SERVE_BINS (bins over path lengths [2, 8]).  One in
    four is an NLOS simulation: a confocal scan of the relay wall with the
    hidden torus (12.5k triangles), SERVE_NLOS_SCAN scan points per side and
    SERVE_NLOS_BINS bins of 0.004 from the wall.  Each asks for `serve_frames`
    frames, one every `serve_period_ms` from its arrival (open loop).  The
    server admits streams by HBM footprint; a frame's latency runs from its
    scheduled submission to its completion (admission wait included); its
    service time is the GPU time between the start and the end of its work on
    its HIP stream (under the load of the others), its queueing delay the
    rest.  The host loop submits due frames, polls tickets and closes a
    stream once its last frame is done."""
    from paper_2605_11536_amd import scenes
    from paper_2605_11536_amd.tof import Renderer, Server, tof_footprint
    rng = np.random.default_rng(args.serve_seed)
    n, F, period = args.serve_streams, args.serve_frames, args.serve_period_ms * 1e-3

    def render_stream(W, nb, gw, seed):
        return scenes.cornell_box(width=W, height=W, frames=F, seed=seed, gate_width=gw, n_bins=nb, bin_t0=2.0,
                                  bin_width=6.0 / nb)

    def nlos_stream(scan, nb, seed):
        return scenes.nlos_confocal(scan=scan, frames=F, seed=seed, torus_nu=125, torus_nv=50, n_bins=nb)

    wls, fps_, kinds = [], [], []
    for i in range(n):
        if rng.random() < 0.25:
            wl = nlos_stream(int(rng.choice(SERVE_NLOS_SCAN)), int(rng.choice(SERVE_NLOS_BINS)), 1000 + i)
            kinds.append("nlos")
        else:
            W = int(rng.choice(SERVE_RES))
            nb = int(rng.choice(SERVE_BINS))
            wl = render_stream(W, nb, float(rng.uniform(0.01, 0.2)), 1000 + i)
            kinds.append("render")
        wls.append(wl)
        fps_.append(tof_footprint(wl.scene, wl.sensor))
    # solo frame time of every class: one stream alone, frames 1..F-1 timed;
    # the mix draws render classes uniformly, NLOS classes uniformly (taken
    # from an earlier run when given, so that both runs share the arrivals)
    classes = [] if solo is not None else (
        [(f"{W}x{nb}", render_stream(W, nb, 0.1, 1)) for W in SERVE_RES for nb in SERVE_BINS] +
        [(f"nlos{sc}x{nb}", nlos_stream(sc, nb, 1)) for sc in SERVE_NLOS_SCAN for nb in SERVE_NLOS_BINS])
    solo = dict(solo) if solo is not None else {}
    for name, wl in classes:
        r = Renderer(wl.scene, wl.sensor)
        r.render(wl.frames[0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for fr in wl.frames[1:]:
            r.render(fr)
        torch.cuda.synchronize()
        solo[name] = (time.perf_counter() - t0) / max(F - 1, 1)
        r.close()
    mean_render = float(np.mean([v for k, v in solo.items() if not k.startswith("nlos")]))
    mean_nlos = float(np.mean([v for k, v in solo.items() if k.startswith("nlos")]))
    mean_solo = 0.75 * mean_render + 0.25 * mean_nlos
    rate = args.serve_rate if args.serve_rate > 0 else args.serve_load / (F * mean_solo)
    arrive = np.cumsum(rng.exponential(1.0 / rate, n))
    arrive -= arrive[0]
    budget = int(args.serve_budget_gib * (1 << 30))
    srv = Server(hbm_budget_bytes=budget)
    srv.set_graphs(graphs)
    due = sorted((arrive[i] + j * period, i, j) for i in range(n) for j in range(F))
    sid, outs, left = {}, {}, [F] * n
    pending = {}
    lat, adm_wait, lat_res, svc, queue, lat_kind = [], [], {}, [], [], {}
    peak_used, peak_adm, used_area = 0, 0, 0.0
    k = 0
    t_open = t_close = 0.0
    t0 = time.perf_counter()
    last = t0
    while k < len(due) or pending:
        now = time.perf_counter() - t0
        while k < len(due) and due[k][0] <= now:
            ts, i, j = due[k]
            k += 1
            if j == 0:
                ta = time.perf_counter()
                sid[i], _ = srv.open(wls[i].scene, wls[i].sensor)
                outs[i] = srv.outputs(sid[i], pt=False)
                t_open += time.perf_counter() - ta
            pending[srv.submit(sid[i], wls[i].frames[j], outs[i])] = (i, j, ts)
        for t in list(pending):
            fin, gpu_ms = srv.query_timed(t)
            if fin:
                i, j, ts = pending.pop(t)
                done = time.perf_counter() - t0
                lat.append(done - ts)
                if gpu_ms is not None:
                    svc.append(gpu_ms * 1e-3)
                    queue.append(max(done - ts - gpu_ms * 1e-3, 0.0))
                lat_kind.setdefault(kinds[i], []).append(done - ts)
                lat_res.setdefault(wls[i].sensor.width, []).append(done - ts)
                if j == 0:
                    adm_wait.append(done - ts)
                left[i] -= 1
                if left[i] == 0:
                    ta = time.perf_counter()
                    srv.close_stream(sid[i])
                    t_close += time.perf_counter() - ta
                    del outs[i]
        info = srv.info()
        tn = time.perf_counter()
        used_area += info["used_bytes"] * (tn - last)
        last = tn
        peak_used = max(peak_used, info["used_bytes"])
        peak_adm = max(peak_adm, info["admitted"])
        if tn - t0 > args.serve_timeout_s:
            raise RuntimeError(f"serving leg exceeded {args.serve_timeout_s} s")
        time.sleep(2e-4)
    wall = time.perf_counter() - t0
    srv.close()
    lat = np.array(lat) * 1e3
    pp = sum(w.sensor.width * w.sensor.height * w.sensor.b_tot for w in wls) * F
    return {"_solo_s": solo, "streams": n, "graphs": graphs, "frames_per_stream": F,
            "arrival_rate_per_s": round(rate, 4),
            "offered_load": round(rate * F * mean_solo, 3),
            "solo_frame_ms": {k: round(v * 1e3, 3) for k, v in solo.items()},
            "host_open_s": round(t_open, 3), "host_close_s": round(t_close, 3),
            "frame_period_ms": args.serve_period_ms, "hbm_budget_gib": args.serve_budget_gib,
            "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                           "p99": round(float(np.percentile(lat, 99)), 3),
                           "max": round(float(lat.max()), 3)},
            "service_ms": {"p50": round(float(np.percentile(svc, 50)) * 1e3, 3),
                           "p99": round(float(np.percentile(svc, 99)) * 1e3, 3)},
            "queueing_ms": {"p50": round(float(np.percentile(queue, 50)) * 1e3, 3),
                            "p99": round(float(np.percentile(queue, 99)) * 1e3, 3)},
            "latency_ms_p50_by_kind": {k: round(float(np.percentile(v, 50)) * 1e3, 3) for k, v in sorted(lat_kind.items())},
            "latency_ms_p99_by_kind": {k: round(float(np.percentile(v, 99)) * 1e3, 3) for k, v in sorted(lat_kind.items())},
            "nlos_streams": kinds.count("nlos"),
            "first_frame_latency_ms_p50": round(float(np.percentile(adm_wait, 50)) * 1e3, 3),
            "latency_ms_p50_by_res": {str(k): round(float(np.percentile(v, 50)) * 1e3, 3)
                                      for k, v in sorted(lat_res.items())},
            "frames_per_s": round(n * F / wall, 3), "pixel_planes_per_s": round(pp / wall, 1),
            "wall_s": round(wall, 3), "peak_admitted": peak_adm,
            "peak_used_gib": round(peak_used / (1 << 30), 2),
            "mean_used_gib": round(used_area / wall / (1 << 30), 2),
            "footprint_gib": {"min": round(min(fps_) / (1 << 30), 3), "max": round(max(fps_) / (1 << 30), 3),
                              "sum": round(sum(fps_) / (1 << 30), 2)},
            "mix": {"kind": kinds, "res": [int(w.sensor.width) for w in wls], "bins": [int(w.sensor.n_bins) for w in wls]}}


def equal_rmse_seq(wl, frame_at, variants, args, torch, Renderer, planes=("gate_image", "histogram")):
    """Equal RMSE against plain ToF PT on the same GPU, over the sequence.

    Each ReSTIR variant (name, sensor) renders frames 0..F of the sequence (F
    = the last frame listed in --rmse-frames); at each listed frame its output
    is compared with a plain-PT reference of that frame (ref_calls x
    ref_trees path trees per pixel), whose own variance is removed from the
    error.  Plain PT at s spp has MSE_1 / s, MSE_1 measured at that frame from
    four independent 1-spp renders, so the spp that matches ReSTIR is s* =
    MSE_1 / MSE_restir and its frame time s* t_1, t_1 timed over 20 frames of
    the sequence.  ReSTIR's frame time is its event time averaged over the
    listed window.  Speedup = t_PT(s*) / t_ReSTIR per listed frame, and their
    mean.  Everything stays on the device: the outputs are large (512^2 x 256
    bins)."""
    import dataclasses
    fl = sorted(int(x) for x in args.rmse_frames.split(","))
    F = fl[-1]
    keys = [k for k, name in (("image", "gate_image"), ("hist", "histogram")) if name in planes]
    outs, t_restir = {}, {}
    for name, sensor in variants:
        r = Renderer(wl.scene, sensor)
        outs[name] = {}
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(F + 1)]
        for i in range(F + 1):
            ev[i][0].record()
            r.render(frame_at(i))
            ev[i][1].record()
            if i in fl:
                outs[name][i] = {k: getattr(r, "out_" + k).double().clone() for k in keys}
        torch.cuda.synchronize()
        r.close()
        t_restir[name] = float(np.mean([ev[i][0].elapsed_time(ev[i][1]) for i in range(fl[0], F + 1)])) * 1e-3
    base = variants[0][1]
    ref_sensor = dataclasses.replace(base, temporal=0, spatial_rounds=0, m_init=args.ref_trees, shrink_k=1.0)
    pt_sensor = dataclasses.replace(base, temporal=0, spatial_rounds=0, m_init=1, shrink_k=1.0)
    q = Renderer(wl.scene, ref_sensor)
    p = Renderer(wl.scene, pt_sensor)
    ref_spp = args.ref_calls * args.ref_trees
    mse = {name: [] for name, _ in variants}
    for f in fl:
        acc = {k: torch.zeros_like(outs[variants[0][0]][f][k]) for k in keys}
        for c in range(args.ref_calls):
            q.render(dataclasses.replace(frame_at(f), index=10_000_000 + 1000 * f + c))
            for k in keys:
                acc[k] += getattr(q, "out_pt_" + k)
        ref = {k: acc[k] / args.ref_calls for k in keys}
        mse1 = {k: 0.0 for k in keys}
        for c in range(4):
            p.render(dataclasses.replace(frame_at(f), index=20_000_000 + 1000 * f + c))
            for k in keys:
                mse1[k] += float(((getattr(p, "out_pt_" + k).double() - ref[k]) ** 2).mean()) / 4
        for name, _ in variants:
            row = {}
            for k in keys:
                m1 = mse1[k] * (1.0 - 1.0 / ref_spp)
                mr = max(float(((outs[name][f][k] - ref[k]) ** 2).mean()) - mse1[k] / ref_spp, 1e-30)
                row[k] = (m1, mr)
            mse[name].append(row)
        del ref, acc
    q.close()
    # plain PT's frame time over consecutive frames (it pays the same geometry update)
    nrep = 20
    p.render(dataclasses.replace(frame_at(nrep), index=30_000_000))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(nrep):
        p.render(dataclasses.replace(frame_at(i), index=30_000_001 + i))
    torch.cuda.synchronize()
    t_pt = (time.perf_counter() - t0) / nrep
    p.close()
    res = {"frames": fl, "reference_spp": ref_spp, "pt_1spp_ms": round(1e3 * t_pt, 3)}
    for name, _ in variants:
        out = {"restir_ms_per_frame": round(1e3 * t_restir[name], 3),
               "restir_frames_per_s": round(1.0 / t_restir[name], 3)}
        for k, pname in (("image", "gate_image"), ("hist", "histogram")):
            if k not in keys:
                continue
            s_star = [row[k][0] / row[k][1] for row in mse[name]]
            sp = [(x * t_pt) / t_restir[name] for x in s_star]
            out[pname] = {"restir_rmse": [round(math.sqrt(row[k][1]), 8) for row in mse[name]],
                          "pt_1spp_rmse": [round(math.sqrt(row[k][0]), 8) for row in mse[name]],
                          "pt_spp_at_equal_rmse": [round(x, 3) for x in s_star],
                          "speedup_per_frame": [round(x, 4) for x in sp],
                          "speedup": round(float(np.mean(sp)), 4)}
        res[name] = out
    return res


def gate_only(wl, frame_at, args, torch, Renderer):
    """The same scene and sequence with the gate alone (no histogram bins):
    the regime the paper targets (a narrow gate), same reuse settings, with 1,
    2, 4, 8 and 16 path trees per pixel (initial candidates) and with either
    MIS of the spatial pass."""
    import dataclasses
    variants = []
    for m_init in (1, 2, 4, 8, 16):
        for mis in (0, 1):
            name = f"m_init{m_init}_" + ("pairwise" if mis else "gbh")
            variants.append((name, dataclasses.replace(wl.sensor, n_bins=0, m_init=m_init, mis_mode=mis)))
    return equal_rmse_seq(wl, frame_at, variants, args, torch, Renderer, planes=("gate_image",))


def specular_stress_leg(args, torch, warm=2, timed=3):
    """The near-specular stress configuration (0.95M triangles, 30% GGX with
    alpha 0.01, 4 bounces, 512 bins + gate, spline camera) at 1920x1080
    (1.06 G pixel-planes, about 220 GiB of device memory): frames/s, ms per
    frame, shifts and rays per frame, timing off, frames warm..warm+timed-1."""
    from paper_2605_11536_amd import scenes
    from paper_2605_11536_amd.tof import Renderer, tof_footprint
    W, H = args.c5_width, args.c5_height
    torch.cuda.empty_cache()   # what the earlier legs' tensors left in torch's cache
    t0 = time.perf_counter()
    wl = scenes.specular_stress(width=W, height=H, frames=warm + timed)
    t_scene = time.perf_counter() - t0
    t0 = time.perf_counter()
    r = Renderer(wl.scene, wl.sensor)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0

    def window():
        ms = []
        for i in range(warm):
            r.render(wl.frames[i])
        torch.cuda.synchronize()
        s0 = r.stats()
        for i in range(warm, warm + timed):
            t0 = time.perf_counter()
            r.render(wl.frames[i])
            torch.cuda.synchronize()
            ms.append(1e3 * (time.perf_counter() - t0))
        return ms, s0, r.stats()

    ms_default, _, _ = window()
    # the launch shape tuned on the same frames (tof_autotune drops the
    # history, so the window starts from an empty one again)
    t0 = time.perf_counter()
    cfg = r.autotune(wl.frames[:warm + timed - 1])
    t_tune = time.perf_counter() - t0
    ms, st0, st1 = window()
    r.close()
    d = {k: (st1[k] - st0[k]) // timed for k in ("shifts", "shifts_ok", "newton_attempts", "newton_converged",
                                                   "newton_paths_ok", "rays")}
    sc = wl.scene
    ggx = sum(2 * int(sc.obj_grid[o, 0]) * int(sc.obj_grid[o, 1]) for o in range(sc.num_objects)
              if sc.obj_type[o] == scenes.OBJ_GRID and sc.mat_type[sc.obj_material[o]] == 1)
    return {"workload": f"specular_stress {W}x{H}: {sc.num_triangles} triangles, "
                        f"{round(100 * ggx / sc.num_triangles, 1)}% GGX (alpha 0.01), 4 bounces, "
                        f"{wl.sensor.n_bins} bins + gate, temporal + 1 spatial round, Newton shift",
            "frames": [warm, warm + timed - 1], "ms_per_frame": [round(x, 2) for x in ms],
            "frames_per_s": round(1e3 * timed / sum(ms), 3), "launch_config": cfg, "autotune_s": round(t_tune, 2),
            "default_launch": {"ms_per_frame": [round(x, 2) for x in ms_default],
                               "frames_per_s": round(1e3 * timed / sum(ms_default), 3)},
            "per_frame": d,
            "hbm_gib": round(tof_footprint(wl.scene, wl.sensor) / (1 << 30), 1),
            "scene_build_s": round(t_scene, 2), "context_create_s": round(t_create, 2),
            "bvh_overflow": st1["bvh_overflow"], "bad_records": st1["bad_records"]}


def bvh_builders(args, torch, warm=5, timed=5):
    """The objects' trees built on the host (binned SAH) and on the device
    (agglomerative clustering over a Morton-sorted order): build time (wall
    clock around the build, readbacks included), 4-wide nodes, refit levels,
    and what the trees cost the frame -- ms per frame (timing off) and node
    visits and triangle tests per visibility ray over frames
    warm..warm+timed-1 -- on the glossy scene at the benchmark's size and on
    the near-specular stress scene (0.95M triangles) at 480x270."""
    from paper_2605_11536_amd import scenes
    from paper_2605_11536_amd.tof import BVH_DEVICE, BVH_HOST, Renderer
    torch.cuda.empty_cache()
    cases = (("glossy_dynamic 512x512", lambda: scenes.glossy_dynamic(width=args.width, height=args.width,
                                                                      frames=warm + timed)),
             ("specular_stress 480x270", lambda: scenes.specular_stress(width=480, height=270, frames=warm + timed)))
    out = {}
    for name, make in cases:
        wl = make()
        res = {"triangles": int(wl.scene.num_triangles)}
        for b, key in ((BVH_HOST, "host"), (BVH_DEVICE, "device")):
            r = Renderer(wl.scene, wl.sensor, bvh_builder=b)
            info = r.bvh_info()
            for i in range(warm):
                r.render(wl.frames[i])
            torch.cuda.synchronize()
            s0 = r.stats()
            t0 = time.perf_counter()
            for i in range(warm, warm + timed):
                r.render(wl.frames[i])
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            s1 = r.stats()
            r.close()
            rays = max(s1["rays"] - s0["rays"], 1)
            res[key] = {"build_ms": round(info["build_ms"], 2), "nodes": info["num_nodes"],
                        "levels": info["num_levels"], "rounds": info["rounds"],
                        "ms_per_frame": round(1e3 * el / timed, 3),
                        "nodes_per_ray": round((s1["node_visits"] - s0["node_visits"]) / rays, 3),
                        "tri_tests_per_ray": round((s1["tri_tests"] - s0["tri_tests"]) / rays, 3)}
        out[name] = res
    return out


def bins_sweep(wl, frame_at, args, torch, Renderer, bins=(4, 16, 64, 256), warm=5, timed=5):
    """Cost against the number of histogram bins B over the same path-length
    range (Sec. 4.5: reuse cost grows with the bins a pixel holds): frames/s,
    shifts and rays per frame, timing off, frames warm..warm+timed-1."""
    import dataclasses
    s0 = wl.sensor
    span = s0.n_bins * s0.bin_width
    out = []
    for nb in bins:
        sensor = dataclasses.replace(s0, n_bins=nb, bin_width=span / nb)
        r = Renderer(wl.scene, sensor)
        for i in range(warm):
            r.render(frame_at(i))
        torch.cuda.synchronize()
        st0 = r.stats()
        t0 = time.perf_counter()
        for i in range(warm, warm + timed):
            r.render(frame_at(i))
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / timed
        st1 = r.stats()
        r.close()
        out.append({"bins": nb, "planes": nb + 1, "ms_per_frame": round(1e3 * dt, 3),
                    "frames_per_s": round(1.0 / dt, 3),
                    "shifts_per_frame": (st1["shifts"] - st0["shifts"]) // timed,
                    "rays_per_frame": (st1["rays"] - st0["rays"]) // timed})
    return {"frames": [warm, warm + timed - 1], "points": out}


if __name__ == "__main__":
    main()
