#!/usr/bin/env python3
"""Mapping-iteration benchmark of the differentiable tile rasterizer.

One step is one mapping iteration over a keyframe window: projection and
binning, per-tile sort, forward render, planar-regulariser gradient, backward
pixel pass with the L1 photometric term fused in (loss and its gradient
formed per pixel), projection backward and the Adam update, for all views of
the window.  Inputs are synthetic (a room-shaped scene standing
in for the paper's indoor sequences) and resident in HBM before timing.

Prints one JSON line.  Extra fields: Mpix/s, the p10/p50/p90 of 50 single
graph replays (after the timed region), per-kernel milliseconds, the
roofline of the dominant kernel (credited FP32 VALU lane-operations from exact
pair counts, against the published FP32 vector peak: 157.3 TFLOP/s, i.e.
78.6 T lane-operations/s with an FMA counted once), and the CPU oracle timed
stage by stage over one whole iteration of the same workload.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("mapping iters/s (fwd+bwd, 10-KF window, 1200×680, 300k "
          "Gaussians) + Mpix/s")
# Published FP32 vector peak, 157.3 TFLOP/s, in lane-operations (an FMA counts
# once): 256 CUs x 128 FP32 lanes x 2.4 GHz.  Half of it is reached only with
# packed (two-lane) FP32 instructions, which these kernels do not use.
PEAK_LANE_OPS = 256 * 128 * 2.4e9
# Credited FP32 VALU lane-operations per pair (what the method must compute).
# Forward: 2 per examined pair (box test), +12 per in-box pair (offset,
# exponent, exponential, opacity, clamp, threshold), +7 per contributing pair
# (transmittance, stop test, weight, three colour FMAs).  Backward: 45 per
# contributing pair (alpha recomputed, transmittance recovered, colour, alpha,
# opacity, mean and conic gradients) and 14 per in-box pair before the
# pixel's last contributor that does not contribute (alpha recomputed and
# rejected).  "revisit" counts all in-box pairs before n_last, contributing
# ones included, so the backward credits revisit - contributing at 14.
FWD_OPS = dict(examined=2, inbox=12, contributing=7)
BWD_OPS = dict(revisit_only=14, contributing=45)


def credited_ops(cnt):
    """(forward, backward) credited lane-operations for the pair counts of
    one launch."""
    fwd = sum(FWD_OPS[k] * cnt[k] for k in FWD_OPS)
    c = dict(cnt, revisit_only=cnt["revisit"] - cnt["contributing"])
    bwd = sum(BWD_OPS[k] * c[k] for k in BWD_OPS)
    return fwd, bwd
LR = (1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3)   # mean, log_scale, quat, opacity, rgb
LAMBDA_COLOR, LAMBDA_REG, REG_FLOOR = 1.0, 1.0, 0.01
LAMBDA_PHOTO = 0.2   # weight of the SSIM term inside the colour loss
DENSIFY_SIGMA = 64   # split threshold: dominated pixels per keyframe
INSERT_TAU = 0.02    # distance threshold of the paper's insertion test (m)


TRAFFIC_FILE = os.path.join(ROOT, "profiles",
                            "render_window10-1200x680-300k_tile32_counters.txt")


def measured_counters(kernel):
    """From the committed rocprofv3 counter summary of the dominant kernel:
    HBM bytes per dispatch (FETCH_SIZE and WRITE_SIZE scaled by a known-size
    copy), VALU issue (instructions x 4 cycles over the SIMD cycles) and the
    FP32 arithmetic rate (TFLOP/s); None each when the summary is for
    another kernel or the kernel's sources changed since it was taken."""
    import hashlib
    none = {"traffic": None, "valu_issue": None, "fp32_tflops": None}
    try:
        kv = dict(l.split(": ", 1) for l in open(TRAFFIC_FILE).read().splitlines()
                  if l and not l.startswith("#") and ": " in l)
        name = kv["traffic_kernel"]
        if not (name.startswith(kernel + ">") or name.startswith(kernel + ",")):
            return none
        h = hashlib.sha256()
        for src in kv["traffic_sources"].split():
            h.update(open(os.path.join(ROOT, src), "rb").read())
        if h.hexdigest() != kv["traffic_sources_sha256"].strip():
            return none
        return {"traffic": int(kv["traffic_bytes"]),
                "valu_issue": float(kv["valu_issue"]),
                "fp32_tflops": float(kv["fp32_tflops"])}
    except (OSError, KeyError, ValueError):
        return none


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    import synth
    if name == "window":
        return synth.config2(0, 10, "1200x680")
    if name == "window640":
        return synth.config2(0, 10, "640x480")
    if name == "single":
        return synth.config1()
    if name == "small":
        return synth.config0()
    raise ValueError(name)


def iteration_ms(w, S, steps=10, warmup=3):
    """Eager mapping iterations (project, sort, render, L1 + planar
    gradients, backward, Adam) on another workload: ms per iteration."""
    import torch
    from paper_2504_02437_amd import raster as R
    dev = "cuda"
    params = R.ParamBuffer.from_gaussians(w.gaussians, device=dev)
    grad, m, v = params.zeros_like(), params.zeros_like(), params.zeros_like()
    rast = R.Rasterizer(w.cameras, params.capacity, S, device=dev)
    rast.fit_key_capacity(params)
    target = torch.from_numpy(w.targets).to(dev)
    dL = torch.empty_like(rast.rgb)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    step_dev = torch.ones(1, dtype=torch.int32, device=dev)

    def step():
        grad.data.zero_()
        loss.zero_()
        rast.forward(params)
        R.planar_reg(params, LAMBDA_REG, REG_FLOOR, grad, loss)
        rast.backward_l1(params, target, LAMBDA_COLOR, grad, loss)
        R.adam(params, grad, m, v, LR, 0.9, 0.999, 1e-15, step_dev)
        step_dev.add_(1)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    if rast.status()[0]:
        rast.fit_key_capacity(params)
    a, b = (torch.cuda.Event(enable_timing=True) for _ in range(2))
    a.record()
    for _ in range(steps):
        step()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def insertion_stress(S, n0=50_000, n_kf=200):
    """The growth run: a 50k-Gaussian initial map as the map initialisation
    builds it from back-projected VO points (points on the room's surfaces,
    the heuristic one-pixel isotropic footprint log(z / f) for their distance
    z from the first keyframe, opacity 0.5), then n_kf keyframes on the random
    walk, each rendered and given 96 patches x 9 candidates through the
    accumulated-alpha mask (capacity 50k + n_kf * 864)."""
    import numpy as np
    import torch
    import synth
    from paper_2504_02437_amd import raster as R
    dev = "cuda"
    g = synth.room_gaussians(np.random.default_rng([3, 1]), n0)
    kf0 = synth.insertion_stream(0, 1)[0].camera
    cam_pos = -kf0.R.T.astype(np.float64) @ kf0.t.astype(np.float64)
    z = np.linalg.norm(g.mean.T.astype(np.float64) - cam_pos, axis=1)
    g.log_scale[:] = np.log(np.maximum(z, 0.1) / kf0.fx).astype(np.float32)
    g.quat[:] = np.array([[1.0], [0.0], [0.0], [0.0]], np.float32)
    g.opacity_logit[:] = 0.0
    cap = n0 + n_kf * 96 * 9
    params = R.ParamBuffer.from_gaussians(g, capacity=cap, device=dev)
    m, v = params.zeros_like(), params.zeros_like()
    kfs = synth.insertion_stream(0, n_kf)
    rast = R.Rasterizer([kfs[0].camera], cap, S, device=dev,
                        key_capacity=R.default_key_capacity(cap, 1))
    t_render, t_insert = [], []
    for i, kf in enumerate(kfs):
        rast.set_cameras([kf.camera])
        img = torch.from_numpy(kf.image).to(dev)
        pts = torch.from_numpy(kf.pts_uvd).to(dev)
        a, b, c = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        a.record()
        rast.forward(params)
        b.record()
        R.insert_gaussians(params, m, v, rast.cams_dev, kf.camera.width,
                           kf.camera.height, img, rast.T[0].contiguous(), pts)
        c.record()
        torch.cuda.synchronize()
        if rast.status()[0]:
            raise RuntimeError("key capacity exceeded in the insertion run")
        t_render.append(a.elapsed_time(b))
        t_insert.append(b.elapsed_time(c))
    return {"keyframes": n_kf, "start_n": n0, "final_n": params.n(),
            "capacity": cap, "ms_per_kf_insert": float(np.mean(t_insert)),
            "ms_per_kf_render": float(np.mean(t_render))}


def host_cpus():
    """The host CPUs as the process sees them: nproc (every logical CPU of
    the machine), the CPUs this process may run on (its affinity mask), the
    OpenMP thread budget the environment sets, and lscpu's description."""
    info = {"nproc": os.cpu_count()}
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        info["affinity"] = os.cpu_count()
    env = os.environ.get("OMP_NUM_THREADS", "")
    info["omp_num_threads"] = int(env) if env.isdigit() else None
    keys = {"Model name": "model", "Socket(s)": "sockets",
            "Core(s) per socket": "cores_per_socket",
            "Thread(s) per core": "threads_per_core", "CPU max MHz": "max_mhz"}
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True,
                             timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in keys:
                info[keys[k.strip()]] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    if "model" not in info:
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    info["model"] = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    return info


def cpu_threads(info):
    """Threads for the CPU baseline: every CPU the process may use, within
    the thread budget the environment grants (OMP_NUM_THREADS)."""
    n = info.get("affinity") or info.get("nproc") or 1
    if info.get("omp_num_threads"):
        n = min(n, info["omp_num_threads"])
    return max(1, n)


def cpu_baseline(w, threads, views=None):
    """The CPU oracle, as it stands, timed stage by stage over the first
    `views` views of the workload (all of them by default: one whole mapping
    iteration), scaled to window iterations/s."""
    import numpy as np
    import oracle
    V = len(w.cameras)
    views = views or V
    cam = list(w.cameras[:views])
    W, H = cam[0].width, cam[0].height
    st = {}
    t = time.perf_counter()

    def lap(name):
        nonlocal t
        now = time.perf_counter()
        st[name] = round(now - t, 3)
        t = now

    t0 = t
    p64 = oracle.params64(w.gaussians)
    proj = oracle.project(p64, cam, 16, publish=True, nthreads=threads)
    lap("project")
    bins = oracle.bin_sort(proj, 16, W, H, emit=False, nthreads=threads)
    lap("bin_sort")
    fwd = oracle.forward(proj, bins, p64["rgb"], W, H, nthreads=threads)
    lap("render_fwd")
    _, dimg = oracle.l1(fwd["img"], w.targets[:views], LAMBDA_COLOR)
    lap("l1")
    b = oracle.backward(proj, bins, p64["rgb"], W, H, dimg, nthreads=threads)
    lap("render_bwd")
    g = oracle.project_bwd(p64, cam, b, nthreads=threads)
    lap("project_bwd")
    _, greg = oracle.planar_reg(p64["log_scale"], LAMBDA_REG, REG_FLOOR)
    g["log_scale"] = g["log_scale"] + greg
    for k, lr in zip(("mean", "log_scale", "quat", "opacity_logit", "rgb"), LR):
        z = np.zeros_like(p64[k])
        oracle.adam(p64[k], g[k], z, z, lr, 1)
    lap("planar_reg_adam")
    dt = time.perf_counter() - t0
    return {"value": views / (dt * V), "unit": "iterations/s",
            "cores": threads, "kind": "oracle",
            "sample": (f"{views} of {V} views, every stage of the iteration, "
                       f"FP64, {threads} threads, {dt:.2f} s"
                       + (f"; scaled x{V / views:g}" if views != V else "")),
            "host": host_cpus(), "stages_s": st}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="window",
                    choices=["window", "window640", "single", "small"])
    ap.add_argument("--tile", type=int, default=0,
                    help="fix the launch shape (default: autotune)")
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--full-box", action="store_true",
                    help="render whole integer boxes (no render-box cut)")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of MIB MiB (a "
                         "known-size reference for HBM traffic counters)")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-others", action="store_true",
                    help="skip the other configurations and the insertion run")
    ap.add_argument("--no-densify", action="store_true",
                    help="skip the per-keyframe densification timing")
    ap.add_argument("--no-ssim", action="store_true",
                    help="skip the full colour loss (L1 + SSIM) timing")
    ap.add_argument("--sh-degree", type=int, default=0, choices=[0, 1, 2, 3],
                    help="give the workload view-dependent colour of this "
                         "degree (coefficients N(0, 0.05))")
    ap.add_argument("--no-per-view", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU "
              "path (the window would shard by views with one gradient "
              "all-reduce). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2504_02437_amd import autotune as AT
    from paper_2504_02437_amd import raster as R

    dev = "cuda"
    if args.calib_copy:
        n = args.calib_copy << 18                  # float32 elements
        src = torch.ones(n, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 2.0, out=dst)   # elementwise: reads and writes 4n B
        torch.cuda.synchronize()
        log(f"bench: calibration copy of {4 * n} bytes")
        del src, dst
    log("bench: building workload", args.workload)
    w = workload(args.workload)
    if args.sh_degree:
        import synth
        w.gaussians = synth.with_sh(w.gaussians, 0, args.sh_degree, 0.05)
    V = len(w.cameras)
    W, H = w.cameras[0].width, w.cameras[0].height
    N = w.gaussians.n
    params = R.ParamBuffer.from_gaussians(w.gaussians, device=dev)
    if args.tile:
        S = R.Settings(tile=args.tile, lds_batch=args.batch,
                       block_threads=args.threads, full_box=args.full_box)
        tuned = None
    else:
        S, times = AT.autotune(params, w.cameras,
                               R.Settings(full_box=args.full_box), reps=2,
                               use_cache=False, cache_path=None, log=log)
        tuned = {f"{t}/{b}/{n}": round(ms, 3) for (t, b, n), ms in
                 sorted(times.items(), key=lambda kv: kv[1])}
    log("bench: launch shape tile", S.tile, "batch", S.lds_batch, "threads",
        S.block_threads)
    grad = params.zeros_like()
    m = params.zeros_like()
    v = params.zeros_like()
    rast = R.Rasterizer(w.cameras, params.capacity, S, device=dev)
    rast.fit_key_capacity(params)
    ws, cams_dev = rast.ws, rast.cams_dev
    rgb, T, nlast = rast.rgb, rast.T, rast.nlast
    target = torch.from_numpy(w.targets).to(dev)
    dL = torch.empty_like(rgb)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    step_dev = torch.ones(1, dtype=torch.int32, device=dev)
    names = ("project_and_bin", "sort_tile_keys", "render_fwd", "planar_reg",
             "render_bwd", "project_bwd", "adam", "loss_ssim")
    scratch = R.ssim_scratch(rgb)
    ev = {k: [] for k in names}

    # Events are created up front, so the timed loop only records them.
    pool = [torch.cuda.Event(enable_timing=True)
            for _ in range(2 * len(names) * (args.steps + 5))]

    def timed(name, fn, on):
        if not on:
            fn()
            return
        a, b = (pool.pop() for _ in range(2)) if len(pool) >= 2 else (
            torch.cuda.Event(enable_timing=True) for _ in range(2))
        a.record()
        fn()
        b.record()
        ev[name].append((a, b))

    def step(on=False, ssim=False):
        grad.data.zero_()
        loss.zero_()
        timed("project_and_bin",
              lambda: R.project_and_bin(ws, params, cams_dev, S), on)
        timed("sort_tile_keys", lambda: R.sort_tile_keys(ws, S), on)
        timed("render_fwd",
              lambda: R.render_fwd(ws, params, S, rgb, T, nlast), on)
        if ssim:
            timed("loss_ssim",
                  lambda: R.loss_colour(rgb, target,
                                        LAMBDA_COLOR * (1 - LAMBDA_PHOTO),
                                        LAMBDA_COLOR * LAMBDA_PHOTO, dL, loss,
                                        scratch=scratch), on)
        timed("planar_reg",
              lambda: R.planar_reg(params, LAMBDA_REG, REG_FLOOR, grad, loss), on)
        if ssim:
            R.render_bwd_pixels(ws, params, S, dL, T, nlast, grad)
        else:
            # The L1 term is fused into the compositing backward.
            timed("render_bwd",
                  lambda: R.render_bwd_l1(ws, params, S, rgb, target,
                                          LAMBDA_COLOR, T, nlast, grad, loss),
                  on)
        timed("project_bwd",
              lambda: R.project_bwd(ws, params, cams_dev, grad), on)
        timed("adam", lambda: R.adam(params, grad, m, v, LR, 0.9, 0.999, 1e-15,
                                     step_dev), on)
        step_dev.add_(1)

    def run(k, on):
        a, b = (torch.cuda.Event(enable_timing=True) for _ in range(2))
        a.record()
        for i in range(k):
            step(on)
            if k >= 4 and (i + 1) % max(1, k // 4) == 0:
                log(f"bench: eager step {i + 1}/{k}")
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / k

    log("bench: warmup", args.warmup)
    run(args.warmup, False)
    # Every iteration is a real optimiser step, so the map drifts as the
    # bench runs (and with it the pair counts).  Each measured phase below
    # starts from this post-warm-up state, restored in place (graph-safe).
    torch.cuda.synchronize()
    snap = [t.clone() for t in (params.data, m.data, v.data, step_dev)]

    def restore():
        for dst, src in zip((params.data, m.data, v.data, step_dev), snap):
            dst.copy_(src)
        torch.cuda.synchronize()

    flags, n_keys = rast.status()
    if flags:
        raise SystemExit(f"device status {flags}: key capacity exceeded")
    counts0 = rast.count_pairs(params)
    log("bench: keys", n_keys, "counts", counts0)
    t0 = time.perf_counter()
    ms_eager = run(args.steps, True)
    wall = time.perf_counter() - t0
    counts1 = rast.count_pairs(params)
    kern = {k: float(np.mean([a.elapsed_time(b) for a, b in ev[k]]))
            for k in names if ev[k]}
    # Medians beside the means: a host-side stall inside a kernel's event
    # pair (the stream waits for the launch) shows as a mean above the
    # median.
    kern_p50 = {k: float(np.median([a.elapsed_time(b) for a, b in ev[k]]))
                for k in names if ev[k]}

    ms_graph = None
    dist = None
    if not args.no_graph:
        # The library captures the iteration (gs_window_build) and replays
        # it (gs_window_run) on a stream of its own.
        log("bench: capturing one iteration in a HIP graph (gs_window_build)")
        gstream = torch.cuda.Stream()
        gstream.wait_stream(torch.cuda.current_stream())
        win = R.WindowGraph(rast, params, grad, target, loss,
                            lam_l1=LAMBDA_COLOR, lam_reg=LAMBDA_REG,
                            reg_floor=REG_FLOOR, m=m, v=v, lr=LR, beta1=0.9,
                            beta2=0.999, eps=1e-15, step=step_dev,
                            stream=gstream)
        for _ in range(args.warmup):
            win.run(gstream)
        restore()
        a, b = (torch.cuda.Event(enable_timing=True) for _ in range(2))
        gstream.synchronize()
        a.record(gstream)
        for i in range(args.steps):
            win.run(gstream)
        b.record(gstream)
        torch.cuda.synchronize()
        ms_graph = a.elapsed_time(b) / args.steps
        log(f"bench: graph {ms_graph:.3f} ms/iteration, eager {ms_eager:.3f}")
        # Spread of single replays, each between two events (after the timed
        # region; not part of `value`).
        restore()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(51)]
        evs[0].record(gstream)
        for i in range(50):
            win.run(gstream)
            evs[i + 1].record(gstream)
        torch.cuda.synchronize()
        per = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(50)])
        dist = {"replays": 50,
                **{f"p{q}": float(np.percentile(per, q)) for q in (10, 50, 90)}}
        win.close()

    # The paper's full colour loss (Eq. 10): 0.8 L1 + 0.2 (1 - SSIM), reported
    # beside the headline iteration (which uses the L1 term only).
    full = None
    if not args.no_ssim:
        log("bench: full colour loss (L1 + SSIM)")
        for _ in range(2):
            step(True, ssim=True)
        ev["loss_ssim"].clear()
        restore()
        a, b = (torch.cuda.Event(enable_timing=True) for _ in range(2))
        k = max(3, args.steps // 2)
        a.record()
        for _ in range(k):
            step(True, ssim=True)
        b.record()
        torch.cuda.synchronize()
        ms_full = a.elapsed_time(b) / k
        ssim_ms = float(np.mean([x.elapsed_time(y) for x, y in ev["loss_ssim"]]))
        full = {"iterations_per_s": 1000.0 / ms_full, "ms_per_iteration": ms_full,
                "launch": "eager", "loss_colour_ms": ssim_ms,
                "lambda_photo": LAMBDA_PHOTO}

    per_view = None
    if not args.no_per_view and V > 1:
        log("bench: per-keyframe plain path")
        singles = [R.Rasterizer([c], params.capacity, S, device=dev)
                   for c in w.cameras]
        for r1 in singles:
            r1.fit_key_capacity(params)
        tgt1 = [target[i:i + 1] for i in range(V)]

        def plain_step():
            grad.data.zero_()
            loss.zero_()
            for i, r1 in enumerate(singles):
                r1.forward(params)
                r1.backward_l1(params, tgt1[i], LAMBDA_COLOR, grad, loss)
            R.planar_reg(params, LAMBDA_REG, REG_FLOOR, grad, loss)
            R.adam(params, grad, m, v, LR, 0.9, 0.999, 1e-15, step_dev)
            step_dev.add_(1)

        for _ in range(2):
            plain_step()
        restore()
        a, b = (torch.cuda.Event(enable_timing=True) for _ in range(2))
        k = max(3, args.steps // 2)
        a.record()
        for _ in range(k):
            plain_step()
        b.record()
        torch.cuda.synchronize()
        ms_plain = a.elapsed_time(b) / k
        per_view = {"iterations_per_s": 1000.0 / ms_plain,
                    "ms_per_iteration": ms_plain,
                    "batched_speedup": ms_plain / (ms_graph or ms_eager)}
        del singles

    # Per-keyframe steps on view 0, on a copy of the scene with room to grow:
    # clarity-enhancing densification (Eq. 8-9: dominant-Gaussian render,
    # histogram and split) and keyframe insertion.
    dens = None
    if not args.no_densify:
        log("bench: densification of one keyframe")
        pd = R.ParamBuffer.from_gaussians(w.gaussians, capacity=N + N // 2,
                                          device=dev)
        saved = pd.data.clone()
        n0 = pd.n()
        r1 = R.Rasterizer([w.cameras[0]], pd.capacity, S, device=dev)
        r1.fit_key_capacity(pd)
        gen = torch.Generator(device=dev)
        gen.manual_seed(0)
        xi = torch.randn(pd.capacity, 2, 3, device=dev, generator=gen)
        dscr = R.densify_scratch(pd.capacity, dev)
        nsplit = torch.zeros(1, dtype=torch.int32, device=dev)
        times_r, times_d = [], []
        for rep in range(6):
            pd.data.copy_(saved)
            pd.n_dev.fill_(n0)
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record()
            dom = r1.forward_dominant(pd)
            e1.record()
            R.densify(pd, None, None, dom, DENSIFY_SIGMA, xi, scratch=dscr,
                      n_split=nsplit)
            e2.record()
            torch.cuda.synchronize()
            if rep:
                times_r.append(e0.elapsed_time(e1))
                times_d.append(e1.elapsed_time(e2))
        dens = {"view": "1200x680, 300k Gaussians", "sigma": DENSIFY_SIGMA,
                "split": int(nsplit), "dominant_render_ms": float(np.mean(times_r)),
                "densify_ms": float(np.mean(times_d))}
        # Keyframe insertion, 96 patches x 9 candidates, against the 300k map:
        # the accumulated-alpha mask and the paper's distance test (Eq. 7).
        rng = np.random.default_rng(0)
        pts = torch.from_numpy(np.stack(
            [rng.integers(1, W - 1, 96), rng.integers(1, H - 1, 96),
             1.0 / rng.uniform(1, 5, 96)], 1).astype(np.float32)).to(dev)
        cam0 = r1.cams_dev
        kf_rgb = target[0].contiguous()
        kf_T = r1.T[0].contiguous()
        ins_scr = torch.empty(96 * 9, dtype=torch.int64, device=dev)
        t_a, t_d = [], []
        for rep in range(6):
            for mode, acc in (("alpha", t_a), ("distance", t_d)):
                pd.data.copy_(saved)
                pd.n_dev.fill_(n0)
                e0, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
                e0.record()
                if mode == "alpha":
                    R.insert_gaussians(pd, None, None, cam0, W, H, kf_rgb, kf_T,
                                       pts)
                else:
                    R.insert_distance(pd, None, None, cam0, W, H, kf_rgb, pts,
                                      INSERT_TAU, scratch=ins_scr)
                e1.record()
                torch.cuda.synchronize()
                if rep:
                    acc.append(e0.elapsed_time(e1))
        dens["insert_alpha_ms"] = float(np.mean(t_a))
        dens["insert_distance_ms"] = float(np.mean(t_d))
        dens["insert_tau"] = INSERT_TAU
        # Learned initialisation of the same candidates: kNN features, the
        # network's forward pass (random weights: the cost does not depend on
        # them) and the accumulated-alpha insertion taking its outputs.
        C = 96 * 9
        feats = torch.empty(C, 32, dtype=torch.float32, device=dev)
        mlp_y = torch.empty(C, 7, dtype=torch.float32, device=dev)
        from paper_2504_02437_amd.init_mlp import N_PARAMS
        wts = (torch.randn(N_PARAMS, generator=torch.Generator().manual_seed(5))
               * 0.1).to(dev)
        t_k, t_l = [], []
        for rep in range(6):
            pd.data.copy_(saved)
            pd.n_dev.fill_(n0)
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record()
            R.knn_features(pd, cam0, W, H, kf_rgb, pts, False, feats)
            e1.record()
            R.mlp_fwd(wts, feats, mlp_y)
            R.insert_gaussians(pd, None, None, cam0, W, H, kf_rgb, kf_T, pts,
                               mlp_out=mlp_y)
            e2.record()
            torch.cuda.synchronize()
            if rep:
                t_k.append(e0.elapsed_time(e1))
                t_l.append(e0.elapsed_time(e2))
        dens["knn_features_ms"] = float(np.mean(t_k))
        dens["insert_learned_ms"] = float(np.mean(t_l))
        del r1, pd, saved, dscr

    # The other configurations at the same launch shape.
    others = None
    if not args.no_others:
        others = {}
        for name in ("window640", "single", "small"):
            wo = workload(name)
            log("bench: workload", name)
            po = R.ParamBuffer.from_gaussians(wo.gaussians, device=dev)
            So, _ = AT.autotune(po, wo.cameras, R.Settings(), reps=2,
                                use_cache=False, cache_path=None)
            del po
            ms_o = iteration_ms(wo, So)
            Vo = len(wo.cameras)
            Wo, Ho = wo.cameras[0].width, wo.cameras[0].height
            others[wo.name] = {"ms_per_iteration": ms_o,
                               "iterations_per_s": 1000.0 / ms_o,
                               "mpix_per_s": Vo * Wo * Ho * 1e-3 / ms_o,
                               "launch": "eager",
                               "shape": f"{So.tile}/{So.lds_batch}/{So.block_threads}"}
        # View-dependent colour of degree 3 (45 coefficient rows) on the
        # headline workload and launch shape.
        log("bench: degree-3 view-dependent colour")
        import synth
        wsh = workload(args.workload)
        wsh.gaussians = synth.with_sh(wsh.gaussians, 0, 3, 0.05)
        ms_sh = iteration_ms(wsh, S)
        others[wsh.name + "-sh3"] = {
            "ms_per_iteration": ms_sh, "iterations_per_s": 1000.0 / ms_sh,
            "launch": "eager", "shape": f"{S.tile}/{S.lds_batch}/{S.block_threads}",
            "degree0_eager_ms": ms_eager}
        del wsh
        log("bench: insertion growth run")
        others["insertion-200kf-1200x680"] = insertion_stress(S)

    cnt = {k: 0.5 * (counts0[k] + counts1[k]) for k in counts0}
    # Pairs under whole integer boxes (the paper's evaluation rule), for
    # comparison with the pairs the render boxes leave to examine.
    cnt_full = cnt
    if not S.full_box:
        rf = R.Rasterizer(w.cameras, params.capacity,
                          dataclasses.replace(S, full_box=True), device=dev)
        rf.fit_key_capacity(params)
        rf.forward(params)
        cnt_full = rf.count_pairs(params)
        del rf
    fwd_ops, bwd_ops = credited_ops(cnt)
    if kern["render_bwd"] >= kern["render_fwd"]:
        dom, ops, t = "render_bwd", bwd_ops, kern["render_bwd"]
    else:
        dom, ops, t = "render_fwd", fwd_ops, kern["render_fwd"]
    achieved = ops / (t * 1e-3) / 1e12
    peak = PEAK_LANE_OPS / 1e12
    meas = measured_counters(
        f"k_render_{dom[7:]}<{S.tile}, {S.lds_batch}, "
        f"{S.block_threads or (256 if S.tile == 32 else 64)}")
    ms = ms_graph if ms_graph is not None else ms_eager
    iters = 1000.0 / ms
    out = {
        "metric": METRIC,
        "value": iters,
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "views": V, "width": W, "height": H,
                   "gaussians": N, "tile": S.tile, "lds_batch": S.lds_batch,
                   "block_threads": S.block_threads or (256 if S.tile == 32 else 64),
                   "launch": "hip_graph" if ms_graph is not None else "eager",
                   "adam_in_step": True, "render_box": not S.full_box,
                   "sh_degree": args.sh_degree},
        "mpix_per_s": V * W * H * iters / 1e6,
        "ms_per_step_eager": ms_eager,
        "ms_per_replay": dist,
        "keys_per_iter": int(n_keys),
        "kernels_ms": kern,
        "kernels_ms_p50": kern_p50,
        "pairs": cnt,
        "pairs_full_box": cnt_full,
        "roofline": {"bound": "alu", "kernel": dom, "achieved": achieved,
                     "peak": peak, "unit": "Tlane-op/s",
                     "frac": achieved / peak,
                     "traffic": meas["traffic"],
                     "valu_issue": meas["valu_issue"],
                     "fp32_tflops": meas["fp32_tflops"],
                     "ops_per_launch": ops,
                     "render_fwd_frac": fwd_ops / (kern["render_fwd"] * 1e-3) / PEAK_LANE_OPS,
                     "render_bwd_frac": bwd_ops / (kern["render_bwd"] * 1e-3) / PEAK_LANE_OPS},
        "per_keyframe_plain": per_view,
        "full_colour_loss": full,
        "densification": dens,
        "other_workloads": others,
        "autotune_ms": tuned,
        "wall_s": wall,
    }
    if not args.no_cpu_baseline:
        threads = args.cpu_threads or cpu_threads(host_cpus())
        log("bench: CPU oracle baseline on", threads, "threads")
        out["cpu_baseline"] = cpu_baseline(w, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
