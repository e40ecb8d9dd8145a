#!/usr/bin/env python3
"""Tracking throughput of the CG-SLAM rasterizer hot path on one MI355X.

Workload (the paper's tracking loop, Sec. 3.4 Eq. 19-20, on a synthetic indoor
room standing in for the paper's RGB-D datasets): 100k Gaussians on the walls of
a 5 x 4 x 3 m room, a 640x480 camera (f = 525), target colour and depth
rendered at the true pose, the solve starting from a perturbed pose.  One step
is one tracking iteration: render (projection, tile sort, blend) -> tracking
loss gradient images -> pose-only backward -> Adam step and retraction.  Solves
of 50 iterations are captured into one HIP graph and replayed; the timed region
is K iterations with all inputs resident in HBM.

Prints one JSON line.  Only N = 1 GPU is supported.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "tracking iters/s (fwd+pose-bwd) 640x480 100k Gaussians; % of HBM roofline"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector (256 CUs x 2.4 GHz)

# Algorithmic FP32 operations, counted from the equations (a fused
# multiply-add counts 2, exp counts 1):
#   alpha of one (pixel, list entry), Eq. 5: mu - p (2), quadratic form (8),
#   * -1/2 (1), exp (1), * opacity (1)                                   = 13
#   blending one Gaussian, Eq. 3, 4, 6, 9 (tracking needs no Eq. 10):
#   1 - alpha, T (1 - alpha), w = alpha T (3), colour (6), depth (2),
#   opacity (1)                                                          = 12
#   backward of one blended Gaussian with colour and depth gradients:
#   T_j (2), w (1), dL/dalpha over the 4 blended quantities (9), behind
#   sums (12), dL/dpower (1), dL/dmu (8), dL/dconic (9), dL/ddepth (2)   = 44
# The forward evaluates alpha for every entry up to where it stops; the
# backward re-evaluates it for every entry up to the last blended one.
FLOP_EVAL = 13
FLOP_BLEND = 12
FLOP_BLEND_BWD = 44


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_workload(torch, R, synth, n=100_000, seed=0):
    sc = synth.room_scene(seed, n, (5.0, 4.0, 3.0))
    scd = {k: torch.from_numpy(v).cuda() for k, v in sc.items()}
    cam = synth.TRACKING_CAMERA
    Rt, tt = synth.level_room_pose(seed)
    st = R.State()
    tgt = R.render(st, scd, R.pose_tensor(Rt, tt), [cam])[0]
    torch.cuda.synchronize()
    prob = R.TrackingProblem(scd, cam, tgt["color"].clone(), tgt["depth"].clone())
    P0 = R.pose_tensor(*synth.perturb_pose(Rt, tt, seed + 1000))
    return sc, prob, P0, (Rt, tt)


def algorithmic_bytes(n, visible, pairs, pixels):
    """HBM bytes one tracking iteration must move: parameters read (56 B per
    Gaussian), projected records written (40 B per visible one), pairs written
    and read back after the sort (24 B) and record gathers per pair (40 B),
    per-pixel sensor depth, 28 B of maps and 8 B of saved state (40 B); the
    backward reads gradient images, saved state and depth (32 B per pixel),
    record ids and records per pair (44 B) and writes and re-reads projected
    gradients plus parameters per visible Gaussian (88 B)."""
    fwd = 56 * n + 40 * visible + 24 * pairs + 40 * pairs + 40 * pixels
    bwd = 32 * pixels + 44 * pairs + 88 * visible
    return fwd + bwd


def cpu_baseline(prob_np, cam, pose0, budget_s: float):
    """The FP64 oracle doing tracking iterations on the host cores."""
    import numpy as np

    import oracle
    sc, tc, td = prob_np
    pose = (np.asarray(pose0[0], np.float64), np.asarray(pose0[1], np.float64))
    m = np.zeros(6)
    v = np.zeros(6)
    lr = np.array([0.00215] * 3 + [0.0015] * 3)
    t0 = time.perf_counter()
    it = 0
    while True:
        maps = oracle.render(sc, cam, pose)
        _, dimg = oracle.tracking_loss(maps, tc, td)
        g = oracle.backward(sc, cam, pose, None, dimg)
        xi, m, v = oracle.adam_step(np.zeros(6), g["pose"], m, v, it + 1, lr)
        pose = oracle.retract(pose, xi)
        it += 1
        el = time.perf_counter() - t0
        if el >= budget_s or it >= 50:
            break
    return dict(value=it / el, unit="it/s", cores=oracle.num_threads(), kind="oracle",
                sample=f"{it} full tracking iterations (render + tracking loss + pose backward + Adam) "
                       f"of the same 100k-Gaussian 640x480 workload in {el:.1f} s")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000, help="timed tracking iterations")
    ap.add_argument("--warmup", type=int, default=200, help="untimed tracking iterations")
    ap.add_argument("--solve-iters", type=int, default=50, help="iterations per captured solve")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stage-timing", action="store_true")
    ap.add_argument("--eager", action="store_true",
                    help="run the solves without graph capture (same kernels; for counter collection)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="only run a plain device copy of this many MB, 10 times (profiler byte-counter scale)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(tracking frames shard by frame, mapping views by view; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2403_16095_amd import rasterizer as R
    from paper_2403_16095_amd import synth

    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(10):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 4, "copy_calibration_bytes_written": n * 4}))
        return
    log("building workload: 100k Gaussians, 640x480")
    sc, prob, P0, true_pose = build_workload(torch, R, synth)
    iters = args.solve_iters
    tune_state = R.State()
    fppl, bppl = R.autotune_tracking(tune_state, prob.scene, P0, [prob.cam], [prob.target_color],
                                     [prob.target_depth])
    del tune_state
    log(f"autotuned pixels per lane: forward {fppl}, backward {bppl}")
    solver = R.TrackingSolver(prob, iters=iters, use_graph=not args.eager, reset_pose=P0, fwd_ppl=fppl,
                              bwd_ppl=bppl)
    solver.prepare(P0)
    solves_w = max(1, math.ceil(args.warmup / iters))
    solves = max(1, math.ceil(args.steps / iters))
    steps, warmup = solves * iters, solves_w * iters
    log(f"warmup {warmup} iterations")
    for _ in range(solves_w):
        solver.run()
    torch.cuda.synchronize()
    solver.check()

    log(f"timed {steps} iterations ({solves} graph replays of {iters})")
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(solves):
        solver.run()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    solver.check()
    ms_per_step = wall * 1e3 / steps
    value = steps / wall
    err_t = float((solver.pose.cpu().double()[9:] - torch.as_tensor(true_pose[1])).abs().max())
    log(f"{value:.1f} it/s ({ms_per_step * 1e3:.1f} us/it wall, {gpu_ms * 1e3 / steps:.1f} us/it events); "
        f"final |t - t_true|_inf = {err_t:.2e} m")

    # Per-stage kernel durations, HIP events recorded by the library on the
    # launch stream, over eager iterations of the same workload.
    stages, stats = {}, None
    if not args.no_stage_timing:
        tst = R.State(timing=True, fwd_ppl=fppl, bwd_ppl=bppl)
        tst.reserve(pairs=solver.state.stats().pairs * 2)
        pose = P0.clone().reshape(1, 12)
        acc = {}
        reps = 20
        dpose = torch.zeros((1, 6), device="cuda")
        for r in range(reps + 2):
            R.tracking_step(tst, prob.scene, pose, [prob.cam], [prob.target_color], [prob.target_depth],
                            dposes=dpose)
            t = tst.timings()
            if r >= 2:
                for k, v in t.items():
                    acc[k] = acc.get(k, 0.0) + v / reps
        stages = acc
        s = tst.stats()
        stats = dict(visible=int(s.visible), pairs=int(s.pairs), evaluations=int(s.processed),
                     blended=int(s.blended), walked=int(s.walked))
        log("stage ms:", {k: round(v, 4) for k, v in stages.items()}, "stats:", stats)

    result = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "it/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "tracking: 100k Gaussians on a 5x4x3 m room, 640x480 f=525, "
                               "render + L1 colour/depth loss + pose-only backward + Adam, 50-iteration "
                               "solves replayed from one HIP graph",
                   "gaussians": 100_000, "width": 640, "height": 480, "solve_iters": iters,
                   "pixels_per_lane": {"forward": fppl, "backward": bppl},
                   "loss_lambda": list(R.TRACK_LAMBDA)},
    }
    if stages:
        # The dominant single kernel and its roofline.
        blend_f, blend_b = stages["blend_fwd"], stages["blend_bwd"]
        flops_fwd = FLOP_EVAL * stats["evaluations"] + FLOP_BLEND * stats["blended"]
        flops_bwd = FLOP_EVAL * stats["walked"] + FLOP_BLEND_BWD * stats["blended"]
        cand = {"blend_fwd": (blend_f, flops_fwd), "blend_bwd": (blend_b, flops_bwd)}
        name = max(cand, key=lambda k: cand[k][0])
        ms, fl = cand[name]
        achieved = fl / (ms * 1e-3) / 1e12
        result["roofline"] = {"bound": "alu", "kernel": name, "achieved": round(achieved, 4),
                              "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                              "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 5), "traffic": None,
                              "avg_ms": round(ms, 5), "algorithmic_flops": fl}
        b = algorithmic_bytes(100_000, stats["visible"], stats["pairs"], 640 * 480)
        result["hbm_roofline"] = {"algorithmic_bytes_per_iter": b,
                                  "achieved_GBs": round(b / (ms_per_step * 1e-3) / 1e9, 2),
                                  "peak_GBs": HBM_PEAK_GBS,
                                  "frac": round(b / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 5)}
        result["stages_ms"] = {k: round(v, 5) for k, v in stages.items()}
        result["stats"] = stats
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        tc = prob.target_color.cpu().numpy()
        td = prob.target_depth.cpu().numpy()
        p0 = P0.cpu().double().numpy()
        result["cpu_baseline"] = cpu_baseline((sc, tc, td), prob.cam, (p0[:9].reshape(3, 3), p0[9:]),
                                              args.cpu_budget)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
