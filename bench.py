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

``--workload`` selects one of the other measured workloads instead (each
prints its own JSON line, timed eagerly with inputs resident in HBM):

* ``mapping``: 500k Gaussians in an 8 x 6 x 3 m room, one 1200x680 view
  (f = 600); render with sensor depth, uncertainty-weighted L1 loss gradient
  images, backward to every Gaussian parameter and the pose.
* ``batched-mapping``: 1M Gaussians, 8 keyframe views of 1200x680 along a
  random walk; the same iteration for all 8 views in one launch sequence
  (per-Gaussian gradients summed over views) against 8 single-view sequences.
* ``batched-tracking``: 1M Gaussians, 32 frames of uneven resolution; a
  20-iteration Adam tracking loop over all frames at once captured in one HIP
  graph, against 32 single-frame graphs of the same loop.
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
# The mapping iteration blends six quantities (colour, alpha-depth, opacity,
# uncertainty with sensor depth, Eq. 3-10) and takes every gradient:
#   forward per blended Gaussian: the 12 above + w (d - D)^2 (3) + the
#   median test (1)                                                      = 16
#   backward per blended Gaussian: T_j (2), w (1), dL/dalpha over the six
#   quantities (15), behind sums (18), dL/dpower and dL/dopacity (2),
#   dL/dmu (8), dL/dconic (9), dL/ddepth with the uncertainty term (6),
#   dL/dcolour (3), opacity sum (1)                                      = 65
FLOP_BLEND_MAP = 16
FLOP_BLEND_BWD_MAP = 65
FP32_REACHABLE_TFLOPS = 78.6     # without packed FP32 (this build disables it)
VALU_CYCLES = 4                  # a wave64 VALU instruction on a 16-lane SIMD
SIMDS = 1024                     # 256 CUs x 4 SIMDs
CLOCK_HZ = 2.4e9


def alu_roofline(kernel, symbol, flops, ms, timing, counters=None):
    """ALU roofline of one kernel: algorithmic flops per launch over its
    measured launch duration, against the published FP32 vector peak and the
    peak reachable without packed FP32; with the committed instruction
    counters of that kernel, the fraction of SIMD cycles issuing VALU."""
    achieved = flops / (ms * 1e-3) / 1e12
    out = {"bound": "alu", "kernel": kernel, "symbol": symbol, "achieved": round(achieved, 4),
           "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 5),
           "peak_reachable": FP32_REACHABLE_TFLOPS, "frac_reachable": round(achieved / FP32_REACHABLE_TFLOPS, 5),
           "traffic": None, "avg_ms": round(ms, 5), "timing": timing, "algorithmic_flops": int(flops)}
    if counters:
        out["traffic"] = counters.get("bytes_per_launch")
        if counters.get("valu_insts"):
            out["valu_insts"] = counters["valu_insts"]
            out["valu_issue_frac"] = round(counters["valu_insts"] * VALU_CYCLES / (SIMDS * CLOCK_HZ * ms * 1e-3), 4)
    return out


def kernel_source_digest() -> str:
    """sha256 over the sources of the blend kernels (raster.hip and the
    headers it includes): the measured traffic stays valid while they do."""
    import hashlib
    d = os.path.join(ROOT, "paper_2403_16095_amd", "csrc")
    h = hashlib.sha256()
    for name in ("common.hpp", "kernels.hpp", "raster.hip"):
        h.update(name.encode())
        with open(os.path.join(d, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_counters(kernel: str):
    """Committed counter profile of `kernel` (profiles/blend_counters.json:
    HBM bytes per launch from FETCH_SIZE and WRITE_SIZE scaled by a copy
    calibration, VALU wave instructions per launch), or None if the kernel
    sources changed since it was taken.  The figures are per launch of the
    workload they were taken on (the fused blend: the 640x480 tracking
    workload; the blend backward: one 1200x680 mapping view), so callers ask
    only for those."""
    path = os.path.join(ROOT, "profiles", "blend_counters.json")
    try:
        with open(path) as f:
            prof = json.load(f)
    except (OSError, ValueError):
        return None
    if prof.get("source_sha256") != kernel_source_digest():
        return None
    return prof.get("kernels", {}).get(kernel)


def copy_bandwidth(torch, mb=1024, reps=10):
    """Achieved HBM bandwidth of a plain device copy (read + write bytes / s)."""
    n = mb * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * n * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del x, y
    return gbs


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def with_sh(synth, sc, seed, degree):
    """The scene with view-dependent colour of the given degree instead of rgb
    (degree 0 keeps rgb)."""
    if degree <= 0:
        return sc
    out = {k: v for k, v in sc.items() if k != "rgb"}
    out["sh"] = synth.sh_coefficients(seed, sc["means"].shape[0], degree)
    return out


def param_floats(degree):
    """float32 parameters per Gaussian: 11 + 3 for rgb, 11 + 3 (degree + 1)^2 with SH."""
    return 14 if degree <= 0 else 11 + 3 * (degree + 1) ** 2


def build_workload(torch, R, synth, n=100_000, seed=0, sh_degree=0):
    sc = with_sh(synth, synth.room_scene(seed, n, (5.0, 4.0, 3.0)), seed + 7, sh_degree)
    scd = {k: torch.from_numpy(v).cuda() for k, v in sc.items()}
    cam = synth.TRACKING_CAMERA
    Rt, tt = synth.level_room_pose(seed)
    st = R.State()
    tgt = R.render(st, scd, R.pose_tensor(Rt, tt), [cam])[0]
    torch.cuda.synchronize()
    prob = R.TrackingProblem(scd, cam, tgt["color"].clone(), tgt["depth"].clone())
    P0 = R.pose_tensor(*synth.perturb_pose(Rt, tt, seed + 1000))
    return sc, prob, P0, (Rt, tt)


def algorithmic_bytes(n, visible, pairs, pixels, sh_degree=0):
    """HBM bytes one tracking iteration must move: parameters read (56 B per
    Gaussian with rgb, 4 (11 + 3 K) B with K SH coefficients per channel; read
    again by the backward for the visible ones), projected records written (40 B per visible one), pairs written
    and read back after the sort (24 B) and record gathers per pair (40 B),
    per-pixel sensor depth, 28 B of maps and 8 B of saved state (40 B); the
    backward reads gradient images, saved state and depth (32 B per pixel),
    record ids and records per pair (44 B) and writes and re-reads projected
    gradients plus parameters per visible Gaussian (88 B)."""
    pb = 4 * param_floats(sh_degree)
    fwd = pb * n + 40 * visible + 24 * pairs + 40 * pairs + 40 * pixels
    bwd = 32 * pixels + 44 * pairs + 88 * visible + (pb - 56) * visible
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

# --------------------------------------------------------------------------
# Mapping and batched workloads

PARAM_WIDTHS = (("means", 3), ("log_scales", 3), ("quats", 4), ("opacity_logits", 1), ("rgb", 3))


def _sync_timed(torch, fn, reps):
    """Run fn() reps times between device synchronisations; returns (wall s,
    event ms) of the whole run."""
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, e0.elapsed_time(e1)


class MappingIteration:
    """Render (colour, depth, uncertainty with sensor depth) -> uncertainty-
    weighted L1 gradient images -> backward to every Gaussian parameter and
    each view's pose, on preallocated buffers; gradients are cleared once per
    iteration and summed over the views by the library."""

    def __init__(self, torch, R, scene, poses, cams, target_colors, target_depths, batched: bool, ppl=(1, 1)):
        B = R.B
        self.torch, self.R, self.B = torch, R, B
        self.batched = batched
        self.V = len(cams)
        n = scene["means"].shape[0]
        dev = poses.device
        self.g = R.gaussians_struct(scene)
        self.poses = poses
        self.cams = [R.camera_struct(c) for c in cams]
        self.tc, self.td = target_colors, target_depths
        sh = scene.get("sh")
        widths = [(k, w) for k, w in PARAM_WIDTHS if not (k == "rgb" and sh is not None)]
        if sh is not None:
            widths.append(("sh", sh.shape[1] * 3))
        self.flat = torch.zeros(n * sum(w for _, w in widths), dtype=torch.float32, device=dev)
        off, views = 0, {}
        for name, w in widths:
            views[name] = self.flat[off:off + n * w].data_ptr()
            off += n * w
        self.dG = B.cgsr_gaussian_grads(views["means"], views["log_scales"], views["quats"], views["opacity_logits"],
                                        views.get("rgb"), views.get("sh"))
        self.dposes = torch.zeros((self.V, 6), dtype=torch.float32, device=dev)
        self.maps, self.grads, self.out_s, self.grad_s = [], [], [], []
        for c in cams:
            H, W = int(c["height"]), int(c["width"])
            m = dict(color=torch.empty((3, H, W), device=dev), depth=torch.empty((H, W), device=dev),
                     uncertainty=torch.empty((H, W), device=dev))
            d = dict(color=torch.empty((3, H, W), device=dev), depth=torch.empty((H, W), device=dev),
                     uncertainty=torch.empty((H, W), device=dev))
            self.maps.append(m)
            self.grads.append(d)
            self.out_s.append(B.cgsr_images(m["color"].data_ptr(), m["depth"].data_ptr(), None, None,
                                            m["uncertainty"].data_ptr()))
            self.grad_s.append(B.cgsr_images(d["color"].data_ptr(), d["depth"].data_ptr(), None, None,
                                             d["uncertainty"].data_ptr()))
        # the iteration reads no work counts (only pair peaks)
        self.ppl = ppl
        self.states = [R.State(sync_capacity=True, count_work=False, fwd_ppl=ppl[0], bwd_ppl=ppl[1])
                       for _ in range(1 if batched else self.V)]

    def _views(self, st, vs):
        B, s = self.B, self.R._stream()
        B.cgsr_render(st.handle, self.g, len(vs), self.poses[vs[0]].data_ptr(), [self.cams[v] for v in vs],
                      [self.td[v].data_ptr() for v in vs], [self.out_s[v] for v in vs], s)
        for v in vs:
            m, d, c = self.maps[v], self.grads[v], self.cams[v]
            B.cgsr_mapping_loss_grad(c.width, c.height, m["color"].data_ptr(), m["depth"].data_ptr(),
                                     m["uncertainty"].data_ptr(), self.tc[v].data_ptr(), self.td[v].data_ptr(),
                                     d["color"].data_ptr(), d["depth"].data_ptr(), d["uncertainty"].data_ptr(),
                                     None, s)
        B.cgsr_backward(st.handle, [self.grad_s[v] for v in vs], self.dG, self.dposes[vs[0]].data_ptr(), s)

    def __call__(self):
        self.flat.zero_()
        self.dposes.zero_()
        if self.batched:
            self._views(self.states[0], list(range(self.V)))
        else:
            for v in range(self.V):
                self._views(self.states[v], [v])

    def autotune(self, repeats=5):
        """The library's render autotuner on this iteration's first state and
        views (after a sizing call, so the gradient images hold real
        gradients); the states made by freeze_capacity then use its pick."""
        B = self.B
        vs = list(range(self.V)) if self.batched else [0]
        out = B.cgsr_autotune_render(self.states[0].handle, self.g, len(vs), self.poses[vs[0]].data_ptr(),
                                     [self.cams[v] for v in vs], [self.td[v].data_ptr() for v in vs],
                                     [self.out_s[v] for v in vs], [self.grad_s[v] for v in vs], self.dG,
                                     self.dposes[vs[0]].data_ptr(), repeats, self.R._stream())
        self.ppl = (int(out.fwd_pixels_per_lane), int(out.bwd_pixels_per_lane))
        self.flat.zero_()
        self.dposes.zero_()
        return self.ppl

    def stage_times(self, reps=5):
        """Stage durations (ms) of the batched form of the iteration, from
        the library's HIP events around each stage, on a timing-enabled state
        with the timed state's pair capacity (eager iterations)."""
        cap = int(self.states[0].stats().pair_capacity)
        tst = self.R.State(sync_capacity=False, timing=True, count_work=False, fwd_ppl=self.ppl[0], bwd_ppl=self.ppl[1])
        tst.reserve(tile_pairs=cap)
        acc = {}
        for r in range(reps + 1):
            self.flat.zero_()
            self.dposes.zero_()
            self._views(tst, list(range(self.V)))
            t = tst.timings()
            if r:
                for k, v in t.items():
                    acc[k] = acc.get(k, 0.0) + v / reps
        tst.check()
        tst.close()
        return acc

    def freeze_capacity(self, margin=1.25):
        """After a sizing call: fixed pair capacity, no per-call readback."""
        for k, st in enumerate(self.states):
            peak = st.stats().peak_pairs
            new = self.R.State(sync_capacity=False, count_work=False, fwd_ppl=self.ppl[0], bwd_ppl=self.ppl[1])
            new.reserve(tile_pairs=int(peak * margin) + 64)
            self.states[k] = new
            st.close()

    def check(self):
        for st in self.states:
            st.check()

    def stats(self):
        tot = dict(visible=0, pairs=0, evaluations=0, blended=0, walked=0)
        for st in self.states:
            s = st.stats()
            for k, a in (("visible", "visible"), ("pairs", "pairs"), ("evaluations", "processed"),
                         ("blended", "blended"), ("walked", "walked")):
                tot[k] += int(getattr(s, a))
        return tot


def mapping_bytes(n, visible, pairs, pixels, sh_degree=0):
    """HBM bytes one mapping iteration must move: the tracking figures plus,
    per pixel, the uncertainty map and its gradient (8 B) and the loss
    gradient pass (read 3 maps + 4 targets, write 3 gradients: 40 B), and per
    visible Gaussian its parameter gradients written (56 B with rgb)."""
    return (algorithmic_bytes(n, visible, pairs, pixels, sh_degree) + 48 * pixels
            + 4 * param_floats(sh_degree) * visible)


def oracle_mapping_seconds(sc, cam, pose, tc, td):
    import oracle
    t0 = time.perf_counter()
    maps = oracle.render(sc, cam, pose, td)
    _, dimg = oracle.uncertainty_weighted_loss(maps, tc, td)
    oracle.backward(sc, cam, pose, td, dimg)
    return time.perf_counter() - t0


def oracle_tracking_seconds(sc, cam, pose, tc, td):
    import oracle
    t0 = time.perf_counter()
    maps = oracle.render(sc, cam, pose)
    _, dimg = oracle.tracking_loss(maps, tc, td)
    oracle.backward(sc, cam, pose, None, dimg)
    return time.perf_counter() - t0


def perturbed_scene(np, sc, seed):
    """The scene being optimised: the target scene with means moved by
    N(0, 5 mm) and colours by N(0, 0.05)."""
    rng = np.random.default_rng(seed)
    out = dict(sc)
    out["means"] = (sc["means"] + rng.normal(0.0, 0.005, sc["means"].shape)).astype(np.float32)
    if "sh" in sc:
        out["sh"] = (sc["sh"] + rng.normal(0.0, 0.2, sc["sh"].shape)).astype(np.float32)
    else:
        out["rgb"] = np.clip(sc["rgb"] + rng.normal(0.0, 0.05, sc["rgb"].shape), 0, 1).astype(np.float32)
    return out


def run_mapping(args, torch, R, synth, views: int):
    import numpy as np
    n = 500_000 if views == 1 else 1_000_000
    seed = 3 if views == 1 else 4
    log(f"building workload: {n} Gaussians, {views} view(s) of 1200x680")
    deg = args.sh_degree
    sc_t = with_sh(synth, synth.room_scene(seed, n, (8.0, 6.0, 3.0)), seed + 7, deg)
    sc = perturbed_scene(np, sc_t, seed + 1000)
    cam = synth.MAPPING_CAMERA
    pose_list = [synth.level_room_pose(seed)] if views == 1 else synth.random_walk_poses(seed + 1000, views)
    P = torch.stack([R.pose_tensor(*p) for p in pose_list]).contiguous()
    cams = [cam] * views
    tst = R.State()
    tgt = R.render(tst, {k: torch.from_numpy(v).cuda() for k, v in sc_t.items()}, P, cams, maps=("color", "depth"))
    tcs = [t["color"].clone() for t in tgt]
    tds = [t["depth"].clone() for t in tgt]
    del tgt, tst
    scd = {k: torch.from_numpy(v).cuda() for k, v in sc.items()}
    modes = [("batched", True)] + ([("sequential", False)] if views > 1 else [])
    ppl = tuple(int(x) for x in args.mapping_ppl.split(",")) if args.mapping_ppl != "auto" else (1, 1)
    res = {}
    for name, batched in modes:
        it = MappingIteration(torch, R, scd, P, cams, tcs, tds, batched, ppl)
        it()
        torch.cuda.synchronize()
        if args.mapping_ppl == "auto":
            tuned = it.autotune()
            log(f"{name}: autotuned pixels per lane (forward, backward): {tuned}")
        it.freeze_capacity()
        for _ in range(args.warmup):
            it()
        wall, ev = _sync_timed(torch, it, args.steps)
        it.check()
        res[name] = dict(ms_per_iter=wall * 1e3 / args.steps, event_ms_per_iter=ev / args.steps, stats=it.stats(),
                         ppl=list(it.ppl))
        log(f"{name}: {res[name]['ms_per_iter']:.3f} ms/iteration ({views} view(s))")
        if batched:
            res[name]["stages"] = it.stage_times()
        del it
    st = res["batched"]["stats"]
    # the timed states keep no work counts: one counting render of the same
    # views gives them (they depend only on the workload)
    cst = R.State()
    R.render(cst, scd, P, cams, tds)
    s = cst.stats()
    st.update(evaluations=int(s.processed), blended=int(s.blended), walked=int(s.walked))
    del cst
    b = mapping_bytes(n, st["visible"], st["pairs"], views * cam["width"] * cam["height"], deg)
    ms = res["batched"]["ms_per_iter"]
    stages = res["batched"]["stages"]
    # the dominant kernel: the blend backward to every parameter
    bwd_flops = FLOP_EVAL * st["walked"] + FLOP_BLEND_BWD_MAP * st["blended"]
    bsym = f"raster_backward_kernel<{res['batched']['ppl'][1]}, true, false, false>"
    # the committed counters are per launch of the single-view workload
    roof = alu_roofline("blend_bwd_map", bsym, bwd_flops, stages["blend_bwd"],
                        "library HIP events around the stage, 5 eager iterations",
                        measured_counters(bsym) if views == 1 else None)
    fwd_flops = FLOP_EVAL * st["evaluations"] + FLOP_BLEND_MAP * st["blended"]
    fwd_tflops = fwd_flops / (stages["blend_fwd"] * 1e-3) / 1e12
    out = {
        "metric": ("mapping iters/s (fwd+full bwd) 1200x680 500k Gaussians" if views == 1 else
                   "batched mapping views/s (fwd+full bwd) 8x1200x680 1M Gaussians")
                  + (f", SH degree {deg}" if deg > 0 else ""),
        "value": round((1 if views == 1 else views) * 1e3 / ms, 3),
        "unit": "it/s" if views == 1 else "views/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": (f"mapping: {n} Gaussians on an 8x6x3 m room, {views} view(s) 1200x680 f=600, "
                                "render with sensor depth + uncertainty-weighted L1 + backward to all "
                                "parameters and poses"), "gaussians": n, "views": views, "sh_degree": deg,
                   "pixels_per_lane": res["batched"]["ppl"], "autotuned": args.mapping_ppl == "auto"},
        "roofline": roof,
        "blend_fwd_roofline": {"achieved": round(fwd_tflops, 4), "unit": "TFLOP/s",
                               "frac": round(fwd_tflops / FP32_VECTOR_PEAK_TFLOPS, 5),
                               "frac_reachable": round(fwd_tflops / FP32_REACHABLE_TFLOPS, 5),
                               "avg_ms": round(stages["blend_fwd"], 5), "algorithmic_flops": int(fwd_flops)},
        "hbm_roofline": {"algorithmic_bytes_per_iter": b, "achieved_GBs": round(b / (ms * 1e-3) / 1e9, 2),
                         "peak_GBs": HBM_PEAK_GBS, "frac": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5)},
        "stages_ms": {k: round(v, 5) for k, v in stages.items()},
        "stats": st,
    }
    if views > 1:
        out["sequential"] = {"ms_per_step": round(res["sequential"]["ms_per_iter"], 5),
                             "pixels_per_lane": res["sequential"]["ppl"],
                             "value": round(views * 1e3 / res["sequential"]["ms_per_iter"], 3),
                             "speedup_batched": round(res["sequential"]["ms_per_iter"] / ms, 3)}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, one view)")
        t = oracle_mapping_seconds(sc, cam, pose_list[0], tcs[0].cpu().numpy(), tds[0].cpu().numpy())
        import oracle
        out["cpu_baseline"] = {"value": round(1.0 / t, 5), "unit": out["unit"],
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": f"one view's full iteration (render + loss + backward) in {t:.1f} s"
                                         + ("" if views == 1 else "; views/s extrapolated from one view")}
    return out


def run_management(args, torch, R, synth):
    """One round of Gaussian management (Sec. 3.3) at mapping sizes: spawning
    from the unobserved pixels of a 1200x680 RGB-D view (opacity of a sparse
    render of the room), clone/split densification of 1M Gaussians, and
    compaction of the 1M together with their Adam moments (10 extra arrays).
    Each call synchronises (it returns the new count), so the figure is wall
    time per call."""
    import numpy as np
    n, seed = 1_000_000, 6
    cam = synth.MAPPING_CAMERA
    log(f"building workload: {n} Gaussians, one 1200x680 RGB-D view")
    full = synth.room_scene(seed, n, (8.0, 6.0, 3.0))
    pose = R.pose_tensor(*synth.level_room_pose(seed))
    st = R.State()
    scd = {k: torch.from_numpy(v).cuda() for k, v in full.items()}
    tgt = R.render(st, scd, pose, [cam], maps=("color", "depth"))[0]
    sparse = {k: v[: n // 40].contiguous() for k, v in scd.items()}
    opac = R.render(st, sparse, pose, [cam], maps=("opacity",))[0]["opacity"]
    color, depth = tgt["color"].contiguous(), tgt["depth"].contiguous()
    rng = np.random.default_rng(seed)
    grad = torch.from_numpy(rng.uniform(0, 4e-3, n).astype(np.float32)).cuda()
    cnt = torch.from_numpy(rng.integers(0, 12, n).astype(np.int32)).cuda()
    z = torch.from_numpy(rng.standard_normal((n, 2, 3)).astype(np.float32)).cuda()
    keep = torch.from_numpy((rng.random(n) < 0.95).astype(np.uint8)).cuda()
    moments = [torch.zeros((n, w), device="cuda") for w in (3, 3, 4, 1, 3)] * 2
    spare = {k: torch.empty((n + cam["width"] * cam["height"],) + v.shape[1:], device="cuda")
             for k, v in scd.items()}

    from paper_2403_16095_amd import binding as B
    # outputs allocated once: the timed calls are the library's own (each
    # synchronises to return its count)
    dens_dst = R.empty_like_set(scd, 2 * n)
    comp_dst = R.empty_like_set(scd, n)
    mom_dst = [torch.empty_like(m) for m in moments]
    stream = torch.cuda.current_stream().cuda_stream

    import ctypes as C
    L = B.lib()
    n_out = C.c_int64(0)

    def prepared(fn, *args):
        """The library call with its ctypes arguments built once, so the timed
        region holds the call alone."""
        def call():
            st = fn(*args)
            if st != B.CGSR_OK and st != B.CGSR_ERR_CAPACITY:
                raise B.CgsrError(st, L.cgsr_last_error().decode())
            return n_out.value
        return call

    spare_s, cam_s = R.arrays_struct(spare), R.camera_struct(cam)
    spawn = prepared(L.cgsr_spawn_gaussians, C.byref(spare_s), n, spare["means"].shape[0], C.byref(cam_s),
                     pose.reshape(12).data_ptr(), color.data_ptr(), depth.data_ptr(), opac.data_ptr(),
                     C.c_float(R.SPAWN_PSI), 1, C.c_float(0.0), C.byref(n_out), stream)
    src_s, dens_s, comp_s = R.arrays_struct(scd), R.arrays_struct(dens_dst), R.arrays_struct(comp_dst)
    densify = prepared(L.cgsr_densify_gaussians, n, grad.data_ptr(), cnt.data_ptr(), C.c_float(2e-4),
                       C.c_float(0.02), z.data_ptr(), C.byref(src_s), C.byref(dens_s), 2 * n, C.byref(n_out), stream)
    k = len(moments)
    ex_src = (C.c_void_p * k)(*[m.data_ptr() for m in moments])
    ex_dst = (C.c_void_p * k)(*[m.data_ptr() for m in mom_dst])
    ex_w = (C.c_int32 * k)(*[m.shape[1] for m in moments])
    compact = prepared(L.cgsr_compact_gaussians, n, keep.data_ptr(), C.byref(src_s), C.byref(comp_s), k, ex_src,
                       ex_dst, ex_w, C.byref(n_out), stream)

    res = {}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for name, fn in (("spawn", spawn), ("densify", densify), ("compact", compact)):
        out = fn()
        torch.cuda.synchronize()
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        gpu_ms = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ev[0].record()
            fn()
            ev[1].record()
            ev[1].synchronize()
            gpu_ms.append(ev[0].elapsed_time(ev[1]))
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        gpu_ms.sort()
        res[name] = dict(ms=round(ms, 4), gpu_ms_median=round(gpu_ms[len(gpu_ms) // 2], 4), result=int(out))
        log(f"{name}: {ms:.3f} ms per call wall, {gpu_ms[len(gpu_ms) // 2]:.3f} ms on the stream -> {out}")
    total = sum(r["ms"] for r in res.values())
    copy_gbs = copy_bandwidth(torch)
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle: the same spawn; densify and compact on a 50k sample, scaled to 1M)")
        from oracle import management as M
        P = pose.cpu().double().numpy()
        t0 = time.perf_counter()
        M.spawn(color.cpu().double().numpy(), depth.cpu().double().numpy(), cam, (P[:9].reshape(3, 3), P[9:]),
                opac.cpu().double().numpy())
        t_spawn = time.perf_counter() - t0
        k = 50_000
        sub = {key: v[:k] for key, v in full.items()}
        t0 = time.perf_counter()
        M.densify(sub, grad[:k].cpu().numpy(), cnt[:k].cpu().numpy(), 2e-4, 0.02, z[:k].cpu().numpy())
        M.compact(sub, keep[:k].cpu().numpy())
        t_rest = (time.perf_counter() - t0) * n / k
        import oracle
        cpu = {"value": round((t_spawn + t_rest) * 1e3, 1), "unit": "ms", "cores": 1, "kind": "oracle",
               "sample": f"spawn on the same view in {t_spawn:.1f} s; densify + compact of 50k Gaussians "
                         f"scaled by 20 (numpy, one thread)"}
    # compaction moves every array once in and the kept ones once out
    floats = 14 + sum(m.shape[1] for m in moments)
    b = n * (floats * 4 + 1) + res["compact"]["result"] * floats * 4
    return {
        "metric": "Gaussian management round (spawn 1200x680 + densify 1M + compact 1M with moments), ms",
        "value": round(total, 4), "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(total, 4), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "management: 1M Gaussians on an 8x6x3 m room; spawn from the pixels a 25k-Gaussian "
                               "render leaves below opacity 0.5 in a 1200x680 view; densify with statistics "
                               "U[0, 4e-3] / U{0..11}, threshold 2e-4, dense scale 0.02; compact keeping 95% "
                               "with 10 moment arrays", "gaussians": n},
        "ops": res,
        "hbm_roofline": {"kernel": "compact", "algorithmic_bytes": b,
                         "stream_ms": res["compact"]["gpu_ms_median"],
                         "achieved_GBs": round(b / (res["compact"]["gpu_ms_median"] * 1e-3) / 1e9, 2),
                         "peak_GBs": HBM_PEAK_GBS,
                         "frac": round(b / (res["compact"]["gpu_ms_median"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
                         "copy_GBs": round(copy_gbs, 1),
                         "frac_of_copy": round(b / (res["compact"]["gpu_ms_median"] * 1e-3) / 1e9 / copy_gbs, 5)},
        **({"cpu_baseline": cpu} if cpu else {}),
    }


def run_batched_tracking(args, torch, R, synth, frames=32, iters=20):
    import numpy as np
    B = R.B
    n = 1_000_000
    seed = 5
    log(f"building workload: {n} Gaussians, {frames} frames of uneven resolution")
    sc = synth.room_scene(seed, n, (8.0, 6.0, 3.0))
    scd = {k: torch.from_numpy(v).cuda() for k, v in sc.items()}
    fr = synth.tracking_frames(seed + 1000, frames)
    cams = [f[0] for f in fr]
    Pt = torch.stack([R.pose_tensor(*f[1]) for f in fr]).contiguous()
    tst = R.State()
    tgt = R.render(tst, scd, Pt, cams, maps=("color", "depth"))
    tcs = [t["color"].clone() for t in tgt]
    tds = [t["depth"].clone() for t in tgt]
    del tgt, tst
    start = [synth.perturb_pose(*f[1], seed + 2000 + k) for k, f in enumerate(fr)]
    P0 = torch.stack([R.pose_tensor(*p) for p in start]).contiguous()
    params = R.adam_params()
    g = R.gaussians_struct(scd)
    cam_s = [R.camera_struct(c) for c in cams]
    lam = R.TRACK_LAMBDA

    def make(vs, margin):
        """Graph of `iters` fused tracking steps over frames vs (reset inside)."""
        V = len(vs)
        pose = torch.empty((V, 12), device="cuda")
        pose0 = P0[vs].contiguous()
        adam = torch.zeros((V, 16), device="cuda")
        # the solve reads no work counts (only pair peaks and overflow)
        st = R.State(sync_capacity=True, count_work=False)
        cs = [cam_s[v] for v in vs]
        tc = [tcs[v].data_ptr() for v in vs]
        td = [tds[v].data_ptr() for v in vs]

        def step():
            B.cgsr_tracking_step(st.handle, g, V, pose.data_ptr(), cs, tc, td, float(lam[0]), float(lam[1]),
                                 None, adam.data_ptr(), params, None, R._stream())
        # Size the tile buckets from an eager run of the same loop (the pair
        # count moves with the poses), then capture it.
        pose.copy_(pose0)
        adam.zero_()
        peak = 0
        for _ in range(iters):
            step()
            peak = max(peak, int(st.stats().peak_pairs))
        st.reserve(tile_pairs=int(peak * margin) + 64)
        for attempt in range(3):
            graph = torch.cuda.CUDAGraph()
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                with torch.cuda.graph(graph, stream=side):
                    torch.mul(pose0, 1.0, out=pose)
                    adam.zero_()
                    for _ in range(iters):
                        step()
            torch.cuda.current_stream().wait_stream(side)
            st.check()          # starts a clean overflow period
            graph.replay()
            torch.cuda.synchronize()
            s = st.stats()
            if not s.overflow:
                break
            # the replayed trajectory needed more pairs than the eager one:
            # grow and capture again
            log(f"frames {vs[0]}..{vs[-1]}: replay needed {s.peak_pairs} pairs (eager peak {peak}); recapturing")
            try:
                st.check()
            except R.B.CgsrError:
                pass
            st.reserve(tile_pairs=int(s.peak_pairs * 1.25) + 64)
        # the graph reads and writes these tensors: keep them alive with it
        return graph, st, pose, (pose0, adam)

    res = {}
    for name, groups in (("batched", [list(range(frames))]), ("sequential", [[v] for v in range(frames)])):
        margin = 1.5
        for attempt in range(3):
            made = [make(vs, margin) for vs in groups]

            def solve():
                for gr, _, _, _ in made:
                    gr.replay()
            reps = max(1, args.steps // iters)
            for _ in range(max(1, args.warmup // iters)):
                solve()
            wall, ev = _sync_timed(torch, solve, reps)
            over = []
            for k, (_, st, _, _) in enumerate(made):
                s = st.stats()
                if s.overflow:
                    over.append((groups[k][0], int(s.peak_pairs), int(s.pair_capacity)))
            if not over:
                break
            # Replays of some solve needed more pairs than its sizing run (the
            # pose trajectory, and with it the visible set, differs from run
            # to run through the order of float atomics): size up and time again.
            log(f"{name}: pair capacity exceeded (first frame, peak, capacity): {over[:4]}; retiming")
            margin *= 2.0
            del made
        fi = frames * iters * reps
        fin = torch.cat([p for _, _, p, _ in made]).cpu()
        res[name] = dict(wall=wall, fi=fi, value=fi / wall, poses=fin)
        if name == "batched":
            # the dominant kernel: the fused tracking blend over all frames,
            # re-run back to back after the last replayed step
            res[name]["blend_ms"] = B.cgsr_time_tracking_blend(made[0][1].handle, 50, R._stream())
        terr = [float((fin[k, 9:].double() - Pt[k, 9:].cpu().double()).abs().max()) for k in range(frames)]
        log(f"{name}: {fi / wall:.1f} frame-iterations/s; final |t - t_true|_inf max {max(terr):.3e} "
            f"median {sorted(terr)[frames // 2]:.3e}")
        del made
    d = float((res["batched"]["poses"] - res["sequential"]["poses"]).abs().max())
    log(f"batched vs sequential final poses max diff {d:.2e}")
    # work counts of one batched step at the start poses (the timed states
    # keep none; they depend only on the workload)
    cst = R.State(sync_capacity=True, count_work=True)
    cpose = P0.clone()
    cd = torch.zeros((frames, 6), device="cuda")
    B.cgsr_tracking_step(cst.handle, g, frames, cpose.data_ptr(), cam_s, [t.data_ptr() for t in tcs],
                         [t.data_ptr() for t in tds], float(lam[0]), float(lam[1]), cd.data_ptr(), None, None, None,
                         R._stream())
    cs = cst.stats()
    stats = dict(visible=int(cs.visible), pairs=int(cs.pairs), evaluations=int(cs.processed),
                 blended=int(cs.blended), walked=int(cs.walked))
    del cst
    flops = (FLOP_EVAL * stats["evaluations"] + FLOP_BLEND * stats["blended"] + FLOP_EVAL * stats["walked"]
             + FLOP_BLEND_BWD * stats["blended"])
    roof = alu_roofline("blend_track", "raster_track_kernel<1, false, false>", flops, res["batched"]["blend_ms"],
                        "50 back-to-back launches between two HIP events")
    ms = res["batched"]["wall"] * 1e3 / (res["batched"]["fi"] / frames)
    out = {
        "metric": "batched tracking frame-iters/s (fwd+pose-bwd) 32 mixed-resolution frames 1M Gaussians",
        "value": round(res["batched"]["value"], 2), "unit": "frame-it/s", "n_gpus": 1,
        "steps": res["batched"]["fi"] // frames, "warmup": max(1, args.warmup // iters) * iters,
        "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batched tracking: {n} Gaussians on an 8x6x3 m room, {frames} frames drawn from "
                               "320x240/640x480/960x540/1200x680 (f = 525 W/640), 20-iteration Adam loops "
                               "captured in one HIP graph", "gaussians": n, "frames": frames,
                   "resolutions": [[c["width"], c["height"]] for c in cams], "solve_iters": iters},
        "sequential": {"value": round(res["sequential"]["value"], 2),
                       "speedup_batched": round(res["batched"]["value"] / res["sequential"]["value"], 3),
                       "final_pose_max_diff": d},
        "roofline": roof,
        "stats": stats,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, one frame per resolution)")
        import oracle
        per_res, tot = {}, 0.0
        for v, c in enumerate(cams):
            key = (c["width"], c["height"])
            if key not in per_res:
                per_res[key] = oracle_tracking_seconds(sc, c, start[v], tcs[v].cpu().numpy(), tds[v].cpu().numpy())
            tot += per_res[key]
        out["cpu_baseline"] = {"value": round(frames / tot, 5), "unit": "frame-it/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": "one tracking iteration per distinct resolution ("
                                         + ", ".join(f"{w}x{h}: {t:.1f} s" for (w, h), t in per_res.items())
                                         + "), extrapolated to the 32-frame mix"}
    return out



def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="tracking",
                    choices=("tracking", "mapping", "batched-mapping", "batched-tracking", "management"))
    ap.add_argument("--steps", type=int, default=2000, help="timed tracking iterations (exactly)")
    ap.add_argument("--warmup", type=int, default=200, help="untimed tracking iterations (exactly)")
    ap.add_argument("--solve-iters", type=int, default=50, help="iterations per captured solve")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stage-timing", action="store_true")
    ap.add_argument("--replays", type=int, default=100, help="solve replays timed one by one for the spread")
    ap.add_argument("--blend-reps", type=int, default=200,
                    help="back-to-back re-runs of the fused blend that time the dominant kernel")
    ap.add_argument("--mapping-ppl", default="auto", metavar="FWD,BWD",
                    help="pixels per lane of the mapping blends (forward, backward), or auto")
    ap.add_argument("--tracking-only", action="store_true",
                    help="only the headline tracking line (no mapping / batched workloads beside it)")
    ap.add_argument("--ppl", type=int, default=0, choices=(0, 1, 2, 4),
                    help="pixels per lane of the tracking blend (0: autotune)")
    ap.add_argument("--eager", action="store_true",
                    help="run the solves without graph capture (same kernels; for counter collection)")
    ap.add_argument("--sh-degree", type=int, default=0, choices=(0, 1, 2, 3),
                    help="view-dependent colour of this SH degree instead of rgb (tracking and mapping workloads)")
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
    if args.workload != "tracking":
        if args.workload == "batched-tracking":
            out = run_batched_tracking(args, torch, R, synth)
        elif args.workload == "management":
            out = run_management(args, torch, R, synth)
        else:
            out = run_mapping(args, torch, R, synth, 1 if args.workload == "mapping" else 8)
        print(json.dumps(out), flush=True)
        return
    deg = args.sh_degree
    log("building workload: 100k Gaussians, 640x480" + (f", SH degree {deg}" if deg else ""))
    sc, prob, P0, true_pose = build_workload(torch, R, synth, sh_degree=deg)
    iters = args.solve_iters
    if args.ppl:
        fppl = bppl = args.ppl
        log(f"pixels per lane: {fppl} (fixed)")
    else:
        probe = R.TrackingSolver(prob, iters=1, use_graph=False, reset_pose=P0)
        fppl, bppl = probe.autotune(P0)
        del probe
        log(f"autotuned pixels per lane (whole steps timed on the solve's state configuration): {fppl}")

    def make_solver(k):
        s_ = R.TrackingSolver(prob, iters=k, use_graph=not args.eager, reset_pose=P0, fwd_ppl=fppl, bwd_ppl=bppl)
        s_.prepare(P0)
        return s_

    solver = make_solver(iters)
    partial = {}

    def run_iterations(k):
        """Exactly k tracking iterations: whole solves of `iters` from the
        start pose, then one solve of the remainder (its own graph)."""
        full, rem = divmod(k, iters)
        for _ in range(full):
            solver.run()
        if rem:
            if rem not in partial:
                partial[rem] = make_solver(rem)
            partial[rem].run()

    steps, warmup = args.steps, args.warmup
    if warmup % iters and (warmup % iters) not in partial:
        partial[warmup % iters] = make_solver(warmup % iters)
    if steps % iters and (steps % iters) not in partial:
        partial[steps % iters] = make_solver(steps % iters)
    log(f"warmup {warmup} iterations")
    run_iterations(warmup)
    torch.cuda.synchronize()
    solver.check()

    log(f"timed {steps} iterations ({steps // iters} solves of {iters}"
        + (f" + one of {steps % iters})" if steps % iters else ")"))
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    run_iterations(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    solver.check()
    for p_ in partial.values():
        p_.check()
    ms_per_step = wall * 1e3 / steps
    value = steps / wall
    log(f"{value:.1f} it/s ({ms_per_step * 1e3:.1f} us/it wall, {gpu_ms * 1e3 / steps:.1f} us/it events)")

    # Spread: every replay of a whole solve timed on its own by HIP events.
    nrep = args.replays
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nrep)]
    torch.cuda.synchronize()
    for a, b in evs:
        a.record(stream)
        solver.run()
        b.record(stream)
    torch.cuda.synchronize()
    solver.check()
    per_it = sorted(a.elapsed_time(b) * 1e3 / iters for a, b in evs)
    q = lambda f: round(per_it[min(nrep - 1, int(f * nrep))], 3)
    spread = {"replays": nrep, "iters_per_replay": iters, "unit": "us/it", "p10": q(0.1), "p50": q(0.5),
              "p90": q(0.9), "min": round(per_it[0], 3), "max": round(per_it[-1], 3)}
    log(f"per-iteration time over {nrep} solve replays: p10 {spread['p10']} p50 {spread['p50']} "
        f"p90 {spread['p90']} us")
    err_t = float((solver.pose.cpu().double()[9:] - torch.as_tensor(true_pose[1])).abs().max())
    log(f"final |t - t_true|_inf = {err_t:.2e} m")

    # The dominant kernel: the fused tracking blend of the solve's last step,
    # re-run back to back between two HIP events on the launch stream.
    blend_ms = solver.state.time_tracking_blend(args.blend_reps)
    log(f"fused tracking blend: {blend_ms * 1e3:.2f} us per launch ({args.blend_reps} back-to-back re-runs)")

    # The other stages: HIP events recorded by the library around each stage,
    # over eager steps of the same workload (each event pair adds a few us).
    stages = {}
    if not args.no_stage_timing:
        tst = R.State(sync_capacity=False, timing=True, fwd_ppl=fppl, bwd_ppl=bppl, count_work=False)
        tst.reserve(tile_pairs=int(solver.state.stats().pair_capacity))
        pose = P0.clone().reshape(1, 12)
        reps = 20
        dpose = torch.zeros((1, 6), device="cuda")
        for r in range(reps + 2):
            R.tracking_step(tst, prob.scene, pose, [prob.cam], [prob.target_color], [prob.target_depth],
                            dposes=dpose)
            t = tst.timings()
            if r >= 2:
                for k, v in t.items():
                    stages[k] = stages.get(k, 0.0) + v / reps
        tst.check()
        log("stage ms (events):", {k: round(v, 4) for k, v in stages.items()})
    # Work counts: the timed kernel keeps none (as in the solve); the same
    # step on a counting state gives them (they depend only on the workload).
    cst = R.State(fwd_ppl=fppl, bwd_ppl=bppl, count_work=True)
    dpose = torch.zeros((1, 6), device="cuda")
    R.tracking_step(cst, prob.scene, P0.clone().reshape(1, 12), [prob.cam], [prob.target_color],
                    [prob.target_depth], dposes=dpose)
    s = cst.stats()
    stats = dict(visible=int(s.visible), pairs=int(s.pairs), evaluations=int(s.processed),
                 blended=int(s.blended), walked=int(s.walked))
    log("stats:", stats)

    result = {
        "metric": METRIC + (f", SH degree {deg}" if deg else ""),
        "value": round(value, 2),
        "unit": "it/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "paper_context": {"value": 126.7, "unit": "it/s", "hardware": "RTX 4090 + i9-14900K",
                          "workload": "Replica Office 0, whole tracking loop, resolution and Gaussian count "
                                      "not stated (1000 / 7.89 ms, Table 5)"},
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "tracking: 100k Gaussians on a 5x4x3 m room, 640x480 f=525, "
                               f"render + L1 colour/depth loss + pose-only backward + Adam, {iters}-iteration "
                               "solves replayed from HIP graphs",
                   "gaussians": 100_000, "width": 640, "height": 480, "solve_iters": iters,
                   "pixels_per_lane": fppl, "sh_degree": deg,
                   "loss_lambda": list(R.TRACK_LAMBDA)},
        "spread": spread,
    }
    # The dominant kernel's ALU roofline: the tracking step's blend forward
    # and pose-only blend backward run as one launch per tile.
    flops = (FLOP_EVAL * stats["evaluations"] + FLOP_BLEND * stats["blended"]
             + FLOP_EVAL * stats["walked"] + FLOP_BLEND_BWD * stats["blended"])
    symbol = f"raster_track_kernel<{fppl}, {'true' if deg else 'false'}, false>"
    result["roofline"] = alu_roofline("blend_track", symbol, flops, blend_ms,
                                      f"{args.blend_reps} back-to-back launches between two HIP events",
                                      measured_counters(symbol))
    b = algorithmic_bytes(100_000, stats["visible"], stats["pairs"], 640 * 480, deg)
    copy_gbs = copy_bandwidth(torch)
    result["hbm_roofline"] = {"algorithmic_bytes_per_iter": b,
                              "achieved_GBs": round(b / (ms_per_step * 1e-3) / 1e9, 2),
                              "peak_GBs": HBM_PEAK_GBS,
                              "frac": round(b / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
                              "copy_GBs": round(copy_gbs, 1),
                              "frac_of_copy": round(b / (ms_per_step * 1e-3) / 1e9 / copy_gbs, 5)}
    if stages:
        result["stage_events_ms"] = {k: round(v, 5) for k, v in stages.items()}
    result["stats"] = stats
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        tc = prob.target_color.cpu().numpy()
        td = prob.target_depth.cpu().numpy()
        p0 = P0.cpu().double().numpy()
        result["cpu_baseline"] = cpu_baseline((sc, tc, td), prob.cam, (p0[:9].reshape(3, 3), p0[9:]),
                                              args.cpu_budget)
    del solver, partial
    if not args.tracking_only and deg == 0:
        result["workloads"] = other_workloads(args, torch, R, synth)
    print(json.dumps(result), flush=True)


def other_workloads(args, torch, R, synth):
    """The mapping, batched-mapping and batched-tracking workloads, each with
    its own steps, ALU roofline and (extrapolated) oracle baseline, reported
    beside the headline so every run records the batched-versus-unbatched
    ratios."""
    out = {}
    for name, fn, steps, warmup in (
            ("mapping", lambda a: run_mapping(a, torch, R, synth, 1), 50, 5),
            ("batched_mapping", lambda a: run_mapping(a, torch, R, synth, 8), 20, 3),
            ("batched_tracking", lambda a: run_batched_tracking(a, torch, R, synth), 20, 20)):
        sub = argparse.Namespace(**vars(args))
        sub.steps, sub.warmup, sub.sh_degree = steps, warmup, 0
        t0 = time.perf_counter()
        log(f"--- {name}")
        r = fn(sub)
        for k in ("n_gpus", "higher_is_better", "scaling", "dtype", "data"):
            r.pop(k, None)
        r["bench_seconds"] = round(time.perf_counter() - t0, 1)
        out[name] = r
        torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main()
