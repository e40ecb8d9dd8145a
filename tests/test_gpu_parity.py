"""HIP path vs the FP64 oracle, through the C ABI.

Renders must match within 1e-4 absolute on every map, gradients within 1e-3
relative (L2 per tensor).  Where float32 and float64 can legitimately take a
different discrete decision (a pixel whose alpha, stop, median or depth order
sits within the rounding margins of its threshold), the pixel must match one
of the results the oracle gives with that decision taken either way
(helpers.check_maps); no pixel is left out.  Tile lists hold the oracle's
binning lists in its order, less pairs shown unreachable (check_tiles).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2403_16095_amd import synth
from helpers import ORDER_MARGIN, check_maps, copy_device, grad_parity, identity_pose, pose12, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MAPS = ("color", "depth", "opacity", "depth_median", "uncertainty")
PARAMS = ("means", "log_scales", "quats", "opacity_logits", "rgb")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_16095_amd import rasterizer
    return rasterizer


def dev(scene):
    return {k: torch.from_numpy(np.ascontiguousarray(v, np.float32)).cuda() for k, v in scene.items()}


def t32(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def gpu_render(R, state, scene_d, pose, cam, dobs=None):
    p = R.pose_tensor(*pose)
    out = R.render(state, scene_d, p, [cam], None if dobs is None else [t32(dobs)])[0]
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}, p


@pytest.fixture(scope="module")
def config1():
    sc = synth.uniform_box_scene(0, 2000)
    cam = synth.SMALL_CAMERA
    tc, td = synth.random_targets(1000, cam)
    return sc, cam, tc, td


def test_render_config1_matches_oracle(R, config1):
    sc, cam, tc, td = config1
    say("case: config1 forward, 2000 Gaussians 64x48")
    st = R.State()
    gpu, _ = gpu_render(R, st, dev(sc), identity_pose(), cam, td)
    check_maps(gpu, sc, cam, identity_pose(), td, max_ambiguous=0.01, label="config1")
    s = st.stats()
    assert s.overflow == 0 and s.pairs > 0


def test_projection_records_match_oracle(R, config1):
    sc, cam, tc, td = config1
    say("case: config1 projection records")
    st = R.State()
    gpu_render(R, st, dev(sc), identity_pose(), cam, td)
    from paper_2403_16095_amd import binding as B
    keys, vals, ranges, recs, pst = B.cgsr_debug_buffers(st.handle)
    n = sc["means"].shape[0]
    rec = torch.empty((n, 12), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    copy_device(rec, recs, n * 12 * 4)
    rec = rec.cpu().numpy().astype(np.float64)
    proj = oracle.project(sc, cam, identity_pose())
    vis = proj["visible"] == 1
    # the mean is stored as a float pair (hi, lo) in slots 0-1 and 10-11
    mu = rec[vis, 0:2].astype(np.float64) + rec[vis, 10:12]
    np.testing.assert_allclose(mu, proj["mu"][vis], rtol=0, atol=1e-6)
    # the conic is stored as (a, k, c') of a (dx + k dy)^2 + c' dy^2
    a, k, cp = rec[vis, 2], rec[vis, 3], rec[vis, 4]
    conic = np.stack([a, k * a, cp + k * k * a], 1)
    np.testing.assert_allclose(conic, proj["conic"][vis], rtol=2e-6, atol=1e-9)
    np.testing.assert_allclose(rec[vis, 5], proj["opacity"][vis], rtol=1e-5)
    np.testing.assert_allclose(rec[vis, 6], proj["depth"][vis], rtol=1e-6)
    np.testing.assert_allclose(rec[vis, 7:10], sc["rgb"][vis], rtol=0, atol=0)


def tile_lists_from_gpu(R, st, n_tiles):
    from paper_2403_16095_amd import binding as B
    keys, vals, ranges, recs, pst = B.cgsr_debug_buffers(st.handle)
    s = st.stats()
    K = int(s.pairs)
    slots = n_tiles * int(s.pair_capacity)   # one bucket per tile
    v = torch.empty(slots, dtype=torch.int32, device="cuda")
    rg = torch.empty((n_tiles, 2), dtype=torch.int32, device="cuda")
    copy_device(v, vals, slots * 4)
    copy_device(rg, ranges, n_tiles * 8)
    v = v.cpu().numpy().astype(np.int64)
    rg = rg.cpu().numpy()
    lists = {t: v[rg[t, 0]:rg[t, 1]] for t in range(n_tiles) if rg[t, 1] > rg[t, 0]}
    assert sum(len(x) for x in lists.values()) == K
    return lists, K


def reaches_tile(proj, i, cam, t):
    """Whether Gaussian i reaches alpha >= 1/255 (Eq. 5, FP64) at a pixel of
    16x16 tile t."""
    tiles_x = (cam["width"] + 15) // 16
    ty, tx = divmod(t, tiles_x)
    xs = np.arange(16 * tx, min(16 * tx + 16, cam["width"]))
    ys = np.arange(16 * ty, min(16 * ty + 16, cam["height"]))
    X, Y = np.meshgrid(xs, ys)
    a, b, c = proj["conic"][i]
    dx, dy = X - proj["mu"][i][0], Y - proj["mu"][i][1]
    return bool((proj["opacity"][i] * np.exp(-0.5 * (a * dx * dx + 2 * b * dx * dy + c * dy * dy))
                 >= 1.0 / 255.0).any())


def check_tiles(R, sc, cam, pose):
    """Each tile's list is the oracle's list under 16x16 binning, in the same
    (depth, id) order, less Gaussians that reach alpha >= 1/255 at no pixel of
    the tile (the projection drops those pairs); every Gaussian that reaches
    one is kept."""
    st = R.State()
    gpu_render(R, st, dev(sc), pose, cam)
    tiles_x, tiles_y = (cam["width"] + 15) // 16, (cam["height"] + 15) // 16
    gl, K = tile_lists_from_gpu(R, st, tiles_x * tiles_y)
    proj = oracle.project(sc, cam, pose)
    ol = oracle.tile_lists(proj, cam, 16)
    # Gaussians whose rectangle edge lies within 1e-3 px of a pixel centre may
    # round either way in float32; depth near-ties may swap.
    edges = proj["rect_edges"]
    near_edge = (np.abs(edges - np.round(edges)) < 1e-3).any(1) & (proj["visible"] == 1)
    amb = set(np.nonzero(near_edge)[0].tolist())
    d = proj["depth"]
    n_checked = n_dropped = 0
    for t in set(gl) | set(ol):
        a = [i for i in gl.get(t, []) if i not in amb]
        full = [i for i in ol.get(t, []) if i not in amb]
        kept = set(a)
        assert kept <= set(full), ("not in the tile's binned list", t)
        for i in full:
            if i not in kept:
                assert not reaches_tile(proj, i, cam, t), ("dropped a Gaussian that reaches the tile", t, i)
                n_dropped += 1
        b = [i for i in full if i in kept]
        if a != b:
            # allow swaps of depth near-ties only
            assert sorted(a) == sorted(b), ("tile membership differs", t)
            for x, y in zip(a, b):
                if x != y:
                    assert abs(d[x] - d[y]) <= ORDER_MARGIN * d[x], ("order differs", t, x, y)
        n_checked += len(a)
    say("pairs", K, "checked", n_checked, "dropped", n_dropped, "ambiguous gaussians", len(amb))
    assert len(amb) <= 0.01 * max(1, int(proj["visible"].sum())) + 5
    return K


def test_tile_lists_match_oracle_binning_config1(R, config1):
    sc, cam, tc, td = config1
    say("case: config1 tile lists")
    check_tiles(R, sc, cam, identity_pose())


def test_tile_lists_match_oracle_binning_tracking_size(R):
    say("case: 100k room, 640x480 tile lists")
    sc = synth.room_scene(0, 100_000, (5.0, 4.0, 3.0))
    pose = synth.level_room_pose(0)
    K = check_tiles(R, sc, synth.TRACKING_CAMERA, pose)
    assert K > 10_000


def test_reach_tests_keep_every_contributor_of_thin_gaussians(R):
    """Needle-like, rotated Gaussians (per-axis log-scales with a wide spread)
    are where a binning rectangle overlaps most cells and tiles the ellipse
    misses, and where the closed-form reach test is most exposed to rounding:
    the tile lists keep every Gaussian that reaches its tile (FP64), and the
    maps still match the oracle (or, at pixels with a near-threshold
    decision, one of its admissible results)."""
    for cam in (synth.SMALL_CAMERA, synth.camera(200, 120, 150.0, 150.0, 100.0, 60.0)):
        say(f"case: 1500 thin Gaussians {cam['width']}x{cam['height']}")
        sc = synth.uniform_box_scene(11, 1500, log_scale=(-3.0, 1.6), opacity=(0.0, 1.5))
        check_tiles(R, sc, cam, identity_pose())
        st = R.State()
        gpu, _ = gpu_render(R, st, dev(sc), identity_pose(), cam)
        check_maps(gpu, sc, cam, identity_pose(), max_ambiguous=0.01, label=f"thin {cam['width']}x{cam['height']}")


@pytest.mark.parametrize("ppl", [2, 4])
def test_pixels_per_lane_variants(R, config1, ppl):
    """Blend kernels with 2 or 4 pixels per lane: forward maps bitwise equal to
    one pixel per lane, gradients within the oracle tolerance."""
    sc, cam, tc, td = config1
    say(f"case: config1 with {ppl} pixels per lane")
    scd = dev(sc)
    ref_state = R.State()
    ref, _ = gpu_render(R, ref_state, scd, identity_pose(), cam, td)
    st = R.State(fwd_ppl=ppl, bwd_ppl=ppl)
    got, _ = gpu_render(R, st, scd, identity_pose(), cam, td)
    for k in MAPS:
        assert np.array_equal(got[k], ref[k]), k
    rng = np.random.default_rng(22)
    H, W = cam["height"], cam["width"]
    dimg = dict(color=rng.standard_normal((3, H, W)), depth=rng.standard_normal((H, W)),
                opacity=rng.standard_normal((H, W)), depth_median=rng.standard_normal((H, W)),
                uncertainty=rng.standard_normal((H, W)))
    grads, dposes = R.backward(st, [{k: t32(v) for k, v in dimg.items()}])
    rb = oracle.backward(sc, cam, identity_pose(), td, dimg)
    for k in PARAMS:
        assert rel_l2(grads[k].cpu().numpy(), rb[k]) <= 1e-3, k
    assert np.abs(dposes[0].cpu().numpy() - rb["pose"]).max() <= 1e-3 * np.abs(rb["pose"]).max()
    # tracking-mode kernels
    d1, d2 = torch.zeros((1, 6), device="cuda"), torch.zeros((1, 6), device="cuda")
    P = R.pose_tensor(*identity_pose())
    R.tracking_step(ref_state, scd, P, [cam], [t32(tc)], [t32(td)], dposes=d1)
    R.tracking_step(st, scd, P, [cam], [t32(tc)], [t32(td)], dposes=d2)
    assert ((d1 - d2).abs().max() / d1.abs().max()).item() < 1e-4


def test_autotuner_picks_a_valid_setting(R):
    say("case: autotuner on a small tracking workload")
    sc = synth.room_scene(5, 20_000, (5.0, 4.0, 3.0))
    cam = synth.camera(320, 240, 262.5, 262.5, 160, 120)
    scd = dev(sc)
    P = R.pose_tensor(*synth.level_room_pose(3))
    st = R.State()
    tgt = R.render(st, scd, P, [cam])[0]
    P_before = P.clone()
    f, b = R.autotune_tracking(st, scd, P, [cam], [tgt["color"]], [tgt["depth"]], repeats=2)
    say("picked", f, b)
    assert f in (1, 2, 4) and b in (1, 2, 4)
    assert torch.equal(P, P_before)
    out = R.render(st, scd, P, [cam])[0]
    assert torch.equal(out["color"], tgt["color"])
    # the solver's own tune: whole steps on its state configuration, then the
    # captured solve runs with the pick
    prob = R.TrackingProblem(scd, cam, tgt["color"].clone(), tgt["depth"].clone())
    solver = R.TrackingSolver(prob, iters=3, reset_pose=P)
    f2, b2 = solver.autotune(P, repeats=2)
    say("solver picked", f2, b2)
    assert f2 == b2 and f2 in (1, 2, 4)
    solver.prepare(P)
    solver.run()
    torch.cuda.synchronize()
    solver.check()


def test_render_autotuner_picks_and_keeps_a_setting(R):
    """cgsr_autotune_render times render + backward for the nine (forward,
    backward) pixels-per-lane pairs, keeps the pick per workload shape, and a
    render with the pick writes the same maps as the default setting."""
    from paper_2403_16095_amd import binding as B
    say("case: render autotuner on a 20k-Gaussian 320x240 mapping workload")
    sc = synth.room_scene(5, 20_000, (5.0, 4.0, 3.0))
    cam = synth.camera(320, 240, 262.5, 262.5, 160, 120)
    scd = dev(sc)
    P = R.pose_tensor(*synth.level_room_pose(3))
    H, W = cam["height"], cam["width"]
    rng = np.random.default_rng(5)
    td = t32(rng.uniform(0.5, 5.0, (H, W)))
    maps = {k: torch.empty(sh, device="cuda") for k, sh in (("color", (3, H, W)), ("depth", (H, W)),
                                                            ("uncertainty", (H, W)))}
    dimgs = {k: t32(rng.standard_normal(v.shape) * 1e-3) for k, v in maps.items()}
    grads = {k: torch.zeros_like(v) for k, v in scd.items()}
    dposes = torch.zeros((1, 6), device="cuda")
    out_s = B.cgsr_images(maps["color"].data_ptr(), maps["depth"].data_ptr(), None, None,
                          maps["uncertainty"].data_ptr())
    grad_s = B.cgsr_images(dimgs["color"].data_ptr(), dimgs["depth"].data_ptr(), None, None,
                           dimgs["uncertainty"].data_ptr())
    dG = B.cgsr_gaussian_grads(grads["means"].data_ptr(), grads["log_scales"].data_ptr(), grads["quats"].data_ptr(),
                               grads["opacity_logits"].data_ptr(), grads["rgb"].data_ptr(), None)
    st = R.State()
    g = R.gaussians_struct(scd)
    cs = [R.camera_struct(cam)]
    picks = []
    for _ in range(2):
        o = B.cgsr_autotune_render(st.handle, g, 1, P.data_ptr(), cs, [td.data_ptr()], [out_s], [grad_s], dG,
                                   dposes.data_ptr(), 2, torch.cuda.current_stream().cuda_stream)
        picks.append((int(o.fwd_pixels_per_lane), int(o.bwd_pixels_per_lane)))
    say("picked", picks)
    assert picks[0] == picks[1] and all(x in (1, 2, 4) for x in picks[0])
    tuned = R.render(st, scd, P, [cam], [td])[0]
    ref = R.render(R.State(), scd, P, [cam], [td])[0]
    torch.cuda.synchronize()
    for k in ("color", "depth", "opacity", "depth_median", "uncertainty"):
        assert torch.equal(tuned[k], ref[k]), k


def test_long_tile_segments_take_the_merge_path(R):
    """More than 4096 Gaussians in one tile: the segment sort goes through its
    chunked LDS sort plus in-workgroup merges; lists and maps must still match."""
    say("case: 10000 Gaussians crowding four tiles of a 64x48 image")
    sc = synth.uniform_box_scene(7, 10_000, xy=(-0.06, 0.06), z=(2.0, 3.0), log_scale=(-5.5, 0.3),
                                 opacity=(-3.0, 1.0))
    cam = synth.SMALL_CAMERA
    st = R.State()
    gpu, _ = gpu_render(R, st, dev(sc), identity_pose(), cam)
    tiles_x, tiles_y = (cam["width"] + 15) // 16, (cam["height"] + 15) // 16
    gl, K = tile_lists_from_gpu(R, st, tiles_x * tiles_y)
    longest = max(len(v) for v in gl.values())
    say("pairs", K, "longest tile list", longest)
    assert longest > 2 * 4096
    proj = oracle.project(sc, cam, identity_pose())
    d = proj["depth"]
    for t, ids in gl.items():
        key = d[ids]
        assert np.all((np.diff(key) > 0) | ((np.diff(key) == 0) & (np.diff(ids) > 0)) |
                      (np.abs(np.diff(key)) <= 1e-6 * key[1:])), t
    check_tiles(R, sc, cam, identity_pose())
    check_maps(gpu, sc, cam, identity_pose(), max_ambiguous=0.05, label="crowded tiles")


def test_backward_config1_all_params(R, config1):
    sc, cam, tc, td = config1
    say("case: config1 full backward")
    rng = np.random.default_rng(21)
    H, W = cam["height"], cam["width"]
    dimg = dict(color=rng.standard_normal((3, H, W)), depth=rng.standard_normal((H, W)),
                opacity=rng.standard_normal((H, W)), depth_median=rng.standard_normal((H, W)),
                uncertainty=rng.standard_normal((H, W)))
    st = R.State()
    gpu_render(R, st, dev(sc), identity_pose(), cam, td)
    grads, dposes = R.backward(st, [{k: t32(v) for k, v in dimg.items()}])
    torch.cuda.synchronize()
    ref = oracle.backward(sc, cam, identity_pose(), td, dimg)
    for k in PARAMS:
        grad_parity(k, grads[k].cpu().numpy(), ref[k], label="config1")
    dp = dposes[0].cpu().numpy()
    e = np.abs(dp - ref["pose"]).max() / np.abs(ref["pose"]).max()
    say("pose", dp, ref["pose"], e)
    assert e <= 1e-3


def test_pose_only_backward_tracking_loss(R, config1):
    sc, cam, tc, td = config1
    say("case: config1 pose-only backward with the tracking loss")
    st = R.State()
    scd = dev(sc)
    gpu, p = gpu_render(R, st, scd, identity_pose(), cam, td)
    ref = oracle.render(sc, cam, identity_pose(), td)
    _, dimg = oracle.tracking_loss(ref, tc, td, lam=(1.0, 1.0))
    grads, dposes = R.backward(st, [{k: t32(v) for k, v in dimg.items()}], param_grads=False)
    rb = oracle.backward(sc, cam, identity_pose(), td, dimg)
    dp = dposes[0].cpu().numpy()
    e = np.abs(dp - rb["pose"]).max() / np.abs(rb["pose"]).max()
    say("pose", dp, rb["pose"], e)
    assert grads is None and e <= 1e-3


def test_tracking_loss_grad_kernel(R, config1):
    sc, cam, tc, td = config1
    say("case: tracking loss gradient kernel")
    rng = np.random.default_rng(3)
    H, W = cam["height"], cam["width"]
    color, depth = rng.random((3, H, W)), rng.uniform(1, 4, (H, W))
    loss = torch.zeros(1, device="cuda")
    dc, dd = R.tracking_loss_grad(t32(color), t32(depth), t32(tc), t32(td), lam=(0.2, 1.0), loss=loss)
    L, ref = oracle.tracking_loss(dict(color=color.astype(np.float32), depth=depth.astype(np.float32)), tc, td,
                                  lam=(0.2, 1.0))
    np.testing.assert_allclose(dc.cpu().numpy(), ref["color"], rtol=1e-6, atol=1e-12)
    np.testing.assert_allclose(dd.cpu().numpy(), ref["depth"], rtol=1e-6, atol=1e-12)
    assert abs(loss.item() - L) <= 1e-5 * abs(L)


def test_pose_adam_step_kernel(R):
    say("case: pose Adam + retraction kernel")
    rng = np.random.default_rng(4)
    Rm = synth.rot_about_axis(rng.standard_normal(3), 0.7)
    t = rng.standard_normal(3)
    pose = R.pose_tensor(Rm, t).reshape(1, 12).clone()
    adam = torch.zeros((1, 16), device="cuda")
    ref_pose = (Rm, t)
    m = v = np.zeros(6)
    lr = np.array([0.00215] * 3 + [0.0015] * 3)
    for k in range(20):
        g = rng.standard_normal(6) * 10 ** rng.uniform(-3, 1)
        dp = t32(g.reshape(1, 6)).clone()
        R.pose_adam_step(pose, dp, adam)
        assert float(dp.abs().max()) == 0.0
        xi, m, v = oracle.adam_step(np.zeros(6), g, m, v, k + 1, lr)
        ref_pose = oracle.retract(ref_pose, xi)
    got = pose.cpu().numpy().reshape(12).astype(np.float64)
    np.testing.assert_allclose(got, pose12(*ref_pose), atol=2e-6)


def test_forward_is_deterministic_and_batched_equals_sequential(R):
    say("case: 3 views batched vs sequential, repeated")
    sc = synth.room_scene(1, 20_000, (5.0, 4.0, 3.0))
    cams = [synth.camera(160, 120, 131.25, 131.25, 80, 60), synth.camera(96, 80, 90, 90, 47.5, 40.2),
            synth.camera(200, 64, 150, 150, 100, 32)]
    poses = [synth.level_room_pose(s) for s in (3, 4, 5)]
    scd = dev(sc)
    P = torch.stack([R.pose_tensor(*p) for p in poses])
    st = R.State()
    batched = R.render(st, scd, P, cams)
    batched = [{k: v.clone() for k, v in o.items()} for o in batched]
    again = R.render(st, scd, P, cams)
    for v in range(3):
        single = R.render(R.State(), scd, P[v].contiguous(), [cams[v]])[0]
        for k in ("color", "depth", "opacity", "depth_median"):
            assert torch.equal(batched[v][k], again[v][k]), ("repeat", v, k)
            assert torch.equal(batched[v][k], single[k]), ("batched", v, k)


def test_batched_backward_equals_sum_of_views(R):
    say("case: batched backward vs per-view backward")
    sc = synth.room_scene(2, 20_000, (5.0, 4.0, 3.0))
    cams = [synth.camera(160, 120, 131.25, 131.25, 80, 60), synth.camera(128, 96, 105, 105, 64, 48)]
    poses = [synth.level_room_pose(s) for s in (6, 7)]
    scd = dev(sc)
    P = torch.stack([R.pose_tensor(*p) for p in poses])
    rng = np.random.default_rng(8)
    dimgs = [dict(color=t32(rng.standard_normal((3, c["height"], c["width"]))),
                  depth=t32(rng.standard_normal((c["height"], c["width"])))) for c in cams]
    st = R.State()
    R.render(st, scd, P, cams)
    gb, pb = R.backward(st, dimgs)
    acc = {k: torch.zeros_like(v) for k, v in gb.items()}
    for v in range(2):
        s1 = R.State()
        R.render(s1, scd, P[v].contiguous(), [cams[v]])
        g1, p1 = R.backward(s1, [dimgs[v]])
        for k in acc:
            acc[k] += g1[k]
        e = (p1[0] - pb[v]).abs().max().item() / p1[0].abs().max().item()
        assert e < 1e-4, (v, e)
    for k in acc:
        e = rel_l2(gb[k].cpu().numpy(), acc[k].cpu().numpy())
        assert e < 1e-5, (k, e)


def test_sampled_pixels_tracking_size(R):
    """Full tracking size (100k Gaussians, 640x480) in the benchmark's launch
    configuration: 3000 sampled pixels against the brute-force oracle."""
    say("case: 100k room 640x480 sampled forward")
    sc = synth.room_scene(0, 100_000, (5.0, 4.0, 3.0))
    cam = synth.TRACKING_CAMERA
    pose = synth.level_room_pose(0)
    st = R.State()
    _, td = synth.random_targets(1001, cam, depth_range=(0.5, 4.0))
    gpu, _ = gpu_render(R, st, dev(sc), pose, cam, td)
    rng = np.random.default_rng(9)
    px = rng.choice(cam["width"] * cam["height"], 3000, replace=False)
    ref = oracle.render(sc, cam, pose, td, candidates=0, pixels=px)
    check_maps(gpu, sc, cam, pose, td, px=px, ref=ref, max_ambiguous=0.03, label="tracking 640x480 sampled")


def test_pose_gradient_tracking_size(R):
    """Full tracking size: the pose gradient of the tracking loss (Eq. 19) over
    all 307200 pixels against the oracle's analytic FP64 gradient."""
    say("case: 100k room 640x480 pose gradient")
    sc = synth.room_scene(0, 100_000, (5.0, 4.0, 3.0))
    cam = synth.TRACKING_CAMERA
    Rt, tt = synth.level_room_pose(0)
    pose = synth.perturb_pose(Rt, tt, 1000)
    ref_t = oracle.render(sc, cam, (Rt, tt))
    st = R.State()
    ref = oracle.render(sc, cam, pose)
    _, dimg = oracle.tracking_loss(ref, ref_t["color"], ref_t["depth"])
    gpu_render(R, st, dev(sc), pose, cam)
    _, dposes = R.backward(st, [{k: t32(v) for k, v in dimg.items()}], param_grads=False)
    rb = oracle.backward(sc, cam, pose, None, dimg)
    dp = dposes[0].cpu().numpy()
    e = np.abs(dp - rb["pose"]).max() / np.abs(rb["pose"]).max()
    say("pose", dp, rb["pose"], e)
    assert e <= 1e-3


def test_empty_and_culled_scenes(R):
    say("case: empty and fully culled scenes")
    cam = synth.SMALL_CAMERA
    empty = {k: np.zeros((0,) + s, np.float32) for k, s in
             dict(means=(3,), log_scales=(3,), quats=(4,), opacity_logits=(), rgb=(3,)).items()}
    st = R.State()
    empty_d = {k: torch.zeros(v.shape, device="cuda") for k, v in empty.items()}
    out, _ = gpu_render(R, st, empty_d, identity_pose(), cam)
    for k, v in out.items():
        assert np.all(v == 0), k
    sc = synth.uniform_box_scene(0, 500)
    sc["means"][:, 2] = -1.0   # all behind the camera
    out, _ = gpu_render(R, st, dev(sc), identity_pose(), cam)
    for k, v in out.items():
        assert np.all(v == 0), k
    assert st.stats().pairs == 0
    grads, dposes = R.backward(st, [dict(color=torch.ones((3, 48, 64), device="cuda"))])
    assert float(dposes.abs().max()) == 0.0 and all(float(g.abs().max()) == 0.0 for g in grads.values())


def test_error_paths(R, config1):
    from paper_2403_16095_amd import binding as B
    say("case: error paths")
    sc, cam, tc, td = config1
    st = R.State()
    with pytest.raises(B.CgsrError) as e:       # backward before any forward
        B.cgsr_backward(st.handle, [B.cgsr_images()], None, torch.zeros(6, device="cuda").data_ptr(), 0)
    assert e.value.status == B.CGSR_ERR_STATE
    scd = dev(sc)
    p = R.pose_tensor(*identity_pose())
    bad = dict(cam, width=0)
    with pytest.raises(B.CgsrError) as e:
        R.render(st, scd, p, [bad])
    assert e.value.status == B.CGSR_ERR_INVALID_ARG
    with pytest.raises(B.CgsrError) as e:       # uncertainty without sensor depth
        B.cgsr_render(st.handle, R.gaussians_struct(scd), 1, p.data_ptr(), [R.camera_struct(cam)], None,
                      [B.cgsr_images(None, None, None, None, torch.empty(48 * 64, device="cuda").data_ptr())], 0)
    assert e.value.status == B.CGSR_ERR_INVALID_ARG
    # capacity overflow without the host sync: flagged, reported by check()
    st2 = R.State(sync_capacity=False)
    st2.reserve(records=2000, pixels=64 * 48, tiles=12, tile_pairs=100)
    R.render(st2, scd, p, [cam])
    with pytest.raises(B.CgsrError) as e:
        st2.check()
    assert e.value.status == B.CGSR_ERR_CAPACITY
    # and with the default sync the same state sizes itself
    st3 = R.State()
    st3.reserve(tile_pairs=100)
    out = R.render(st3, scd, p, [cam])
    st3.check()


def test_autograd_function_matches_explicit_backward(R, config1):
    say("case: autograd Function")
    sc, cam, tc, td = config1
    scd = {k: v.clone().requires_grad_(True) for k, v in dev(sc).items()}
    p = R.pose_tensor(*identity_pose())
    xi = torch.zeros(6, device="cuda", requires_grad=True)
    out = R.rasterize(scd, p, cam, t32(td), xi=xi)
    loss = (out["color"] * t32(tc)).sum() + out["depth"].sum() + 0.5 * out["uncertainty"].sum()
    loss.backward()
    dimg = dict(color=tc.astype(np.float64), depth=np.ones(td.shape), uncertainty=0.5 * np.ones(td.shape))
    ref = oracle.backward(sc, cam, identity_pose(), td, dimg)
    for k in PARAMS:
        assert rel_l2(scd[k].grad.cpu().numpy(), ref[k]) <= 1e-3, k
    assert np.abs(xi.grad.cpu().numpy() - ref["pose"]).max() <= 1e-3 * np.abs(ref["pose"]).max()


def test_fused_tracking_step_matches_separate_calls(R):
    """cgsr_tracking_step (loss gradient formed inside the blend, pose-only
    backward, Adam) equals render -> tracking_loss_grad -> backward -> Adam."""
    say("case: fused tracking step vs separate calls, 2 frames")
    sc = synth.room_scene(4, 30_000, (5.0, 4.0, 3.0))
    cams = [synth.camera(320, 240, 262.5, 262.5, 160, 120), synth.camera(160, 128, 131.25, 131.25, 80, 64)]
    scd = dev(sc)
    tgt_poses = [synth.level_room_pose(s) for s in (21, 22)]
    st = R.State()
    P_t = torch.stack([R.pose_tensor(*p) for p in tgt_poses])
    tg = R.render(st, scd, P_t, cams)
    tc = [t["color"].clone() for t in tg]
    td = [t["depth"].clone() for t in tg]
    P0 = torch.stack([R.pose_tensor(*synth.perturb_pose(*p, 30 + k)) for k, p in enumerate(tgt_poses)])
    # separate calls
    Ps, adam_s = P0.clone(), torch.zeros((2, 16), device="cuda")
    losses_sep = []
    for it in range(3):
        outs = R.render(st, scd, Ps, cams, maps=("color", "depth"))
        dimgs, Ls = [], []
        for v in range(2):
            L = torch.zeros(1, device="cuda")
            dc, dd = R.tracking_loss_grad(outs[v]["color"], outs[v]["depth"], tc[v], td[v], loss=L)
            dimgs.append(dict(color=dc, depth=dd))
            Ls.append(L.item())
        _, dp = R.backward(st, dimgs, param_grads=False)
        R.pose_adam_step(Ps, dp, adam_s)
        losses_sep.append(Ls)
    # fused
    Pf, adam_f = P0.clone(), torch.zeros((2, 16), device="cuda")
    losses_fused = []
    for it in range(3):
        L = torch.zeros(2, device="cuda")
        R.tracking_step(st, scd, Pf, cams, tc, td, adam=adam_f, loss=L)
        losses_fused.append(L.cpu().tolist())
    torch.cuda.synchronize()
    say("losses separate", losses_sep, "fused", losses_fused)
    np.testing.assert_allclose(np.array(losses_fused), np.array(losses_sep), rtol=2e-5)
    assert (Pf - Ps).abs().max().item() < 1e-5
    # the gradient alone (no Adam) equals the separate backward
    dposes = torch.zeros((2, 6), device="cuda")
    R.tracking_step(st, scd, P0, cams, tc, td, dposes=dposes)
    outs = R.render(st, scd, P0, cams, maps=("color", "depth"))
    dimgs = [dict(zip(("color", "depth"), R.tracking_loss_grad(outs[v]["color"], outs[v]["depth"], tc[v], td[v])))
             for v in range(2)]
    _, dp = R.backward(st, dimgs, param_grads=False)
    e = ((dposes - dp).abs().max() / dp.abs().max()).item()
    say("fused vs separate pose gradient", e)
    assert e < 1e-4


def test_tracking_step_without_work_counts(R):
    """count_work = 0 (the fused step keeps only colour, depth, transmittance
    and the last blended entry per pixel) gives the same losses, poses and
    pose gradients as the counting kernel; its statistics report the work
    counts as unknown (-1).  Buckets of at most one key per thread are sorted
    inside the fused kernel, larger ones by the segmented sort: both give the
    same steps."""
    say("case: tracking step with and without work counts, 2 frames")
    sc = synth.room_scene(5, 30_000, (5.0, 4.0, 3.0))
    cams = [synth.camera(320, 240, 262.5, 262.5, 160, 120), synth.camera(160, 128, 131.25, 131.25, 80, 64)]
    scd = dev(sc)
    tgt_poses = [synth.level_room_pose(s) for s in (23, 24)]
    ref = R.State()
    P_t = torch.stack([R.pose_tensor(*p) for p in tgt_poses])
    tg = R.render(ref, scd, P_t, cams)
    tc = [t["color"].clone() for t in tg]
    td = [t["depth"].clone() for t in tg]
    P0 = torch.stack([R.pose_tensor(*synth.perturb_pose(*p, 40 + k)) for k, p in enumerate(tgt_poses)])
    out = {}
    for count, big in ((True, False), (False, False), (False, True)):
        st = R.State(count_work=count)
        if big:
            st.reserve(tile_pairs=600)   # more than the 256 threads of a tile's workgroup
        P, adam = P0.clone(), torch.zeros((2, 16), device="cuda")
        losses = []
        for it in range(3):
            L = torch.zeros(2, device="cuda")
            R.tracking_step(st, scd, P, cams, tc, td, adam=adam, loss=L)
            losses.append(L.cpu().tolist())
        dposes = torch.zeros((2, 6), device="cuda")
        R.tracking_step(st, scd, P0, cams, tc, td, dposes=dposes)
        stats = st.stats()
        assert (stats.pair_capacity > 256) == big
        out[(count, big)] = (np.array(losses), P.cpu(), dposes.cpu(), stats)
    (l1, p1, d1, s1), (l0, p0, d0, s0) = out[(True, False)], out[(False, False)]
    lb, pb, db, sb = out[(False, True)]
    # the per-record gradient sums are float atomics (order-dependent rounding),
    # so later iterations' poses and losses differ from run to run at rounding level
    np.testing.assert_allclose(lb, l1, rtol=1e-5)
    assert (pb - p1).abs().max().item() < 1e-6
    assert ((db - d1).abs().max() / d1.abs().max()).item() < 1e-5
    assert sb.pairs == s1.pairs
    np.testing.assert_allclose(l0, l1, rtol=1e-5)
    assert (p0 - p1).abs().max().item() < 1e-6
    e = ((d0 - d1).abs().max() / d1.abs().max()).item()
    say("pose gradient, without vs with counts", e)
    assert e < 1e-5
    assert s1.processed > 0 and s1.blended > 0 and s1.walked > 0
    assert s0.processed == -1 and s0.blended == -1 and s0.walked == -1
    assert s0.visible == s1.visible and s0.pairs == s1.pairs and s0.peak_pairs == s1.peak_pairs


def test_render_without_work_counts(R, config1):
    """A render with count_work = 0 writes the same maps and leaves the same
    backward as one with the counts; its statistics report them as -1."""
    sc, cam, tc, td = config1
    say("case: config1 render and backward without work counts")
    scd = dev(sc)
    outs, grads = {}, {}
    rng = np.random.default_rng(31)
    H, W = cam["height"], cam["width"]
    dimg = dict(color=rng.standard_normal((3, H, W)), depth=rng.standard_normal((H, W)),
                opacity=rng.standard_normal((H, W)), depth_median=rng.standard_normal((H, W)),
                uncertainty=rng.standard_normal((H, W)))
    for count in (True, False):
        st = R.State(count_work=count)
        outs[count], _ = gpu_render(R, st, scd, identity_pose(), cam, td)
        s = st.stats()
        assert (s.processed > 0) == count and (s.processed == -1) == (not count)
        grads[count] = R.backward(st, [{k: t32(v) for k, v in dimg.items()}])
    for k in MAPS:
        assert np.array_equal(outs[True][k], outs[False][k]), k
    for k in PARAMS:
        a, b = grads[True][0][k].cpu().numpy(), grads[False][0][k].cpu().numpy()
        assert rel_l2(b, a) <= 1e-6, k
    d1, d0 = grads[True][1][0].cpu().numpy(), grads[False][1][0].cpu().numpy()
    assert np.abs(d0 - d1).max() <= 1e-5 * np.abs(d1).max()


def test_tracking_step_bucket_capacity(R):
    """The fused tracking step (which sorts its own tile buckets when they
    hold at most one key per thread) with buckets exactly as large as the
    fullest tile gives the gradient it gives with roomy ones; with smaller
    buckets the dropped pairs are reported: the statistics give the count
    the fullest tile needed and the next check raises the capacity error."""
    from paper_2403_16095_amd import binding as B
    say("case: tracking step bucket capacity, 40k Gaussians 320x240")
    sc = synth.room_scene(6, 40_000, (5.0, 4.0, 3.0))
    cam = synth.camera(320, 240, 262.5, 262.5, 160, 120)
    scd = dev(sc)
    tgt = synth.level_room_pose(25)
    ref_st = R.State()
    tg = R.render(ref_st, scd, R.pose_tensor(*tgt).reshape(1, 12), [cam])[0]
    tc, td = tg["color"].clone(), tg["depth"].clone()
    P0 = R.pose_tensor(*synth.perturb_pose(*tgt, 50)).reshape(1, 12)

    def step(st):
        d = torch.zeros((1, 6), device="cuda")
        R.tracking_step(st, scd, P0, [cam], [tc], [td], dposes=d)
        torch.cuda.synchronize()
        return d

    roomy = R.State(sync_capacity=False)
    roomy.reserve(tile_pairs=256)
    d_ref = step(roomy)
    peak = roomy.stats().peak_pairs
    roomy.check()
    say("fullest tile", peak)
    assert 64 < peak <= 256, "the case needs a fullest tile between the smallest bucket and 256 pairs"
    exact = R.State(sync_capacity=False)
    exact.reserve(tile_pairs=peak)
    d_ex = step(exact)
    assert exact.stats().pair_capacity == peak
    exact.check()
    assert ((d_ex - d_ref).abs().max() / d_ref.abs().max()).item() < 1e-5
    small = R.State(sync_capacity=False)
    small.reserve(tile_pairs=max(64, peak // 2))
    step(small)
    s = small.stats()
    assert s.overflow == 1 and s.peak_pairs == peak
    with pytest.raises(B.CgsrError) as e:
        small.check()
    assert e.value.status == B.CGSR_ERR_CAPACITY


def test_graph_tracking_replays_match_eager(R):
    """The captured 50-iteration tracking solve replayed several times, with
    eager work in between, matches the same loop run eagerly."""
    say("case: hipGraph tracking solve vs eager")
    sc = synth.room_scene(3, 30_000, (5.0, 4.0, 3.0))
    cam = synth.camera(320, 240, 262.5, 262.5, 160, 120)
    Rt, tt = synth.level_room_pose(11)
    scd = dev(sc)
    st = R.State()
    tgt = R.render(st, scd, R.pose_tensor(Rt, tt), [cam])[0]
    prob = R.TrackingProblem(scd, cam, tgt["color"].clone(), tgt["depth"].clone())
    P0 = R.pose_tensor(*synth.perturb_pose(Rt, tt, 5))
    eager = R.TrackingSolver(prob, iters=50, use_graph=False)
    eager.prepare(P0)
    eager.run()
    torch.cuda.synchronize()
    ref = eager.pose.clone()
    graph = R.TrackingSolver(prob, iters=50, use_graph=True)
    graph.prepare(P0)
    for rep in range(3):
        graph.reset(P0)
        graph.run()
        torch.cuda.synchronize()
        _ = (torch.randn(1000, device="cuda") * 2).sum().item()   # unrelated eager work between replays
        graph.check()
        d = (graph.pose - ref).abs().max().item()
        say("replay", rep, "max |pose - eager|", d)
        assert d < 1e-4
    # the solve lowered the tracking loss (Eq. 19) and moved the camera centre
    # toward the true one
    def loss_at(P):
        out = R.render(R.State(), scd, P, [cam])[0]
        L = torch.zeros(1, device="cuda")
        R.tracking_loss_grad(out["color"], out["depth"], prob.target_color, prob.target_depth, loss=L)
        return L.item()

    def centre(P):
        p = P.double().cpu().numpy()
        return -p[:9].reshape(3, 3).T @ p[9:]

    c_true = -np.asarray(Rt).T @ np.asarray(tt)
    l0, l1 = loss_at(P0), loss_at(ref)
    e0, e1 = np.abs(centre(P0) - c_true).max(), np.abs(centre(ref) - c_true).max()
    say("loss before/after", l0, l1, "centre error before/after", e0, e1)
    assert l1 < 0.5 * l0 and e1 < e0


def test_kept_tile_order_across_tile_counts_and_captures(R):
    """A fused tracking step on a frame that fits the chip orders its tiles by
    the lengths the previous step left (every eager step, and the first step
    of each graph capture); steps of another tile count and renders that write
    their own order in between, eager and between replays of a captured solve
    fragment, leave the pose gradients those of a fresh state."""
    say("case: kept tile order, eager and captured, changing tile counts")
    sc = synth.room_scene(6, 30_000, (5.0, 4.0, 3.0))
    scd = dev(sc)
    cam_a = synth.camera(320, 240, 262.5, 262.5, 160, 120)   # 300 tiles
    cam_b = synth.camera(160, 128, 131.25, 131.25, 80, 64)    # 80 tiles
    cam_c = synth.camera(480, 320, 393.75, 393.75, 240, 160)  # 600 tiles, rendered without fusion
    pa, pb = synth.level_room_pose(31), synth.level_room_pose(32)
    Pa, Pb = R.pose_tensor(*pa), R.pose_tensor(*pb)
    ref_st = R.State()
    tgt = {}
    for name, cam, P in (("a", cam_a, Pa), ("b", cam_b, Pb)):
        out = R.render(ref_st, scd, P, [cam])[0]
        tgt[name] = (out["color"].clone(), out["depth"].clone())
    Pa0 = R.pose_tensor(*synth.perturb_pose(*pa, 41))
    Pb0 = R.pose_tensor(*synth.perturb_pose(*pb, 42))
    cams = {"a": (cam_a, Pa0), "b": (cam_b, Pb0)}

    def step(st, name, dp):
        cam, P0 = cams[name]
        R.tracking_step(st, scd, P0, [cam], [tgt[name][0]], [tgt[name][1]], dposes=dp)

    ref = {}
    for name in cams:
        dp = torch.zeros((1, 6), device="cuda")
        step(R.State(), name, dp)
        ref[name] = dp.clone()

    def check(dp, name, label):
        e = ((dp - ref[name]).abs().max() / ref[name].abs().max()).item()
        say(label, name, "pose gradient vs fresh state", e)
        assert e < 1e-4, (label, name, e)

    def eager(st, name, label):
        dp = torch.zeros((1, 6), device="cuda")
        step(st, name, dp)
        check(dp, name, label)

    st = R.State()
    for name in ("a", "b", "c", "a", "b", "a"):
        if name == "c":
            R.render(st, scd, Pa, [cam_c])   # writes an order of its own tile count
        else:
            eager(st, name, "eager")
    st.check()
    # a captured fragment of two steps on frame a, taken right after an eager
    # step on the same frame (the capture still computes its own order)
    dps = [torch.zeros((1, 6), device="cuda") for _ in range(2)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        for dp in dps:
            dp.zero_()
            step(st, "a", dp)
    torch.cuda.synchronize()
    for rep in range(3):
        eager(st, "b", f"between replays {rep}")
        R.render(st, scd, Pa, [cam_c])
        # a graph reads the camera table the state holds when it replays:
        # an eager call on its frame first
        eager(st, "a", f"between replays {rep}")
        graph.replay()
        torch.cuda.synchronize()
        st.check()
        for dp in dps:
            check(dp, "a", f"replay {rep}")


@pytest.mark.parametrize("width,height", [(640, 512), (800, 480)])
def test_kept_tile_order_at_full_runs_and_a_long_last_run(R, width, height):
    """The kept order's edge shapes: 1280 tiles fill five runs of 256 (no last
    run to place by load), 1500 leave a last run of 220 positions (ranked four
    lanes to a position).  Steps that take the order (and its quadrant
    rotations) from the previous step's measured work, eager and replayed from
    a captured solve fragment, give the pose gradient and loss of a fresh
    state's step."""
    tiles = (width // 16) * (height // 16)
    say("case: kept tile order,", width, "x", height, "=", tiles, "tiles, last run", tiles % 256)
    sc = synth.room_scene(8, 30_000, (5.0, 4.0, 3.0))
    scd = dev(sc)
    cam = synth.camera(width, height, 0.82 * width, 0.82 * width, width / 2, height / 2)
    pose = synth.level_room_pose(71)
    out = R.render(R.State(), scd, R.pose_tensor(*pose), [cam])[0]
    tc, td = out["color"].clone(), out["depth"].clone()
    P0 = R.pose_tensor(*synth.perturb_pose(*pose, 72))

    def step(st, dp, loss):
        R.tracking_step(st, scd, P0, [cam], [tc], [td], dposes=dp, loss=loss)

    ref, ref_loss = torch.zeros((1, 6), device="cuda"), torch.zeros(1, device="cuda")
    step(R.State(), ref, ref_loss)
    torch.cuda.synchronize()

    def check(dp, loss, label):
        e = ((dp - ref).abs().max() / ref.abs().max()).item()
        el = abs(loss.item() - ref_loss.item()) / abs(ref_loss.item())
        say(label, "pose gradient vs fresh state", e, "loss", el)
        assert e < 1e-4 and el < 1e-5, (label, e, el)

    st = R.State()
    for k in range(3):   # the second and third take the order the one before measured
        dp, loss = torch.zeros((1, 6), device="cuda"), torch.zeros(1, device="cuda")
        step(st, dp, loss)
        torch.cuda.synchronize()
        st.check()
        check(dp, loss, f"eager step {k}")
    cap = int(st.stats().pair_capacity)
    say("bucket capacity", cap)
    assert cap <= 256, "the fused kernel ranks its own bucket, so the step keeps its order"
    dps = [torch.zeros((1, 6), device="cuda") for _ in range(2)]
    losses = [torch.zeros(1, device="cuda") for _ in range(2)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        for dp, loss in zip(dps, losses):
            dp.zero_()
            loss.zero_()
            step(st, dp, loss)
    torch.cuda.synchronize()
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        st.check()
        for dp, loss in zip(dps, losses):
            check(dp, loss, f"replay {rep}")


def _tile_order(R, st):
    """(tile of each position, quadrant rotations, kept) of the last render."""
    from paper_2403_16095_amd import binding as B
    ptr, tiles, kept = B.cgsr_debug_tile_order(st.handle)
    if ptr is None:
        return None, None, kept
    buf = torch.empty(tiles, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    copy_device(buf, ptr, tiles * 4)
    e = buf.cpu().numpy().view(np.uint32).astype(np.int64)
    return e & 0x3FFFFFFF, e >> 30, kept


def _tile_lengths(R, st, tiles):
    from paper_2403_16095_amd import binding as B
    _, _, ranges, _, _ = B.cgsr_debug_buffers(st.handle)
    rg = torch.empty((tiles, 2), dtype=torch.int32, device="cuda")
    copy_device(rg, ranges, tiles * 8)
    rg = rg.cpu().numpy().astype(np.int64)
    return rg[:, 1] - rg[:, 0]


def _order_bin(n):
    """The order kernels' length bins: the leading bit and the next four."""
    out = []
    for x in np.asarray(n, np.int64).tolist():
        lead = x.bit_length() - 1
        frac = (x >> (lead - 4) if lead >= 4 else x << (4 - lead)) & 15
        out.append(0 if x == 0 else 1 + 16 * lead + frac)
    return np.array(out, np.int64)


def test_tile_orders_are_permutations_longest_first(R):
    """The order kernels' own output: a render's order (from the sorted
    ranges) and a fused step's order at 3225 tiles (from the pair counters)
    take every tile once, with non-increasing length bins; the order a fused
    step keeps at 1200 tiles takes every tile once and gives each workgroup a
    quadrant rotation; a launch of more tiles than the order kernels take
    (11 views, 35 475 tiles) has no order, and the debug view says so."""
    say("case: tile orders of renders and fused tracking steps")
    sc = synth.room_scene(0, 100_000, (5.0, 4.0, 3.0))
    scd = {k: torch.from_numpy(np.ascontiguousarray(v, np.float32)).cuda() for k, v in sc.items()}
    true = synth.level_room_pose(0)
    P = R.pose_tensor(*synth.perturb_pose(*true, 1000)).reshape(1, 12)
    for cam, fused in ((synth.MAPPING_CAMERA, False), (synth.MAPPING_CAMERA, True),
                       (synth.TRACKING_CAMERA, True)):
        tiles = ((cam["width"] + 15) // 16) * ((cam["height"] + 15) // 16)
        st = R.State(count_work=False)
        tgt = R.render(R.State(), scd, R.pose_tensor(*true), [cam])[0]
        tc, td = tgt["color"].contiguous(), tgt["depth"].contiguous()
        if fused:
            d = torch.zeros((1, 6), device="cuda")
            R.tracking_step(st, scd, P.clone(), [cam], [tc], [td], dposes=d)
            torch.cuda.synchronize()
            st.reserve(tile_pairs=int(st.stats().peak_pairs * 1.5) + 64)
            for _ in range(2):   # the second step keeps the order the first measured
                R.tracking_step(st, scd, P.clone(), [cam], [tc], [td], dposes=d)
        else:
            R.render(st, scd, P, [cam])
        torch.cuda.synchronize()
        st.check()
        order, rot, kept = _tile_order(R, st)
        say(cam["width"], "x", cam["height"], "fused" if fused else "render", tiles, "tiles, kept", kept)
        assert order is not None
        assert np.array_equal(np.sort(order), np.arange(tiles)), "every tile exactly once"
        if kept:
            assert tiles < 1536 and fused
            assert rot.min() >= 0 and rot.max() <= 3 and len(np.unique(rot)) > 1, "rotations in use"
        else:
            assert (rot == 0).all()
            bins = _order_bin(_tile_lengths(R, st, tiles)[order])
            assert (np.diff(bins) <= 0).all(), "longest list first"
    st = R.State(count_work=False)
    views = 11
    R.render(st, scd, P.repeat(views, 1), [synth.MAPPING_CAMERA] * views, maps=("color",))
    torch.cuda.synchronize()
    st.check()
    order, _, kept = _tile_order(R, st)
    say(views, "views: order", order, "kept", kept)
    assert order is None and kept == 0


def test_replay_with_another_camera_table_is_reported(R):
    """A captured tracking step replayed after an eager call with another
    (smaller) camera on the same state runs with that call's camera table:
    cgsr_state_check reports it (CGSR_ERR_STATE) and clears the flag, and a
    replay after a call with the graph's own camera is correct again."""
    from paper_2403_16095_amd import binding as B
    say("case: graph replay with a rewritten camera table")
    sc = synth.room_scene(7, 20_000, (5.0, 4.0, 3.0))
    scd = dev(sc)
    cam_a = synth.camera(320, 240, 262.5, 262.5, 160, 120)
    cam_b = synth.camera(160, 128, 131.25, 131.25, 80, 64)
    pa, pb = synth.level_room_pose(51), synth.level_room_pose(52)
    tgt = {}
    for name, cam, pose in (("a", cam_a, pa), ("b", cam_b, pb)):
        out = R.render(R.State(), scd, R.pose_tensor(*pose), [cam])[0]
        tgt[name] = (cam, R.pose_tensor(*synth.perturb_pose(*pose, 61)), out["color"].clone(), out["depth"].clone())

    def step(st, name, dp):
        cam, P0, tc, td = tgt[name]
        R.tracking_step(st, scd, P0, [cam], [tc], [td], dposes=dp)

    ref = torch.zeros((1, 6), device="cuda")
    step(R.State(), "a", ref)
    st = R.State()
    scratch = torch.zeros((1, 6), device="cuda")
    for name in ("b", "a"):   # size the state for both frames, then leave frame a's table
        step(st, name, scratch)
    st.check()
    dp = torch.zeros((1, 6), device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        dp.zero_()
        step(st, "a", dp)
    torch.cuda.synchronize()

    def replay_matches():
        graph.replay()
        torch.cuda.synchronize()
        st.check()
        e = ((dp - ref).abs().max() / ref.abs().max()).item()
        say("replay pose gradient vs fresh state", e)
        assert e < 1e-4

    replay_matches()
    step(st, "b", scratch)   # rewrites the table
    graph.replay()
    torch.cuda.synchronize()
    with pytest.raises(B.CgsrError) as err:
        st.check()
    assert err.value.status == B.CGSR_ERR_STATE
    st.check()               # the flag was cleared
    step(st, "a", scratch)   # the graph's own camera again
    replay_matches()


def test_wave_lists_within_8x8_binning(R):
    """Each wave walks the Gaussians whose binning rectangle reaches its 8x8
    cell, less those that cannot reach alpha >= 1/255 on the cell: on a scene
    where no pixel reaches the stop threshold, every pixel's alpha evaluations
    lie between the number of its cell's Gaussians that reach alpha >= 1/255
    at some pixel of the cell (FP64, from the oracle's projection) and the
    length of its cell's list under 8x8 binning by enumeration (the oracle's
    tile lists with tile = 8); some cells are shortened, and the forward
    still matches the oracle."""
    say("case: per-wave 8x8 lists, 3000 faint Gaussians 64x48 and 200x120")
    from paper_2403_16095_amd import binding as B
    for cam in (synth.SMALL_CAMERA, synth.camera(200, 120, 150.0, 150.0, 100.0, 60.0)):
        sc = synth.uniform_box_scene(5, 3000, opacity=(-4.0, 0.5))
        st = R.State()
        gpu, _ = gpu_render(R, st, dev(sc), identity_pose(), cam)
        ref = oracle.render(sc, cam, identity_pose())
        assert ref["t_final"].min() > 1e-3, "no pixel may stop"
        check_maps(gpu, sc, cam, identity_pose(), ref=ref, max_ambiguous=0.01, label="faint")
        H, W = cam["height"], cam["width"]
        proj = oracle.project(sc, cam, identity_pose())
        lists = oracle.tile_lists(proj, cam, tile=8)
        cells_x = (W + 7) // 8
        expect = np.zeros((H, W), np.int64)
        needed = np.zeros((H, W), np.int64)
        for cell, ids in lists.items():
            cy, cx = divmod(cell, cells_x)
            ys, xs = np.arange(8 * cy, min(8 * cy + 8, H)), np.arange(8 * cx, min(8 * cx + 8, W))
            X, Y = np.meshgrid(xs, ys)
            n_need = 0
            for i in ids:
                a, b, c = proj["conic"][i]
                dx, dy = X - proj["mu"][i][0], Y - proj["mu"][i][1]
                alpha = proj["opacity"][i] * np.exp(-0.5 * (a * dx * dx + 2 * b * dx * dy + c * dy * dy))
                n_need += bool((alpha >= 1.0 / 255.0).any())
            expect[np.ix_(ys, xs)] = len(ids)
            needed[np.ix_(ys, xs)] = n_need
        keys, vals, ranges, recs, pst = B.cgsr_debug_buffers(st.handle)
        ps = torch.empty((H * W, 4), dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        copy_device(ps, pst, H * W * 16)
        got = ps[:, 3].cpu().numpy().reshape(H, W)
        say("entries walked", int(got.sum()), "8x8 binning", int(expect.sum()), "needed", int(needed.sum()))
        assert (got <= expect).all() and (got >= needed).all()
        assert got.sum() < expect.sum()
        assert expect.max() > 10
