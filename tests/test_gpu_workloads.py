"""HIP path vs the FP64 oracle at the mapping and batched workload sizes.

Mapping: 500k Gaussians in an 8x6x3 m room, 1200x680 (f = 600), every map
and every parameter gradient of the uncertainty-weighted mapping loss.
Batched mapping: 1M Gaussians, 8 keyframe views along a random walk, one
launch sequence vs 8 single-view ones, sampled pixels vs the oracle.
Batched tracking: 1M Gaussians, 32 frames of uneven resolution in one
launch sequence, per-frame pose gradients vs the oracle's analytic
backward and (one frame) its frozen-decision central differences, and a 20-step
graph-captured Adam loop vs the same loop run eagerly.
Tolerances, and the admissible results of near-threshold pixels, are those
of test_gpu_parity.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2403_16095_amd import synth
from helpers import check_maps, grad_parity, rel_l2

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


def to_np(out):
    return {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}


def test_mapping_size_all_maps_and_gradients(R):
    say("case: mapping 500k Gaussians, 1200x680, full backward of the uncertainty-weighted loss")
    sc = synth.room_scene(0, 500_000, (8.0, 6.0, 3.0))
    cam = synth.MAPPING_CAMERA
    pose = synth.level_room_pose(0)
    tc, td = synth.random_targets(1003, cam, depth_range=(0.5, 5.0))
    scd = dev(sc)
    st = R.State()
    P = R.pose_tensor(*pose)
    out = R.render(st, scd, P, [cam], [t32(td)])[0]
    gpu = to_np(out)
    ref = oracle.render(sc, cam, pose, td)
    check_maps(gpu, sc, cam, pose, td, ref=ref, max_ambiguous=0.06, label="mapping 1200x680")
    # the device mapping-loss kernel against the oracle's loss on the same
    # seeded synthetic maps
    rng = np.random.default_rng(77)
    H, W = cam["height"], cam["width"]
    syn = dict(color=rng.random((3, H, W)).astype(np.float32), depth=rng.uniform(0.5, 5, (H, W)).astype(np.float32),
               uncertainty=rng.uniform(0, 0.3, (H, W)).astype(np.float32))
    L = torch.zeros(1, device="cuda")
    dimg_d = R.mapping_loss_grad(t32(syn["color"]), t32(syn["depth"]), t32(syn["uncertainty"]), t32(tc), t32(td),
                                 loss=L)
    Lr, dimg_r = oracle.uncertainty_weighted_loss({k: v.astype(np.float64) for k, v in syn.items()}, tc, td)
    assert abs(L.item() - Lr) <= 1e-4 * abs(Lr)
    for k in ("color", "depth", "uncertainty"):
        np.testing.assert_allclose(dimg_d[k].cpu().numpy(), dimg_r[k], rtol=1e-5, atol=1e-12)
    # backward from identical upstream gradients
    _, dimg = oracle.uncertainty_weighted_loss(ref, tc, td)
    grads, dposes = R.backward(st, [{k: t32(v) for k, v in dimg.items()}])
    rb = oracle.backward(sc, cam, pose, td, dimg)
    for k in PARAMS:
        grad_parity(k, grads[k].cpu().numpy(), rb[k], label="mapping 1200x680")
    e = np.abs(dposes[0].cpu().numpy() - rb["pose"]).max() / np.abs(rb["pose"]).max()
    say("pose rel err", e)
    assert e <= 1e-3


def test_batched_mapping_8_views_full_size(R):
    say("case: 1M Gaussians, 8 keyframe views 1200x680 in one launch sequence")
    sc = synth.room_scene(1, 1_000_000, (8.0, 6.0, 3.0))
    cam = synth.MAPPING_CAMERA
    poses = synth.random_walk_poses(7, 8)
    scd = dev(sc)
    P = torch.stack([R.pose_tensor(*p) for p in poses])
    st = R.State()
    outs = R.render(st, scd, P, [cam] * 8)
    outs = [{k: v.clone() for k, v in o.items()} for o in outs]
    rng = np.random.default_rng(5)
    dimgs = [dict(color=t32(rng.standard_normal((3, cam["height"], cam["width"])) * 1e-6),
                  depth=t32(rng.standard_normal((cam["height"], cam["width"])) * 1e-6)) for _ in range(8)]
    gb, pb = R.backward(st, dimgs)
    acc = {k: torch.zeros_like(v) for k, v in gb.items()}
    s1 = R.State()
    for v in range(8):
        single = R.render(s1, scd, P[v].contiguous(), [cam])[0]
        for k in ("color", "depth", "opacity", "depth_median"):
            assert torch.equal(single[k], outs[v][k]), (v, k)
        g1, p1 = R.backward(s1, [dimgs[v]])
        for k in acc:
            acc[k] += g1[k]
        e = ((p1[0] - pb[v]).abs().max() / p1[0].abs().max()).item()
        assert e < 1e-4, (v, e)
    for k in acc:
        e = rel_l2(gb[k].cpu().numpy(), acc[k].cpu().numpy())
        say(k, "batched vs sum of views", e)
        assert e < 1e-4, k
    # sampled pixels of two views against the oracle
    for v in (0, 5):
        px = rng.choice(cam["width"] * cam["height"], 1500, replace=False)
        gpu = {k: outs[v][k].cpu().numpy().astype(np.float64) for k in ("color", "depth", "opacity", "depth_median")}
        check_maps(gpu, sc, cam, poses[v], None, px=px, max_ambiguous=0.15, label=f"batched mapping view {v}")


def test_batched_tracking_32_frames(R):
    say("case: 1M Gaussians, 32 frames of uneven resolution, one tracking launch sequence")
    sc = synth.room_scene(2, 1_000_000, (8.0, 6.0, 3.0))
    frames = synth.tracking_frames(11, 32)
    cams = [f[0] for f in frames]
    true = [f[1] for f in frames]
    scd = dev(sc)
    st = R.State()
    Pt = torch.stack([R.pose_tensor(*p) for p in true])
    tg = R.render(st, scd, Pt, cams, maps=("color", "depth"))
    tc = [t["color"].clone() for t in tg]
    td = [t["depth"].clone() for t in tg]
    start = [synth.perturb_pose(*p, 100 + k) for k, p in enumerate(true)]
    P0 = torch.stack([R.pose_tensor(*p) for p in start])
    dposes = torch.zeros((32, 6), device="cuda")
    R.tracking_step(st, scd, P0, cams, tc, td, dposes=dposes)
    # per-frame pose gradients against the oracle (a few frames) and against
    # single-frame steps (all frames)
    s1 = R.State()
    for v in range(32):
        d1 = torch.zeros((1, 6), device="cuda")
        R.tracking_step(s1, scd, P0[v].contiguous(), [cams[v]], [tc[v]], [td[v]], dposes=d1)
        e = ((d1[0] - dposes[v]).abs().max() / d1.abs().max()).item()
        assert e < 1e-4, (v, e)
    # per-frame pose gradients against the oracle, both sides on the same
    # seeded random target images
    rt = [synth.random_targets(500 + k, cams[k], depth_range=(0.5, 5.0)) for k in range(32)]
    dposes_r = torch.zeros((32, 6), device="cuda")
    R.tracking_step(st, scd, P0, cams, [t32(c) for c, _ in rt], [t32(d) for _, d in rt], dposes=dposes_r)
    for v in (0, 7, 19):
        cam = cams[v]
        ref = oracle.render(sc, cam, start[v])
        _, dimg = oracle.tracking_loss(ref, rt[v][0], rt[v][1])
        rb = oracle.backward(sc, cam, start[v], None, dimg)
        e = np.abs(dposes_r[v].cpu().numpy() - rb["pose"]).max() / np.abs(rb["pose"]).max()
        say("frame", v, cam["width"], "x", cam["height"], "pose grad rel err", e)
        assert e <= 1e-3
    # one frame against frozen-decision central differences of the oracle
    v = next((k for k, c in enumerate(cams) if c["width"] == 320), 0)
    cam = cams[v]
    ref = oracle.render(sc, cam, start[v])
    _, dimg = oracle.tracking_loss(ref, rt[v][0], rt[v][1])
    fd = oracle.fd_linear(sc, cam, start[v], None, dimg, [("pose", 0, c) for c in range(6)])
    e = np.abs(dposes_r[v].cpu().numpy() - fd).max() / np.abs(fd).max()
    say("frame", v, cam["width"], "x", cam["height"], "pose grad vs frozen FD rel err", e)
    assert e <= 1e-3
    # 20-step Adam loop captured in one graph vs the same loop eagerly
    params = R.adam_params()
    Pe, ae = P0.clone(), torch.zeros((32, 16), device="cuda")
    for _ in range(20):
        R.tracking_step(st, scd, Pe, cams, tc, td, adam=ae, params=params)
    torch.cuda.synchronize()
    Pg, ag = P0.clone(), torch.zeros((32, 16), device="cuda")
    gst = R.State()
    R.tracking_step(gst, scd, Pg, cams, tc, td, adam=ag, params=params)   # sizes the workspace
    gst.reserve(tile_pairs=int(gst.stats().peak_pairs * 1.5))
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            for _ in range(20):
                R.tracking_step(gst, scd, Pg, cams, tc, td, adam=ag, params=params)
    torch.cuda.current_stream().wait_stream(side)
    Pg.copy_(P0)
    ag.zero_()
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    gst.check()
    d = (Pg - Pe).abs().max().item()
    say("graph vs eager 20-step poses max diff", d)
    assert d < 1e-4
    c_err0 = np.mean([np.abs(-np.asarray(s[0]).T @ s[1] + np.asarray(t[0]).T @ t[1]).max() for s, t in zip(start, true)])
    Pn = Pg.double().cpu().numpy()
    c_err1 = np.mean([np.abs(-Pn[k, :9].reshape(3, 3).T @ Pn[k, 9:] + np.asarray(true[k][0]).T @ true[k][1]).max()
                      for k in range(32)])
    say("mean camera-centre error before/after", c_err0, c_err1)
    assert c_err1 < c_err0
