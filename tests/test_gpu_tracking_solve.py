"""The benchmarked tracking iteration against the FP64 oracle, in the
benchmark's workload and launch configuration.

Workload: 100k Gaussians on the walls of a 5 x 4 x 3 m room, 640x480
(f = 525), target colour and depth rendered (by the oracle) at the true
pose, start pose perturbed by N(0, 2 cm) and 1 degree; loss Eq. 19 with
lambda = (0.2, 1.0); Adam on the pose tangent (Sec. 4 learning rates) with
the left retraction (Eq. 20).

Launch configuration: TrackingSolver as the benchmark builds it -- the fused
tracking kernel without work counts, tile buckets sized from an eager step
(x1.5 + 64), so at one pixel per lane every bucket holds at most one key per
thread and the kernel ranks its own bucket (no sort launch), iterations
captured into one HIP graph and replayed.  Pixels per lane 1, 2 and 4.

Checks: the loss of the first iteration within 1e-5 relative of the oracle's
(plus the largest change the admissible results of near-threshold pixels
could make), the pose gradient within 1e-3 of its infinity norm, and the pose
after 5 graph-replayed Adam steps against the oracle's own 5-step solve.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2403_16095_amd import synth
from helpers import DECISION_MARGIN, ORDER_MARGIN, unambiguous

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

STEPS = 5
LAM = (0.2, 1.0)
LR = np.array([0.00215] * 3 + [0.0015] * 3)   # (rho, phi): translation, rotation


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_16095_amd import rasterizer
    return rasterizer


def pixel_loss(color, depth, tc, td):
    """Per-pixel summand of Eq. 19 times H*W."""
    return LAM[0] * np.abs(color - tc).sum(0) + LAM[1] * np.abs(depth - td)


@pytest.fixture(scope="module")
def solve():
    """The oracle's 5-step solve, with what the checks need of its first step."""
    sc = synth.room_scene(0, 100_000, (5.0, 4.0, 3.0))
    cam = synth.TRACKING_CAMERA
    true = synth.level_room_pose(0)
    start = synth.perturb_pose(*true, 1000)
    tgt = oracle.render(sc, cam, true)
    tc, td = tgt["color"].astype(np.float32), tgt["depth"].astype(np.float32)
    H, W = cam["height"], cam["width"]
    pose = (np.asarray(start[0], np.float64), np.asarray(start[1], np.float64))
    m, v = np.zeros(6), np.zeros(6)
    poses, losses, grads = [pose], [], []
    for it in range(1, STEPS + 1):
        maps = oracle.render(sc, cam, pose)
        loss, dimg = oracle.tracking_loss(maps, tc, td, lam=LAM)
        g = oracle.backward(sc, cam, pose, None, dimg)["pose"]
        if it == 1:
            first = maps
        losses.append(loss)
        grads.append(g)
        xi, m, v = oracle.adam_step(np.zeros(6), g, m, v, it, LR)
        pose = oracle.retract(pose, xi)
        poses.append(pose)
    # the largest change of the first loss that the admissible results of
    # near-threshold pixels can make
    amb = np.nonzero(~unambiguous(first).reshape(-1))[0]
    alts, count = oracle.render_alternatives(sc, cam, start, None, amb, DECISION_MARGIN, ORDER_MARGIN)
    ref_px = pixel_loss(first["color"].reshape(3, -1)[:, amb], first["depth"].reshape(-1)[amb],
                        tc.reshape(3, -1)[:, amb], td.reshape(-1)[amb])
    alt_px = pixel_loss(np.moveaxis(alts[:, :, 0:3], 2, 0), alts[:, :, 3], tc.reshape(3, -1)[:, amb][:, :, None],
                        td.reshape(-1)[amb][:, None])
    valid = np.arange(alts.shape[1])[None, :] < np.minimum(count, alts.shape[1])[:, None]
    spread = np.where(valid, np.abs(alt_px - ref_px[:, None]), 0.0).max(1)
    assert (count <= alts.shape[1]).all(), "every ambiguous pixel's alternatives are listed"
    loss_slack = float(spread.sum()) / (H * W)
    say("oracle losses", losses, "ambiguous pixels", amb.size, "loss slack", loss_slack)
    return dict(scene=sc, cam=cam, true=true, start=start, tc=tc, td=td, poses=poses, losses=losses,
                grads=grads, loss_slack=loss_slack)


@pytest.mark.parametrize("ppl", [1, 2, 4])
def test_benchmarked_solve_matches_oracle(R, solve, ppl):
    say(f"case: benchmarked tracking solve, 100k room 640x480, {ppl} pixel(s) per lane")
    sc, cam = solve["scene"], solve["cam"]
    scd = {k: torch.from_numpy(np.ascontiguousarray(v, np.float32)).cuda() for k, v in sc.items()}
    tc = torch.from_numpy(solve["tc"]).cuda()
    td = torch.from_numpy(solve["td"]).cuda()
    prob = R.TrackingProblem(scd, cam, tc, td)
    assert tuple(prob.lam) == LAM and np.allclose([prob.lr_rho] * 3 + [prob.lr_phi] * 3, LR)
    P0 = R.pose_tensor(*solve["start"])
    solver = R.TrackingSolver(prob, iters=STEPS, use_graph=True, reset_pose=P0, fwd_ppl=ppl, bwd_ppl=ppl)
    solver.prepare(P0)
    st = solver.state
    assert st.settings.count_work == 0
    cap = int(st.stats().pair_capacity)
    say("bucket capacity", cap, "fullest tile", int(st.stats().peak_pairs))
    if ppl == 1:
        assert cap <= 256, "the benchmark's configuration: the fused kernel ranks its own bucket"
    # first iteration: loss and pose gradient from the same state, captured
    dpose = torch.zeros((1, 6), device="cuda")
    loss = torch.zeros(1, device="cuda")
    P = P0.clone().reshape(1, 12)
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            R.tracking_step(st, scd, P, [cam], [tc], [td], dposes=dpose, loss=loss)
    torch.cuda.current_stream().wait_stream(side)
    for rep in range(2):
        dpose.zero_()
        loss.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        st.check()
        L, g = float(loss.item()), dpose[0].double().cpu().numpy()
        Lr, gr = solve["losses"][0], solve["grads"][0]
        el = abs(L - Lr)
        eg = np.abs(g - gr).max() / np.abs(gr).max()
        say(f"replay {rep}: loss {L:.8f} oracle {Lr:.8f} |diff| {el:.3e} (bar {1e-5 * Lr + solve['loss_slack']:.3e});",
            "pose gradient rel err", eg)
        assert el <= 1e-5 * Lr + solve["loss_slack"]
        assert eg <= 1e-3
    # the 5-step solve, replayed from its graph
    for rep in range(2):
        solver.run()
        torch.cuda.synchronize()
        solver.check()
        p = solver.pose.double().cpu().numpy()
        Rr, tr = solve["poses"][STEPS]
        dR, dt = np.abs(p[:9].reshape(3, 3) - Rr).max(), np.abs(p[9:] - tr).max()
        R0, t0 = solve["poses"][0]
        say(f"solve replay {rep}: |R - R_oracle| {dR:.3e}, |t - t_oracle| {dt:.3e} m "
            f"(the solve moved R by {np.abs(Rr - R0).max():.3e}, t by {np.abs(tr - t0).max():.3e} m)")
        assert dR <= 1e-5 and dt <= 1e-5


@pytest.mark.parametrize("ppl", [1, 4])
def test_blend_timing_reruns_leave_the_state_as_the_step_left_it(R, ppl):
    """cgsr_time_tracking_blend (how the benchmark times its dominant kernel)
    re-runs the last step's fused blend; a state that was timed then takes
    its next step exactly as one that was not (pose gradients equal up to the
    float atomics' order), with the kernel ranking its own buckets (ppl 1) or
    reading the segmented sort's lists (ppl 4)."""
    say(f"case: blend timing re-runs, 100k room 640x480, {ppl} pixel(s) per lane")
    sc = synth.room_scene(0, 100_000, (5.0, 4.0, 3.0))
    cam = synth.TRACKING_CAMERA
    true = synth.level_room_pose(0)
    scd = {k: torch.from_numpy(np.ascontiguousarray(v, np.float32)).cuda() for k, v in sc.items()}
    tgt = R.render(R.State(), scd, R.pose_tensor(*true), [cam])[0]
    tc, td = tgt["color"].contiguous(), tgt["depth"].contiguous()
    P1 = R.pose_tensor(*synth.perturb_pose(*true, 1000)).reshape(1, 12)
    P2 = R.pose_tensor(*synth.perturb_pose(*true, 1001)).reshape(1, 12)
    grads = []
    for timed in (False, True):
        st = R.State(sync_capacity=True, fwd_ppl=ppl, bwd_ppl=ppl, count_work=False)
        d = torch.zeros((1, 6), device="cuda")
        R.tracking_step(st, scd, P1.clone(), [cam], [tc], [td], dposes=d)
        torch.cuda.synchronize()
        st.reserve(tile_pairs=int(st.stats().peak_pairs * 1.5) + 64)
        cap = int(st.stats().pair_capacity)
        if ppl == 1:
            assert cap <= 256, "the kernel ranks its own buckets"
        else:
            assert cap > 256 // ppl, "the segmented sort orders the buckets"
        d.zero_()
        R.tracking_step(st, scd, P1.clone(), [cam], [tc], [td], dposes=d)
        g1 = d.clone()
        if timed:
            ms = [st.time_tracking_blend(reps) for reps in (1, 20)]
            say(f"blend re-run: {ms[0] * 1e3:.1f} us (1 launch), {ms[1] * 1e3:.1f} us (average of 20)")
            assert all(0.0 < m < 10.0 for m in ms)
        d.zero_()
        R.tracking_step(st, scd, P2.clone(), [cam], [tc], [td], dposes=d)
        torch.cuda.synchronize()
        st.check()
        grads.append((g1.double().cpu().numpy(), d.double().cpu().numpy()))
        if timed:
            R.render(st, scd, P2.clone(), [cam])
            with pytest.raises(R.B.CgsrError, match="not a tracking step"):
                st.time_tracking_blend(5)
    for a, b in zip(*grads):
        err = np.abs(a - b).max() / np.abs(a).max()
        say("pose gradient, timed state vs untimed:", err)
        assert err <= 1e-5


def test_ordered_fused_step_equals_separate_calls(R):
    """A 1200x680 tracking frame holds 3225 tiles, more than fit the chip at
    once, so the fused kernel (ranking its own buckets) takes its tiles
    longest list first, ordered from the pair counters before it runs.  Its
    loss and pose gradient equal those of render -> tracking_loss_grad ->
    backward (whose blends take the order from the sorted ranges), and the
    maps that render writes equal a render of a fresh state."""
    say("case: ordered fused tracking step, 100k room at 1200x680")
    sc = synth.room_scene(0, 100_000, (5.0, 4.0, 3.0))
    cam = synth.MAPPING_CAMERA
    true = synth.level_room_pose(0)
    scd = {k: torch.from_numpy(np.ascontiguousarray(v, np.float32)).cuda() for k, v in sc.items()}
    tgt = R.render(R.State(), scd, R.pose_tensor(*true), [cam])[0]
    tc, td = tgt["color"].contiguous(), tgt["depth"].contiguous()
    P = R.pose_tensor(*synth.perturb_pose(*true, 1000)).reshape(1, 12)
    st = R.State(sync_capacity=True, count_work=False)
    d = torch.zeros((1, 6), device="cuda")
    R.tracking_step(st, scd, P.clone(), [cam], [tc], [td], dposes=d)
    torch.cuda.synchronize()
    st.reserve(tile_pairs=int(st.stats().peak_pairs * 1.5) + 64)
    assert int(st.stats().pair_capacity) <= 256, "the fused kernel ranks its own buckets"
    tiles = ((cam["width"] + 15) // 16) * ((cam["height"] + 15) // 16)
    assert tiles >= 1536
    d.zero_()
    L = torch.zeros(1, device="cuda")
    R.tracking_step(st, scd, P.clone(), [cam], [tc], [td], dposes=d, loss=L)
    torch.cuda.synchronize()
    st.check()
    sep = R.State()
    out = R.render(sep, scd, P.clone(), [cam], maps=("color", "depth"))[0]
    L2 = torch.zeros(1, device="cuda")
    dc, dd = R.tracking_loss_grad(out["color"], out["depth"], tc, td, loss=L2)
    _, dp = R.backward(sep, [dict(color=dc, depth=dd)], param_grads=False)
    fresh = R.render(R.State(), scd, P.clone(), [cam], maps=("color", "depth"))[0]
    torch.cuda.synchronize()
    for k in ("color", "depth"):
        assert torch.equal(out[k], fresh[k]), k
    a, b = d[0].double().cpu().numpy(), dp[0].double().cpu().numpy()
    err = np.abs(a - b).max() / np.abs(b).max()
    say("loss fused", float(L), "separate", float(L2), "pose gradient rel diff", err)
    assert abs(float(L) - float(L2)) <= 1e-5 * abs(float(L2))
    assert err <= 1e-5
