"""HIP per-Gaussian depth uncertainty (Sec. 3.2, Eq. 13) and tau pruning vs
the FP64 oracle.

Which Gaussian dominates a pixel is decided by comparing float weights, so
per-pixel dominant maps are compared where every decision of the pixel is
clear (the render margins of test_gpu_parity plus a relative gap >= 1e-4
between the two largest weights).  Per-Gaussian sums and counts are then
checked for every Gaussian: an ambiguous pixel can move at most one count
and one contribution between the Gaussians it names on either side, and a
contribution w (D - d)^2 is one summand of the pixel's Eq. 10 uncertainty U,
so |S_gpu - S_ref| may exceed the float tolerance by at most the summed U of
the ambiguous pixels that name the Gaussian, and the counts by their number.
Gaussians that no ambiguous pixel names must match to the float tolerance.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2403_16095_amd import synth
from helpers import DECISION_MARGIN, unambiguous

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_16095_amd import rasterizer
    return rasterizer


def t32(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def sensor_depth(seed, cam, lo, hi, missing=0.05):
    rng = np.random.default_rng(seed)
    D = rng.uniform(lo, hi, (cam["height"], cam["width"])).astype(np.float32)
    D[rng.random(D.shape) < missing] = 0.0
    return D


def compare_window(R, sc, cams, poses, depths):
    """GPU window (one batched call) vs oracle per keyframe; returns GPU sums."""
    n = sc["means"].shape[0]
    scd = {k: t32(v) for k, v in sc.items()}
    P = torch.stack([R.pose_tensor(*p) for p in poses]).contiguous()
    nu_sum = torch.zeros(n, device="cuda")
    nu_cnt = torch.zeros(n, dtype=torch.int32, device="cuda")
    st = R.State()
    _, doms = R.render_nu(st, scd, P, cams, [t32(d) for d in depths], nu_sum, nu_cnt, maps=("depth",), dominant=True)
    gs, gc = nu_sum.cpu().numpy().astype(np.float64), nu_cnt.cpu().numpy().astype(np.int64)
    o_sum, o_cnt = np.zeros(n), np.zeros(n, np.int64)
    slack_sum, slack_cnt = np.zeros(n), np.zeros(n, np.int64)
    n_amb = n_px = 0
    for v, (cam, pose, D) in enumerate(zip(cams, poses, depths)):
        D64 = D.astype(np.float64)
        r = oracle.gaussian_uncertainty(sc, cam, pose, D64, o_sum, o_cnt)
        ref = oracle.render(sc, cam, pose, D64)
        gd = doms[v].cpu().numpy()
        clear = unambiguous(ref) & (r["margin"] >= DECISION_MARGIN)
        assert np.array_equal(gd[clear], r["dominant"][clear]), f"view {v}: dominant map differs"
        amb = ~clear & (D > 0)
        U = ref["uncertainty"][amb] * (1 + 1e-3) + 1e-9
        for ids in (r["dominant"][amb], gd[amb]):
            ok = ids >= 0
            np.add.at(slack_sum, ids[ok], U[ok])
            np.add.at(slack_cnt, ids[ok], 1)
        n_amb += int(amb.sum())
        n_px += amb.size
    involved = (o_cnt > 0) | (gc > 0)
    touched = slack_cnt > 0
    say(f"ambiguous pixels {n_amb}/{n_px}; Gaussians with dominated pixels {int(involved.sum())}, "
        f"named by an ambiguous pixel {int((touched & involved).sum())}")
    assert np.all(np.abs(gc - o_cnt) <= slack_cnt)
    tol = 1e-4 * np.abs(o_sum) + 1e-7
    assert np.all(np.abs(gs - o_sum) <= tol + slack_sum)
    clean = ~touched
    assert np.array_equal(gc[clean], o_cnt[clean])
    err = np.abs(gs[clean] - o_sum[clean]) / np.maximum(np.abs(o_sum[clean]), 1e-3)
    say("max rel err of clean nu sums", err.max(initial=0.0))
    assert err.max(initial=0.0) <= 1e-4
    return nu_sum, nu_cnt


def test_nu_parity_scene(R):
    say("case: nu, 2000 Gaussians, 64x48, two keyframes")
    sc = synth.uniform_box_scene(0)
    cam = synth.SMALL_CAMERA
    poses = [(np.eye(3), np.zeros(3)), (synth.rot_about_axis([0, 1, 0], np.deg2rad(4.0)), np.array([0.05, 0.0, 0.0]))]
    depths = [sensor_depth(1000 + k, cam, 1.5, 4.0) for k in range(2)]
    compare_window(R, sc, [cam, cam], poses, depths)


def test_nu_mapping_size_keyframe_window(R):
    say("case: nu, 500k Gaussians, 4 keyframes 1200x680 in one call")
    sc = synth.room_scene(0, 500_000, (8.0, 6.0, 3.0))
    cam = synth.MAPPING_CAMERA
    poses = synth.random_walk_poses(7, 4)
    depths = [sensor_depth(2000 + k, cam, 0.5, 5.0) for k in range(4)]
    nu_sum, nu_cnt = compare_window(R, sc, [cam] * 4, poses, depths)
    # one batched window == the keyframes one call at a time
    scd = {k: t32(v) for k, v in sc.items()}
    s2 = torch.zeros_like(nu_sum)
    c2 = torch.zeros_like(nu_cnt)
    st = R.State()
    for k in range(4):
        R.render_nu(st, scd, R.pose_tensor(*poses[k]), [cam], [t32(depths[k])], s2, c2, maps=("depth",))
    assert torch.equal(c2, nu_cnt)
    assert ((s2 - nu_sum).abs() <= 1e-5 * nu_sum.abs() + 1e-9).all()


def test_nu_prune_kernel_matches_oracle_rule(R):
    rng = np.random.default_rng(9)
    n = 300_001
    cnt = rng.integers(0, 50, n).astype(np.int32)
    cnt[rng.random(n) < 0.2] = 0
    S = (rng.gamma(0.5, 0.05, n) * np.maximum(cnt, 1)).astype(np.float32)
    o = rng.normal(1.0, 2.0, n).astype(np.float32)
    nu_ref = oracle.nu_from_sums(S.astype(np.float64), cnt)
    o_ref, mask_ref = oracle.prune_uncertain(o.astype(np.float64), nu_ref)
    logits = t32(o)
    nu, pruned = R.nu_prune(t32(S), torch.from_numpy(cnt).cuda(), opacity_logits=logits)
    nu = nu.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(nu, nu_ref, rtol=2e-7, atol=0)
    clear = np.abs(nu_ref - oracle.NU_TAU) > 1e-5 * oracle.NU_TAU
    gpu_mask = nu > oracle.NU_TAU
    assert np.array_equal(gpu_mask[clear], mask_ref[clear])
    assert int(pruned.item()) == int(gpu_mask.sum())
    np.testing.assert_allclose(logits.cpu().numpy()[clear], o_ref[clear], rtol=0, atol=1e-6)
    # empty input is a no-op
    R.nu_prune(torch.zeros(0, device="cuda"), torch.zeros(0, dtype=torch.int32, device="cuda"))
