"""HIP mapping objective (Eq. 18: Eq. 11, 12, 14-17) vs the FP64 oracle.

The objective kernels take rendered maps as plain inputs, so their parity
test feeds both sides the same seeded synthetic maps (64x48 and the
1200x680 mapping size, whose 16-pixel SSIM tiles end in a ragged row); the
state's last render only supplies the view sizes and the visible Gaussians
of the isotropy term, which the oracle takes from its own projection.  An
end-to-end case then runs render -> objective -> backward on both sides.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import mapping as OM
from paper_2403_16095_amd import synth
from helpers import grad_parity, rel_l2

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


def synthetic_maps(seed, H, W):
    rng = np.random.default_rng(seed)
    f = np.float32
    depth = rng.uniform(1.5, 4.0, (H, W)).astype(f)
    median = (depth + rng.normal(0, 0.1, (H, W))).astype(f)
    median[rng.random((H, W)) < 0.2] = 0.0                       # no median Gaussian
    maps = dict(color=rng.random((3, H, W)).astype(f), depth=depth, depth_median=median,
                uncertainty=rng.uniform(0, 0.5, (H, W)).astype(f))
    maps["uncertainty"][rng.random((H, W)) < 0.05] = 0.0
    tc = rng.random((3, H, W)).astype(f)
    td = rng.uniform(1.5, 4.0, (H, W)).astype(f)
    return maps, tc, td


def oracle_objective(maps, tc, td, log_scales, visible, omega):
    m64 = {k: v.astype(np.float64) for k, v in maps.items()}
    m64["has_median"] = maps["depth_median"] > 0
    return OM.mapping_objective(m64, tc.astype(np.float64), td.astype(np.float64), log_scales, visible, omega)


@pytest.mark.parametrize("size", ["small", "mapping"])
def test_objective_kernels_on_synthetic_maps(R, size):
    if size == "small":
        sc, cam, pose = synth.uniform_box_scene(0), synth.SMALL_CAMERA, (np.eye(3), np.zeros(3))
    else:
        sc, cam = synth.room_scene(0, 200_000, (8.0, 6.0, 3.0)), synth.MAPPING_CAMERA
        pose = synth.level_room_pose(0)
    say("case: mapping objective on synthetic maps,", size, cam["width"], "x", cam["height"])
    H, W = cam["height"], cam["width"]
    scd = {k: t32(v) for k, v in sc.items()}
    st = R.State()
    R.render(st, scd, R.pose_tensor(*pose), [cam], maps=("depth",))
    maps, tc, td = synthetic_maps(11, H, W)
    omega = OM.OMEGA_REPLICA
    dls = torch.zeros_like(scd["log_scales"])
    loss = torch.zeros(1, device="cuda")
    dimg = R.mapping_objective(st, [{k: t32(v) for k, v in maps.items()}], [t32(tc)], [t32(td)], omega,
                               dlog_scales=dls, loss=loss)[0]
    vis = oracle.project(sc, cam, pose)["visible"]
    L, ref, ref_ls = oracle_objective(maps, tc, td, sc["log_scales"].astype(np.float64), vis, omega)
    say("loss gpu", loss.item(), "oracle", L)
    assert abs(loss.item() - L) <= 2e-5 * abs(L)
    for k in ("depth", "depth_median", "uncertainty"):
        # sign-based terms: equal up to float rounding of the weights / (H W)
        np.testing.assert_allclose(dimg[k].cpu().numpy(), ref[k], rtol=1e-6, atol=0, err_msg=k)
    gc = dimg["color"].cpu().numpy().astype(np.float64)
    err = np.abs(gc - ref["color"]).max() / np.abs(ref["color"]).max()
    say("colour gradient (L1 + SSIM) max rel err", err)
    assert err <= 1e-4
    # the SSIM part alone, relative to its own scale
    ssim_ref = ref["color"] - omega[0] * OM.color_l1(maps["color"].astype(np.float64), tc)[1]
    ssim_gpu = gc - omega[0] * np.sign(maps["color"].astype(np.float64) - tc) / (H * W)
    e2 = rel_l2(ssim_gpu, ssim_ref)
    say("SSIM gradient rel l2", e2)
    assert e2 <= 1e-4
    e3 = rel_l2(dls.cpu().numpy(), ref_ls)
    say("isotropy gradient rel l2", e3)
    assert e3 <= 1e-4


def test_objective_needs_its_inputs(R):
    sc, cam = synth.uniform_box_scene(0), synth.SMALL_CAMERA
    st = R.State()
    R.render(st, {k: t32(v) for k, v in sc.items()}, R.pose_tensor(np.eye(3), np.zeros(3)), [cam], maps=("depth",))
    maps, tc, td = synthetic_maps(1, cam["height"], cam["width"])
    m = {k: t32(v) for k, v in maps.items()}
    del m["uncertainty"]
    from paper_2403_16095_amd.binding import CgsrError
    with pytest.raises(CgsrError):
        R.mapping_objective(st, [m], [t32(tc)], [t32(td)])          # var weight without uncertainty
    R.mapping_objective(st, [m], [t32(tc)], [t32(td)], omega=(0.7, 0.1, 0.25, 0.25, 0.1, 0.0))


def test_render_objective_backward_end_to_end(R):
    say("case: render -> Eq. 18 -> backward, 2000 Gaussians 64x48")
    sc, cam = synth.uniform_box_scene(0), synth.SMALL_CAMERA
    pose = (np.eye(3), np.zeros(3))
    tc, td = synth.random_targets(1000, cam)
    scd = {k: t32(v) for k, v in sc.items()}
    st = R.State()
    out = R.render(st, scd, R.pose_tensor(*pose), [cam], [t32(td)])[0]
    omega = OM.OMEGA_REPLICA
    dls = torch.zeros_like(scd["log_scales"])
    dimg = R.mapping_objective(st, [out], [t32(tc)], [t32(td)], omega, dlog_scales=dls)
    grads, dposes = R.backward(st, dimg)
    grads["log_scales"] += dls
    ref = oracle.render(sc, cam, pose, td)
    maps = dict(color=ref["color"], depth=ref["depth"], depth_median=ref["depth_median"],
                uncertainty=ref["uncertainty"], has_median=ref["median_id"] >= 0)
    vis = oracle.project(sc, cam, pose)["visible"]
    _, rdimg, rls = OM.mapping_objective(maps, tc, td, sc["log_scales"].astype(np.float64), vis, omega)
    rb = oracle.backward(sc, cam, pose, td, rdimg)
    rb["log_scales"] = rb["log_scales"] + rls
    for k in ("means", "log_scales", "quats", "opacity_logits", "rgb"):
        grad_parity(k, grads[k].cpu().numpy(), rb[k], label="Eq. 18 end to end")
    e = np.abs(dposes[0].cpu().numpy() - rb["pose"]).max() / np.abs(rb["pose"]).max()
    say("pose rel err", e)
    assert e <= 1e-3
