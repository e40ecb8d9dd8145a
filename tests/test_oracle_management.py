"""Pins of the Gaussian-management oracle (Sec. 3.3) against things other
than itself: spawned Gaussians project back onto their pixels at their depth
(the oracle's projection, Eq. 1-2), show their pixel's colour (the oracle's
render), are counted by brute force over the mask; split halves sit at
Mahalanobis distance |z| from their parent; clones are exact copies."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from oracle import management as M
from paper_2403_16095_amd import synth


@pytest.fixture(scope="module")
def view():
    cam = synth.camera(40, 30, 35.0, 33.0, 19.5, 14.5)
    rng = np.random.default_rng(0)
    color = rng.random((3, 30, 40))
    depth = rng.uniform(1.0, 3.0, (30, 40))
    depth[rng.random((30, 40)) < 0.1] = 0.0            # missing measurements
    opacity = rng.random((30, 40))
    pose = (Rotation.from_rotvec([0.1, -0.2, 0.05]).as_matrix(), np.array([0.3, -0.1, 0.5]))
    return cam, color, depth, opacity, pose


def test_spawn_mask_by_brute_force(view):
    cam, color, depth, opacity, pose = view
    new, idx = M.spawn(color, depth, cam, pose, opacity)
    expect = [v * 40 + u for v in range(30) for u in range(40) if depth[v, u] > 0 and opacity[v, u] < 0.5]
    assert idx.tolist() == expect
    dense, idx2 = M.spawn(color, depth, cam, pose, None, stride=3)
    assert idx2.tolist() == [v * 40 + u for v in range(0, 30, 3) for u in range(0, 40, 3) if depth[v, u] > 0]
    assert new["means"].shape == (len(expect), 3)


def test_spawned_means_project_onto_their_pixels(view):
    cam, color, depth, opacity, pose = view
    new, idx = M.spawn(color, depth, cam, pose, opacity)
    pr = oracle.project(new, cam, pose)
    u, v = idx % 40, idx // 40
    np.testing.assert_allclose(pr["mu"][:, 0], u, atol=1e-9)
    np.testing.assert_allclose(pr["mu"][:, 1], v, atol=1e-9)
    np.testing.assert_allclose(pr["depth"], depth.ravel()[idx], rtol=1e-12)
    # isotropic, one pixel's footprint at that depth
    f = 0.5 * (cam["fx"] + cam["fy"])
    np.testing.assert_allclose(np.exp(new["log_scales"]), np.repeat(depth.ravel()[idx, None] / f, 3, 1))


def test_spawned_gaussian_shows_its_pixel_colour():
    """A single spawned Gaussian, made opaque, rendered from the spawning
    camera: the pixel under it blends its colour with alpha = 0.99 (rgb and
    degree-3 view-dependent colour alike)."""
    cam = synth.camera(21, 21, 20.0, 20.0, 10.0, 10.0)
    pose = (Rotation.from_rotvec([0.2, 0.1, -0.1]).as_matrix(), np.array([0.1, 0.2, 0.3]))
    color = np.zeros((3, 21, 21))
    color[:, 10, 10] = [0.2, 0.7, 0.4]
    depth = np.zeros((21, 21))
    depth[10, 10] = 2.0
    for deg in (None, 3):
        new, idx = M.spawn(color, depth, cam, pose, None, init_logit=10.0, sh_degree=deg)
        assert idx.tolist() == [10 * 21 + 10]
        new["log_scales"] = new["log_scales"] + np.log(3.0)   # wide enough that alpha caps at the centre
        m = oracle.render(new, cam, pose)
        np.testing.assert_allclose(m["color"][:, 10, 10], 0.99 * np.array([0.2, 0.7, 0.4]), rtol=1e-9)


def test_compaction_keeps_order():
    rng = np.random.default_rng(1)
    p = dict(a=rng.random((50, 3)), b=rng.random(50))
    keep = rng.random(50) < 0.4
    c = M.compact(p, keep)
    np.testing.assert_array_equal(c["a"], p["a"][np.nonzero(keep)[0]])
    assert c["b"].shape == (keep.sum(),)


def test_densify_clone_and_split():
    rng = np.random.default_rng(2)
    n = 40
    sc = {k: v.astype(np.float64) for k, v in synth.uniform_box_scene(3, n).items()}
    grad = rng.uniform(0, 2e-3, n)
    denom = rng.integers(0, 5, n)
    z = rng.standard_normal((n, 2, 3))
    out, clone, split = M.densify(sc, grad, denom, 1e-4, 0.05, z)
    stat = np.where(denom > 0, grad / np.maximum(denom, 1), 0)
    smax = np.exp(sc["log_scales"]).max(1)
    assert np.array_equal(clone, (stat >= 1e-4) & (smax <= 0.05))
    assert np.array_equal(split, (stat >= 1e-4) & (smax > 0.05))
    nk, nc, ns = (~split).sum(), clone.sum(), split.sum()
    assert clone.any() and split.any()
    assert out["means"].shape[0] == nk + nc + 2 * ns
    # kept then clones: exact copies
    np.testing.assert_array_equal(out["means"][:nk], sc["means"][~split])
    np.testing.assert_array_equal(out["rgb"][nk:nk + nc], sc["rgb"][clone])
    # halves: Mahalanobis distance |z| from the parent, scales / 1.6
    for j, i in enumerate(np.nonzero(split)[0]):
        Rq = Rotation.from_quat(np.roll(sc["quats"][i], -1)).as_matrix()   # scipy is scalar-last
        S = np.exp(sc["log_scales"][i])
        Sigma = Rq @ np.diag(S ** 2) @ Rq.T
        for k in range(2):
            m = out["means"][nk + nc + 2 * j + k]
            d = m - sc["means"][i]
            np.testing.assert_allclose(d @ np.linalg.solve(Sigma, d), z[i, k] @ z[i, k], rtol=1e-9)
            np.testing.assert_allclose(np.exp(out["log_scales"][nk + nc + 2 * j + k]), S / 1.6, rtol=1e-12)
            np.testing.assert_array_equal(out["quats"][nk + nc + 2 * j + k], sc["quats"][i])
