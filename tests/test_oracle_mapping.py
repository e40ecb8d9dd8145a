"""Pins of the mapping-objective oracle (Eq. 11, 12, 14-18): SSIM against an
independent scipy implementation and closed forms, every gradient against
central differences, and hand-computed isotropy and alignment cases."""
import numpy as np
import pytest
from scipy.ndimage import gaussian_filter

from oracle import mapping as M


def scipy_ssim_map(x, y):
    """SSIM with scipy's Gaussian filter: sigma 1.5 truncated at radius 5
    (11 taps), zero ('constant') padding, per channel."""
    def blur(z):
        return np.stack([gaussian_filter(c, 1.5, mode="constant", cval=0.0, truncate=5 / 1.5) for c in z])
    mx, my = blur(x), blur(y)
    sxx = blur(x * x) - mx ** 2
    syy = blur(y * y) - my ** 2
    sxy = blur(x * y) - mx * my
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    return ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx ** 2 + my ** 2 + c1) * (sxx + syy + c2))


def test_ssim_matches_scipy_gaussian_filter():
    rng = np.random.default_rng(0)
    x, y = rng.random((3, 23, 31)), rng.random((3, 23, 31))
    m, smap = M.ssim(x, y)
    ref = scipy_ssim_map(x, y)
    np.testing.assert_allclose(smap, ref, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(m, ref.mean(), rtol=1e-12)


def test_ssim_closed_forms():
    rng = np.random.default_rng(1)
    x = rng.random((3, 16, 16))
    assert M.ssim(x, x)[0] == pytest.approx(1.0, abs=1e-12)
    loss, g = M.ssim_loss(x, x)
    assert abs(loss) < 1e-12 and np.abs(g).max() < 1e-10
    # constant images a, b: away from the zero-padded border the variances
    # vanish and SSIM = (2ab + C1) / (a^2 + b^2 + C1)
    a, b = 0.3, 0.7
    _, smap = M.ssim(np.full((1, 30, 30), a), np.full((1, 30, 30), b))
    inner = smap[0, 5:-5, 5:-5]
    np.testing.assert_allclose(inner, (2 * a * b + 1e-4) / (a * a + b * b + 1e-4), rtol=1e-12)
    w = M.gaussian_window_1d()
    assert w.shape == (11,) and w.sum() == pytest.approx(1.0) and np.argmax(w) == 5


def fd(f, x, idx, h=1e-6):
    xp, xm = x.copy(), x.copy()
    xp[idx] += h
    xm[idx] -= h
    return (f(xp) - f(xm)) / (2 * h)


def test_ssim_gradient_central_differences():
    rng = np.random.default_rng(2)
    x, y = rng.random((3, 9, 8)), rng.random((3, 9, 8))
    _, g = M.ssim_loss(x, y)
    for idx in [(0, 0, 0), (1, 4, 3), (2, 8, 7), (0, 5, 0), (2, 2, 6)]:
        assert g[idx] == pytest.approx(fd(lambda z: M.ssim_loss(z, y)[0], x, idx), rel=1e-6, abs=1e-10)


def test_iso_loss_hand_values_and_gradient():
    ls = np.log(np.array([[1.0, 2.0, 4.0], [0.5, 0.5, 0.5], [3.0, 1.0, 2.0], [9.0, 1.0, 1.0]]))
    vis = np.array([1, 1, 1, 0])
    L, g = M.iso_loss(ls, vis)
    # ratios 4, 1, 3 over 3 visible Gaussians: (3 + 0 + 2) / 3
    assert L == pytest.approx(5.0 / 3.0)
    assert np.all(g[3] == 0) and np.all(g[1] == 0)
    np.testing.assert_allclose(g[0], [-4 / 3, 0, 4 / 3])
    np.testing.assert_allclose(g[2], [1.0, -1.0, 0.0])
    rng = np.random.default_rng(3)
    ls = rng.normal(-3, 0.5, (6, 3))
    vis = rng.integers(0, 2, 6)
    vis[0] = 1
    _, g = M.iso_loss(ls, vis)
    for idx in [(0, 0), (0, 1), (0, 2), (3, 1), (5, 2)]:
        assert g[idx] == pytest.approx(fd(lambda z: M.iso_loss(z, vis)[0], ls, idx), rel=1e-6, abs=1e-12)


def test_align_var_and_l1_terms():
    D = np.array([[2.0, 3.0], [1.0, 4.0]])
    Dm = np.array([[1.5, 3.5], [0.0, 4.0]])
    has = np.array([[True, True], [False, True]])
    L, gd, gm = M.align_loss(D, Dm, has)
    assert L == pytest.approx((0.5 + 0.5 + 0 + 0) / 4)
    np.testing.assert_allclose(gd, [[0.25, -0.25], [0, 0]])
    np.testing.assert_allclose(gm, -gd)
    U = np.array([[0.0, 2.0], [1.0, 0.5]])
    L, g = M.var_loss(U)
    assert L == pytest.approx(3.5 / 4)
    np.testing.assert_allclose(g, [[0, 0.25], [0.25, 0.25]])


def test_objective_is_the_weighted_sum_and_linear_in_omega():
    rng = np.random.default_rng(4)
    H, W = 12, 10
    maps = dict(color=rng.random((3, H, W)), depth=rng.uniform(1, 3, (H, W)), depth_median=rng.uniform(1, 3, (H, W)),
                uncertainty=rng.random((H, W)), has_median=rng.random((H, W)) > 0.2)
    tc, td = rng.random((3, H, W)), rng.uniform(1, 3, (H, W))
    ls = rng.normal(-3, 0.4, (20, 3))
    vis = rng.integers(0, 2, 20)
    parts = []
    for k in range(6):
        om = [0.0] * 6
        om[k] = 1.0
        parts.append(M.mapping_objective(maps, tc, td, ls, vis, om))
    L, dimg, dls = M.mapping_objective(maps, tc, td, ls, vis)
    w = M.OMEGA_REPLICA
    assert L == pytest.approx(sum(w[k] * parts[k][0] for k in range(6)))
    for key in dimg:
        np.testing.assert_allclose(dimg[key], sum(w[k] * parts[k][1][key] for k in range(6)), atol=1e-15)
    np.testing.assert_allclose(dls, sum(w[k] * parts[k][2] for k in range(6)), atol=1e-15)
    # each unit-weight part is the matching single term
    assert parts[0][0] == pytest.approx(M.color_l1(maps["color"], tc)[0])
    assert parts[3][0] == pytest.approx(M.align_loss(maps["depth"], maps["depth_median"], maps["has_median"])[0])
    assert M.OMEGA_REPLICA == (0.7, 0.1, 0.25, 0.25, 0.1, 0.15)
