"""Pins of the oracle's view-dependent colour (Sec. 3.1: each Gaussian's
colour comes from spherical-harmonic coefficients) against things other than
itself: scipy's spherical harmonics, orthonormality on the sphere by
quadrature, numerical derivatives, the constant-colour special case, a
closed-form single-Gaussian render, and frozen-decision finite differences
of the full render."""
import numpy as np
import pytest
from scipy import special
from scipy.spatial.transform import Rotation

import oracle
from paper_2403_16095_amd import synth

IDENTITY = (np.eye(3), np.zeros(3))


def real_sh_scipy(l, m, d):
    """Real harmonic (l, m) from scipy's complex one, which carries the
    Condon-Shortley phase: sqrt2 Re Y_l^m (m > 0), sqrt2 Im Y_l^|m| (m < 0)."""
    polar, azim = np.arccos(np.clip(d[2], -1, 1)), np.arctan2(d[1], d[0])
    z = special.sph_harm_y(l, abs(m), polar, azim)
    if m == 0:
        return z.real
    return np.sqrt(2.0) * (z.real if m > 0 else z.imag)


def unit_dirs(rng, n):
    d = rng.standard_normal((n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


@pytest.mark.parametrize("degree", [0, 1, 2, 3])
def test_basis_matches_scipy(degree):
    rng = np.random.default_rng(degree)
    for d in unit_dirs(rng, 50):
        Y, _ = oracle.sh_basis(degree, d)
        ref = [real_sh_scipy(l, m, d) for l in range(degree + 1) for m in range(-l, l + 1)]
        np.testing.assert_allclose(Y, ref, atol=1e-14)


def test_basis_is_orthonormal_on_the_sphere():
    """Gauss-Legendre in cos(theta) times a uniform azimuth grid integrates
    products of two degree-3 harmonics exactly."""
    zs, wz = np.polynomial.legendre.leggauss(12)
    phis = np.arange(24) * (2 * np.pi / 24)
    G = np.zeros((16, 16))
    for z, w in zip(zs, wz):
        s = np.sqrt(1 - z * z)
        for ph in phis:
            Y, _ = oracle.sh_basis(3, [s * np.cos(ph), s * np.sin(ph), z])
            G += w * (2 * np.pi / 24) * np.outer(Y, Y)
    np.testing.assert_allclose(G, np.eye(16), atol=1e-13)


def test_basis_gradient_matches_numerical_derivative_on_the_sphere():
    """The tangential part of dY (the only part the chain rule through the
    normalised direction keeps) against central differences of Y(d + h t)
    renormalised, for tangent vectors t."""
    rng = np.random.default_rng(7)
    for d in unit_dirs(rng, 20):
        _, dY = oracle.sh_basis(3, d)
        for t in unit_dirs(rng, 3):
            t = t - d * (t @ d)
            t /= np.linalg.norm(t)
            h = 1e-6
            yp, _ = oracle.sh_basis(3, (d + h * t) / np.linalg.norm(d + h * t))
            ym, _ = oracle.sh_basis(3, (d - h * t) / np.linalg.norm(d - h * t))
            np.testing.assert_allclose(dY @ t, (yp - ym) / (2 * h), atol=1e-8)


def test_degree_zero_reproduces_constant_colour():
    """Degree 0 is a constant colour: with sh_0 = (rgb - 1/2) / Y_00 and
    Y_00 = 1 / sqrt(4 pi) every map equals the rgb render."""
    sc = {k: v.astype(np.float64) for k, v in synth.uniform_box_scene(3, 300).items()}
    cam = synth.SMALL_CAMERA
    pose = (Rotation.from_rotvec([0.02, -0.03, 0.01]).as_matrix(), np.array([0.05, 0.0, 0.1]))
    shs = dict(sc)
    shs["sh"] = ((sc["rgb"] - 0.5) * np.sqrt(4 * np.pi))[:, None, :]
    del shs["rgb"]
    a = oracle.render(sc, cam, pose)
    b = oracle.render(shs, cam, pose)
    for k in ("color", "depth", "opacity", "depth_median"):
        np.testing.assert_allclose(b[k], a[k], atol=1e-13)


def single_opaque_gaussian(center, sh):
    return dict(means=np.array([center], np.float64), log_scales=np.full((1, 3), -1.0),
                quats=np.array([[1.0, 0, 0, 0]]), opacity_logits=np.array([8.0]),
                sh=np.asarray(sh, np.float64)[None])


def test_colour_follows_the_viewing_direction_from_the_camera_centre():
    """One opaque Gaussian seen from a camera whose centre is C: at the pixel
    under its mean the colour is alpha (1/2 + k_c Y_1^0(d)) with
    Y_1^0(d) = sqrt(3 / (4 pi)) d_z and d = (X - C) / |X - C|, the only
    coefficient being that of (l, m) = (1, 0)."""
    cam = synth.camera(33, 33, 30.0, 30.0, 16.0, 16.0)
    rng = np.random.default_rng(5)
    for _ in range(5):
        R = Rotation.from_rotvec(rng.normal(0, 0.4, 3)).as_matrix()
        C = rng.normal(0, 1.0, 3)
        t = -R @ C
        # put the Gaussian on the optical axis, 3 m in front of the camera
        X = C + 3.0 * R.T @ np.array([0.0, 0.0, 1.0])
        k = np.array([0.3, -0.2, 0.1])
        sh = np.zeros((4, 3))
        sh[2] = k
        m = oracle.render(single_opaque_gaussian(X, sh), cam, (R, t))
        d = (X - C) / np.linalg.norm(X - C)
        alpha = min(0.99, 1.0 / (1.0 + np.exp(-8.0)))
        expect = alpha * (0.5 + k * np.sqrt(3 / (4 * np.pi)) * d[2])
        np.testing.assert_allclose(m["color"][:, 16, 16], expect, rtol=1e-12)


def test_negative_colour_is_clamped_to_zero_with_zero_gradient():
    cam = synth.camera(33, 33, 30.0, 30.0, 16.0, 16.0)
    sh = np.zeros((1, 3))
    sh[0] = [-3.0, 1.0, -0.5]     # 1/2 + Y_00 k: negative, positive, positive
    sc = single_opaque_gaussian([0.0, 0.0, 3.0], sh)
    m = oracle.render(sc, cam, IDENTITY)
    assert m["color"][0, 16, 16] == 0.0 and m["color"][1, 16, 16] > 0 and m["color"][2, 16, 16] > 0
    dimg = dict(color=np.ones((3, 33, 33)))
    g = oracle.backward(sc, cam, IDENTITY, None, dimg)
    assert g["sh"][0, 0, 0] == 0.0 and g["sh"][0, 0, 1] > 0


def sh_scene(seed, n, degree, rest_std=0.3, **kw):
    sc = {k: v.astype(np.float64) for k, v in synth.uniform_box_scene(seed, n, **kw).items()}
    sc["sh"] = synth.sh_coefficients(seed + 1, n, degree, rest_std=rest_std).astype(np.float64)
    del sc["rgb"]
    return sc


def test_sh_gradients_match_frozen_fd_on_tiny_scene():
    """Every coefficient, mean and pose coordinate of a degree-3 scene under
    a non-trivial pose: the direction term reaches the means and the
    translation part of the pose."""
    rng = np.random.default_rng(21)
    cam = synth.camera(10, 8, 8.0, 8.5, 4.6, 4.2)
    sc = sh_scene(6, 8, 3, xy=(-0.5, 0.5), z=(1.5, 3.0), log_scale=(-1.6, 0.3))
    R = Rotation.from_rotvec([0.05, -0.08, 0.03]).as_matrix()
    pose = (R, np.array([0.3, -0.2, 0.1]))
    dimg = dict(color=rng.standard_normal((3, 8, 10)), depth=rng.standard_normal((8, 10)))
    g = oracle.backward(sc, cam, pose, None, dimg)
    coords = [("sh", i, c) for i in range(8) for c in range(48)]
    coords += [("means", i, c) for i in range(8) for c in range(3)]
    coords += [("pose", 0, c) for c in range(6)]
    fd = oracle.fd_linear(sc, cam, pose, None, dimg, coords)
    an = []
    for kind, i, c in coords:
        if kind == "sh":
            an.append(g["sh"][i, c // 3, c % 3])
        elif kind == "pose":
            an.append(g["pose"][c])
        else:
            an.append(g[kind][i, c])
    an = np.array(an)
    scale = np.abs(an).max()
    np.testing.assert_allclose(an, fd, rtol=1e-5, atol=1e-7 * scale)


def test_camera_translation_equals_moving_every_gaussian():
    """At the identity pose a camera translation rho puts every Gaussian at
    X + rho in the camera frame and the camera centre at -rho, which is the
    same as moving every mean by +rho with the camera fixed -- for the
    geometry and for the viewing directions alike -- so d L / d rho is the
    sum of the mean gradients (no finite differences involved)."""
    rng = np.random.default_rng(3)
    cam = synth.SMALL_CAMERA
    sc = sh_scene(9, 400, 3)
    dimg = dict(color=rng.standard_normal((3, 48, 64)), depth=rng.standard_normal((48, 64)),
                opacity=rng.standard_normal((48, 64)))
    g = oracle.backward(sc, cam, IDENTITY, None, dimg)
    np.testing.assert_allclose(g["pose"][:3], g["means"].sum(0), rtol=1e-10,
                               atol=1e-12 * np.abs(g["means"]).sum())


def test_direction_term_is_material_at_parity_sizes():
    """On the GPU parity scene (strongly view-dependent coefficients) the pose
    gradient through the camera centre is well above the 1e-3 parity
    tolerance, so a GPU path without it fails: freezing
    every Gaussian's colour at its value for this pose (an rgb scene) changes
    the translation gradient by much more than that."""
    cam = synth.SMALL_CAMERA
    sc = sh_scene(1, 2000, 3, rest_std=1.0)
    pose = (Rotation.from_rotvec([0.03, -0.05, 0.02]).as_matrix(), np.array([0.12, -0.07, 0.2]))
    rng = np.random.default_rng(8)
    dimg = dict(color=rng.standard_normal((3, 48, 64)))
    g = oracle.backward(sc, cam, pose, None, dimg)
    R, t = pose
    C = -R.T @ t
    rgb = np.zeros((2000, 3))
    for i in range(2000):
        v = sc["means"][i] - C
        Y, _ = oracle.sh_basis(3, v / np.linalg.norm(v))
        rgb[i] = np.maximum(0.0, Y @ sc["sh"][i] + 0.5)
    frozen = {k: v for k, v in sc.items() if k != "sh"}
    frozen["rgb"] = rgb
    a = oracle.render(sc, cam, pose)
    b = oracle.render(frozen, cam, pose)
    np.testing.assert_allclose(b["color"], a["color"], atol=1e-12)   # same colours at this pose
    gf = oracle.backward(frozen, cam, pose, None, dimg)
    diff = np.abs(g["pose"][:3] - gf["pose"][:3]).max() / np.abs(g["pose"]).max()
    assert diff > 5e-3, diff
    np.testing.assert_allclose(g["pose"][3:], gf["pose"][3:], rtol=1e-10, atol=1e-12)
