"""Pins of the oracle's per-Gaussian depth uncertainty (Sec. 3.2, Eq. 13) and
the pruning rule that uses it, against closed forms, hand-computed cases, a
plain per-pixel Python enumeration on a tiny scene, and invariants."""
import numpy as np
import pytest

import oracle
from paper_2403_16095_amd import synth

IDENTITY = (np.eye(3), np.zeros(3))


def one(means, log_scales, quats, p, rgb):
    return dict(means=np.array([means], np.float64), log_scales=np.array([log_scales], np.float64),
                quats=np.array([quats], np.float64), opacity_logits=np.array([np.log(p / (1 - p))], np.float64),
                rgb=np.array([rgb], np.float64))


def stack(*scenes):
    return {k: np.concatenate([s[k] for s in scenes], 0) for k in scenes[0]}


def test_single_isotropic_gaussian_closed_form():
    """One isotropic Gaussian dominates every pixel of its support, with
    weight alpha(r) (T = 1); pixels with no sensor depth do not count."""
    cam = synth.SMALL_CAMERA
    z, s, sig = 2.0, 0.05, 0.88
    sc = one([0, 0, z], [np.log(s)] * 3, [0.3, -0.4, 0.5, 0.1], sig, [0.2, 0.5, 0.9])
    v, u = np.mgrid[0:cam["height"], 0:cam["width"]]
    D = 2.0 + 0.01 * u - 0.02 * v
    D[::5, ::3] = 0.0                                     # missing measurements
    var = (cam["fx"] * s / z) ** 2 + 0.3
    r2 = (u - cam["cx"]) ** 2 + (v - cam["cy"]) ** 2
    a = np.minimum(0.99, sig * np.exp(-r2 / (2 * var)))
    a[a < 1 / 255] = 0.0
    valid = (a > 0) & (D > 0)
    r = oracle.gaussian_uncertainty(sc, cam, IDENTITY, D)
    assert r["count"][0] == valid.sum()
    np.testing.assert_allclose(r["sum"][0], (a * (D - z) ** 2)[valid].sum(), rtol=1e-13)
    assert np.array_equal(r["dominant"] == 0, a > 0)
    assert np.all(r["dominant"][a == 0] == -1)
    assert np.all(r["margin"][a > 0] == 1.0)               # no runner-up
    nu = oracle.nu_from_sums(r["sum"], r["count"])
    np.testing.assert_allclose(nu[0], (a * (D - z) ** 2)[valid].mean(), rtol=1e-13)


@pytest.mark.parametrize("a_far, far_wins", [(0.4, False), (0.5, True)])
def test_dominant_is_the_largest_weight_not_the_first(a_far, far_wins):
    """Near alpha 0.3 (w = 0.3) in front of far alpha a (w = 0.7 a): 0.28 loses,
    0.35 wins; the margin is (w1 - w2) / w1."""
    cam = synth.SMALL_CAMERA
    far = one([0, 0, 3.0], [-2] * 3, [1, 0, 0, 0], a_far, [0, 1, 0])
    near = one([0, 0, 1.5], [-2] * 3, [1, 0, 0, 0], 0.3, [1, 0, 0])
    sc = stack(far, near)
    D = np.full((cam["height"], cam["width"]), 2.0)
    r = oracle.gaussian_uncertainty(sc, cam, IDENTITY, D)
    cy, cx = int(cam["cy"]), int(cam["cx"])
    w_near, w_far = 0.3, 0.7 * a_far
    assert r["dominant"][cy, cx] == (0 if far_wins else 1)
    w1, w2 = max(w_near, w_far), min(w_near, w_far)
    np.testing.assert_allclose(r["margin"][cy, cx], (w1 - w2) / w1, rtol=1e-6)


def _python_blend_dominant(sc, cam, D):
    """Brute force: per pixel, every Gaussian in depth order, Eq. 4-5 with the
    skip / cap / stop rules, keeping the largest alpha T."""
    proj = oracle.project(sc, cam, IDENTITY)
    vis = np.nonzero(proj["visible"])[0]
    order = vis[np.lexsort((vis, proj["depth"][vis]))]
    n = sc["means"].shape[0]
    S, M = np.zeros(n), np.zeros(n, np.int64)
    for v in range(cam["height"]):
        for u in range(cam["width"]):
            T, best, wbest = 1.0, -1, 0.0
            for i in order:
                dx, dy = proj["mu"][i, 0] - u, proj["mu"][i, 1] - v
                a_, b_, c_ = proj["conic"][i]
                al = proj["opacity"][i] * np.exp(-0.5 * (a_ * dx * dx + c_ * dy * dy) - b_ * dx * dy)
                if al < 1 / 255:
                    continue
                al = min(0.99, al)
                if T * (1 - al) < 1e-4:
                    break
                if al * T > wbest:
                    best, wbest = i, al * T
                T *= 1 - al
            if best >= 0 and D[v, u] > 0:
                S[best] += wbest * (D[v, u] - proj["depth"][best]) ** 2
                M[best] += 1
    return S, M


def test_tiny_scene_matches_python_enumeration():
    cam = synth.camera(12, 9, 10.0, 10.0, 6.0, 4.5)
    sc = synth.uniform_box_scene(7, 25, log_scale=(-2.0, 0.3), opacity=(0.5, 1.0))
    rng = np.random.default_rng(3)
    D = rng.uniform(1.0, 4.5, (cam["height"], cam["width"]))
    D[rng.random(D.shape) < 0.1] = 0.0
    S, M = _python_blend_dominant(sc, cam, D)
    r = oracle.gaussian_uncertainty(sc, cam, IDENTITY, D, candidates=0)
    assert np.array_equal(r["count"], M)
    np.testing.assert_allclose(r["sum"], S, rtol=1e-12, atol=1e-15)
    assert M.sum() > 50 and (M > 0).sum() > 5


@pytest.fixture(scope="module")
def config1():
    sc = synth.uniform_box_scene(0)
    _, D = synth.random_targets(1000, synth.SMALL_CAMERA)
    return sc, synth.SMALL_CAMERA, D.astype(np.float64)


def test_invariants_on_parity_scene(config1):
    sc, cam, D = config1
    r = oracle.gaussian_uncertainty(sc, cam, IDENTITY, D)
    m = oracle.render(sc, cam, IDENTITY, D)
    # every pixel with a blended Gaussian and a measurement counts exactly once
    assert r["count"].sum() == ((m["n_contrib"] > 0) & (D > 0)).sum()
    assert np.all(r["sum"] >= 0)
    assert np.array_equal(r["dominant"] >= 0, m["n_contrib"] > 0)
    rb = oracle.gaussian_uncertainty(sc, cam, IDENTITY, D, candidates=0)
    assert np.array_equal(rb["count"], r["count"])
    np.testing.assert_allclose(rb["sum"], r["sum"], rtol=1e-13)
    # brute force and candidate lists agree (above); window accumulation is
    # the sum of the single-keyframe parts
    pose2 = (synth.rot_about_axis([0, 1, 0], np.deg2rad(4.0)), np.array([0.05, 0.0, 0.0]))
    r2 = oracle.gaussian_uncertainty(sc, cam, pose2, D)
    acc = oracle.gaussian_uncertainty(sc, cam, IDENTITY, D)
    oracle.gaussian_uncertainty(sc, cam, pose2, D, acc["sum"], acc["count"])
    np.testing.assert_allclose(acc["sum"], r["sum"] + r2["sum"], rtol=1e-13)
    assert np.array_equal(acc["count"], r["count"] + r2["count"])


def test_uncertainty_per_pixel_bounded_by_eq10(config1):
    """A dominated pixel contributes w (D - d)^2 for one blended Gaussian, one
    of the non-negative summands of Eq. 10 at that pixel: sum_i S_i <= sum_p U_p."""
    sc, cam, D = config1
    r = oracle.gaussian_uncertainty(sc, cam, IDENTITY, D)
    m = oracle.render(sc, cam, IDENTITY, D)
    assert r["sum"].sum() <= m["uncertainty"].sum() + 1e-12


def test_permutation_of_gaussians_permutes_nu(config1):
    sc, cam, D = config1
    perm = np.random.default_rng(1).permutation(sc["means"].shape[0])
    scp = {k: v[perm] for k, v in sc.items()}
    r = oracle.gaussian_uncertainty(sc, cam, IDENTITY, D)
    rp = oracle.gaussian_uncertainty(scp, cam, IDENTITY, D)
    # equal-depth ties could reorder; the parity scene has none
    np.testing.assert_allclose(rp["sum"], r["sum"][perm], rtol=1e-12)
    assert np.array_equal(rp["count"], r["count"][perm])


def test_nu_and_pruning_rule():
    S = np.array([0.0, 0.3, 0.05, 1.0, 0.2])
    M = np.array([0, 10, 1, 100, 4])
    nu = oracle.nu_from_sums(S, M)
    np.testing.assert_allclose(nu, [0.0, 0.03, 0.05, 0.01, 0.05])
    o = np.array([2.0, 2.0, -6.0, 2.0, 0.0])
    o2, mask = oracle.prune_uncertain(o, nu)
    assert mask.tolist() == [False, True, True, False, True]
    low = np.log(0.01 / 0.99)
    np.testing.assert_allclose(o2, [2.0, low, -6.0, 2.0, low])   # never raised
    # the threshold is strict
    _, m2 = oracle.prune_uncertain(o, np.array([0.025] * 5))
    assert not m2.any()
