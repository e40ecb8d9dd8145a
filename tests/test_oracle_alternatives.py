"""Pins of oracle.render_alternatives: the admissible results of a pixel
whose decisions (alpha skip and blending stop of Eq. 3-5, the median of
Eq. 7-8, the depth order of near-tied Gaussians) sit within rounding of their
thresholds.

Each hand case puts one decision exactly on its threshold and checks that
both outcomes appear, with values computed here from Eq. 3-9 by hand; the
scene-level tests tie the unbranched walk to oracle.render.
"""
import numpy as np
import pytest

import oracle
from paper_2403_16095_amd import synth

IDENTITY = (np.eye(3), np.zeros(3))
CAM = synth.SMALL_CAMERA            # fx = fy = 60, centre (32, 24)
CENTRE = 24 * CAM["width"] + 32     # the pixel a Gaussian on the optical axis is centred on
DM, OM = 1e-4, 1.2e-7


def logit(p):
    return np.log(p / (1.0 - p))


def on_axis(zs, opacities, colours, log_scale=-2.0):
    """Isotropic Gaussians on the optical axis: G = 1 at the centre pixel, so
    alpha there is the opacity itself (capped at 0.99)."""
    n = len(zs)
    return dict(means=np.array([[0.0, 0.0, z] for z in zs]), log_scales=np.full((n, 3), log_scale),
                quats=np.tile([1.0, 0.0, 0.0, 0.0], (n, 1)), opacity_logits=logit(np.asarray(opacities, float)),
                rgb=np.asarray(colours, float))


def alternatives(sc, px=(CENTRE,), dm=DM, om=OM, dobs=None):
    alts, count = oracle.render_alternatives(sc, CAM, IDENTITY, dobs, list(px), dm, om)
    return alts, count


def as_set(alts, count):
    return sorted(tuple(np.round(a, 12)) for a in alts[:count])


def blend(entries):
    """Eq. 3-9 by hand over (alpha, colour, depth) in order: colour, depth,
    opacity, median depth, final T (the walk is assumed not to stop)."""
    T, C, D, O, med = 1.0, np.zeros(3), 0.0, 0.0, 0.0
    for a, c, d in entries:
        w = a * T
        C, D, O = C + w * np.asarray(c), D + w * d, O + w
        if med == 0.0 and T * (1 - a) < 0.5:
            med = d
        T *= 1 - a
    return C, D, O, med, T


def row(C, D, O, med, T, unc=0.0):
    return tuple(np.round([*C, D, O, med, unc, T], 12))


def test_exact_depth_tie_gives_both_orders():
    c1, c2 = [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]
    sc = on_axis([2.0, 2.0], [0.6, 0.3], [c1, c2])
    alts, count = alternatives(sc)
    expect = sorted([row(*blend([(0.6, c1, 2.0), (0.3, c2, 2.0)])), row(*blend([(0.3, c2, 2.0), (0.6, c1, 2.0)]))])
    assert count[0] == 2 and as_set(alts[0], 2) == expect
    # without the order margin only the (depth, index) order remains
    alts, count = alternatives(sc, om=0.0)
    assert count[0] == 1 and as_set(alts[0], 1) == [row(*blend([(0.6, c1, 2.0), (0.3, c2, 2.0)]))]


def test_alpha_on_the_skip_threshold_gives_both_outcomes():
    a1 = (1.0 / 255.0) * (1.0 + 1e-9)
    c1, c2 = [0.2, 0.4, 0.6], [0.9, 0.1, 0.3]
    sc = on_axis([2.0, 3.0], [a1, 0.4], [c1, c2])
    alts, count = alternatives(sc)
    expect = sorted([row(*blend([(0.4, c2, 3.0)])), row(*blend([(a1, c1, 2.0), (0.4, c2, 3.0)]))])
    assert count[0] == 2 and as_set(alts[0], 2) == expect
    alts, count = alternatives(sc, dm=0.0)
    assert count[0] == 1 and as_set(alts[0], 1) == [row(*blend([(a1, c1, 2.0), (0.4, c2, 3.0)]))]


def test_transmittance_on_the_stop_threshold_gives_both_outcomes():
    """Two capped Gaussians (alpha 0.99) take T to 0.01 * 0.01 = 1e-4, the stop
    threshold: the walk may stop before the second or blend it (and then stop
    before the third, at T = 5e-5)."""
    cA, cB, cC = [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]
    sc = on_axis([2.0, 2.5, 3.0], [0.995, 0.995, 0.5], [cA, cB, cC])
    alts, count = alternatives(sc)
    only_a = row(*blend([(0.99, cA, 2.0)]))
    a_and_b = row(*blend([(0.99, cA, 2.0), (0.99, cB, 2.5)]))
    assert count[0] == 2 and as_set(alts[0], 2) == sorted([only_a, a_and_b])
    ref = oracle.render(sc, CAM, IDENTITY, pixels=[CENTRE], candidates=0)
    got = row(ref["color"][:, 0], ref["depth"][0], ref["opacity"][0], ref["depth_median"][0], ref["t_final"][0])
    assert got in (only_a, a_and_b)


def test_median_on_the_half_threshold_gives_both_outcomes():
    """alpha = 1/2 takes T exactly to 0.5: the first Gaussian may or may not be
    the median (strict < 0.5, Eq. 8); if not, the next blended one is."""
    c1, c2 = [0.3, 0.3, 0.3], [0.7, 0.2, 0.1]
    sc = on_axis([2.0, 3.5], [0.5, 0.3], [c1, c2])
    alts, count = alternatives(sc)
    C, D, O, _, T = blend([(0.5, c1, 2.0), (0.3, c2, 3.5)])
    assert count[0] == 2 and as_set(alts[0], 2) == sorted([row(C, D, O, 2.0, T), row(C, D, O, 3.5, T)])


def test_uncertainty_follows_each_alternative():
    """Eq. 10 against a sensor depth, on both orders of an exact tie."""
    c1, c2 = [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]
    sc = on_axis([2.0, 2.0], [0.6, 0.3], [c1, c2])
    D = np.full((CAM["height"], CAM["width"]), 2.75)
    alts, count = alternatives(sc, dobs=D)
    assert count[0] == 2
    np.testing.assert_allclose(alts[0, :2, 6], (0.6 + 0.4 * 0.3) * 0.75 ** 2, rtol=1e-14)


@pytest.fixture(scope="module")
def config1():
    return synth.uniform_box_scene(0, 2000), synth.random_targets(1000, CAM)[1]


def test_without_margins_every_pixel_has_the_render_alone(config1):
    sc, td = config1
    px = np.arange(CAM["width"] * CAM["height"])
    alts, count = alternatives(sc, px, dm=0.0, om=0.0, dobs=td)
    ref = oracle.render(sc, CAM, IDENTITY, td)
    assert (count == 1).all()
    want = np.stack([ref["color"][0].ravel(), ref["color"][1].ravel(), ref["color"][2].ravel(), ref["depth"].ravel(),
                     ref["opacity"].ravel(), ref["depth_median"].ravel(), ref["uncertainty"].ravel(),
                     ref["t_final"].ravel()], 1)
    assert np.array_equal(alts[:, 0, :], want)


def test_every_pixel_keeps_the_render_among_its_alternatives(config1):
    """The walk that takes every decision as float64 does is one of the
    alternatives; pixels whose decisions all clear the margins (by
    oracle.render's own margin maps) have no other result."""
    sc, td = config1
    px = np.arange(CAM["width"] * CAM["height"])
    alts, count = alternatives(sc, px, dobs=td)
    assert (count >= 1).all() and (count <= 64).all()
    ref = oracle.render(sc, CAM, IDENTITY, td)
    want = np.stack([ref["color"][0].ravel(), ref["color"][1].ravel(), ref["color"][2].ravel(), ref["depth"].ravel(),
                     ref["opacity"].ravel(), ref["depth_median"].ravel(), ref["uncertainty"].ravel(),
                     ref["t_final"].ravel()], 1)
    for k in range(px.size):
        assert (np.abs(alts[k, :count[k]] - want[k]).max(1) == 0).any(), k
    clear = ((ref["decision_margin"] >= DM) & (ref["order_margin"] >= OM) & (ref["stop_order_margin"] >= OM)).ravel()
    for k in np.nonzero(clear)[0]:
        assert np.array_equal(alts[k, :count[k]], np.repeat(want[k][None], count[k], 0)), k
    assert (count[~clear] >= 1).all()


def test_candidate_lists_give_the_brute_force_alternatives(config1):
    sc, td = config1
    rng = np.random.default_rng(2)
    px = rng.choice(CAM["width"] * CAM["height"], 300, replace=False)
    a1, c1 = oracle.render_alternatives(sc, CAM, IDENTITY, td, px, 1e-2, 1e-3, candidates=1)
    a0, c0 = oracle.render_alternatives(sc, CAM, IDENTITY, td, px, 1e-2, 1e-3, candidates=0)
    assert np.array_equal(c0, c1)
    for k in range(px.size):
        assert as_set(a0[k], min(c0[k], 64)) == as_set(a1[k], min(c1[k], 64))


def test_too_many_alternatives_are_reported():
    """Twelve Gaussians at one depth: more orders than the list holds."""
    sc = on_axis([2.0] * 12, [0.2] * 12, [[k / 12, 0.5, 1 - k / 12] for k in range(12)])
    alts, count = oracle.render_alternatives(sc, CAM, IDENTITY, None, [CENTRE], DM, OM, max_alts=8)
    assert count[0] == 9


def test_map_checker_takes_admissible_results_and_catches_planted_errors(config1):
    """helpers.check_maps (the GPU parity checker) on oracle maps: the
    oracle's own render passes; so does the other order of an exact depth
    tie (an admissible result); a clear pixel off by 2e-4 and an ambiguous
    pixel matching none of its alternatives fail."""
    from helpers import check_maps, grad_parity
    sc, td = config1
    ref = oracle.render(sc, CAM, IDENTITY, td)
    res = check_maps(ref, sc, CAM, IDENTITY, td, label="oracle vs itself")
    assert res["worst_clear"] == 0.0 and res["worst_alt"] == 0.0
    clear = np.nonzero(((ref["decision_margin"] >= 1e-4) & (ref["order_margin"] >= 1.2e-7)
                        & (ref["stop_order_margin"] >= 1.2e-7)).ravel())[0]
    bad = {k: (None if v is None else v.copy()) for k, v in ref.items()}
    bad["depth"].reshape(-1)[clear[7]] += 2e-4
    with pytest.raises(AssertionError):
        check_maps(bad, sc, CAM, IDENTITY, td, label="planted clear-pixel error")
    # an exact depth tie: the second order is admissible, a value off both is not
    c1, c2 = [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]
    tie = on_axis([2.0, 2.0], [0.6, 0.3], [c1, c2])
    r2 = oracle.render(tie, CAM, IDENTITY)
    other = blend([(0.3, c2, 2.0), (0.6, c1, 2.0)])
    swapped = {k: (None if v is None else v.copy()) for k, v in r2.items()}
    for c in range(3):
        swapped["color"][c].reshape(-1)[CENTRE] = other[0][c]
    assert not np.allclose(swapped["color"], r2["color"], atol=1e-4)
    check_maps(swapped, tie, CAM, IDENTITY, label="other order of a tie")
    swapped["color"][0].reshape(-1)[CENTRE] += 1e-2
    with pytest.raises(AssertionError):
        check_maps(swapped, tie, CAM, IDENTITY, label="planted ambiguous-pixel error")
    # the gradient report: the binding relative L2 bar and the element-wise count
    g = np.random.default_rng(3).standard_normal(1000)
    assert grad_parity("g", g, g) == 0.0
    assert grad_parity("g", g * (1 + 5e-4), g) == 0.0
    assert 0.0 < grad_parity("g", g + 1e-2 * (np.arange(1000) == 3), g) <= 1e-3
    with pytest.raises(AssertionError):
        grad_parity("g", g * 1.01, g)
