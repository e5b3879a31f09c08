"""Pins of the oracle's residual-weighted sampler (Supp. E q_residual, eq. 16;
stratified per tile as in Sec. 4.4; importance weights of eq. 11-12).

None of these restates the sampler's formula: they check a closed-form
probability, the Horvitz-Thompson identity that any correct draw/weight pair
satisfies, and the degenerate cases."""
import math

import numpy as np

from oracle.sampling import draw_uniforms, sample_residual


def tile_pattern(T, pattern):
    return np.broadcast_to(np.asarray(pattern, np.float64), (1, T, 256)).copy()


def test_uniform_scores_give_uniform_draws_and_weight_256_over_k():
    """Equal residuals: q = 1/256 in the tile, so w = 256/k exactly and the
    draws are uniform over the 256 pixels (chi-square, 255 dof)."""
    T, k = 2000, 13
    pix, w, _ = sample_residual(3, 0, [4], T, k, np.full((1, T, 256), 0.7))
    assert np.allclose(w, 256.0 / k, rtol=1e-12)
    counts = np.bincount(pix.reshape(-1), minlength=256)
    e = pix.size / 256
    chi2 = float(((counts - e) ** 2 / e).sum())
    assert chi2 < 255 + 6 * math.sqrt(2 * 255)


def test_single_hot_pixel_has_closed_form_probability():
    """One pixel with |r| = ln 255 and 255 pixels with |r| = 0: the hot pixel
    holds e^{ln 255} / (e^{ln 255} + 255) = 1/2 of the mass."""
    T, k = 4000, 13
    sc = np.zeros(256)
    sc[77] = math.log(255.0)
    pix, w, _ = sample_residual(5, 2, [1], T, k, tile_pattern(T, sc))
    frac = float(np.mean(pix == 77))
    n = pix.size
    assert abs(frac - 0.5) < 5 * math.sqrt(0.25 / n)
    # its weight is 1 / (k * 1/2), the others 1 / (k * 1/510)
    assert np.allclose(w[pix == 77], 2.0 / k, rtol=1e-12)
    assert np.allclose(w[pix != 77], 510.0 / k, rtol=1e-12)


def test_horvitz_thompson_estimate_is_unbiased():
    """For any f, E[sum_j w_j f(p_j)] = sum_p f(p) when w = 1/(k q) of the
    distribution the draws follow; checked over 6000 independent tiles."""
    rng = np.random.default_rng(0)
    T, k = 6000, 8
    sc = rng.uniform(0, 3, size=256)
    f = rng.normal(size=256) + 2.0
    pix, w, _ = sample_residual(11, 1, [0], T, k, tile_pattern(T, sc))
    est = (w * f[pix.astype(np.int64)]).sum(axis=-1).reshape(-1)
    se = est.std(ddof=1) / math.sqrt(est.size)
    assert abs(est.mean() - f.sum()) < 5 * se


def test_draws_are_counter_based_and_independent_of_scores():
    """The uniform numbers depend on (seed, iteration, camera, tile, slot)
    only; they are exact 24-bit fractions in [0, 1)."""
    u = draw_uniforms(9, 4, [2, 7], 5, 13)
    assert u.shape == (2, 5, 13) and u.min() >= 0 and u.max() < 1
    assert np.all(u * 2 ** 24 == np.floor(u * 2 ** 24))
    assert np.array_equal(u, draw_uniforms(9, 4, [2, 7], 5, 13))
    assert not np.array_equal(u, draw_uniforms(9, 5, [2, 7], 5, 13))
    assert not np.array_equal(u[0], u[1])


def test_dominant_pixel_is_always_drawn_with_weight_one_over_k():
    """A residual far above the rest (|r| = 800 vs 0) holds all the mass:
    every draw picks it, with weight 1/k; no overflow."""
    T, k = 50, 13
    sc = np.zeros(256)
    sc[200] = 800.0
    pix, w, _ = sample_residual(1, 0, [0], T, k, tile_pattern(T, sc))
    assert np.all(pix == 200)
    assert np.allclose(w, 1.0 / k)


def test_margin_is_distance_to_interval_ends():
    """The margin is at most half the chosen pixel's probability and the draw
    lies inside its interval of the cumulative distribution."""
    rng = np.random.default_rng(2)
    T, k = 40, 13
    sc = rng.uniform(0, 2, size=(1, T, 256))
    pix, w, m = sample_residual(4, 0, [3], T, k, sc)
    q = 1.0 / (k * w)
    assert np.all(m >= 0) and np.all(m <= q / 2 + 1e-15)
