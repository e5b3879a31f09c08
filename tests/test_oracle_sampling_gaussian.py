"""Pins of the oracle's contribution-weighted sampler (Supp. E q_Gaussian,
eq. 17; stratified per tile as in Sec. 4.4; importance weights of eq. 11-12)
and of the per-pixel contributor count G_p it draws from.

None of these restates the sampler's formula: a closed-form probability, the
Horvitz-Thompson identity, the degenerate cases (empty tile, zero-count
pixels), a brute-force count of blended Gaussians, and the closed-form count
of a stack of opaque layers."""
import math

import numpy as np

from oracle import Oracle
from oracle.sampling import sample_gaussian
from oracle.solver import contributor_counts
from test_oracle_geometry import axis_camera, one_gaussian_scene


def tile_pattern(T, pattern):
    return np.broadcast_to(np.asarray(pattern, np.float64), (1, T, 256)).copy()


def test_closed_form_probability_and_weights():
    """Pixel 5 with G = 3 and pixel 200 with G = 1, the rest 0: q = 3/4 and
    1/4, weights Z/(k G) = 4/(3k) and 4/k; no other pixel is ever drawn."""
    T, k = 5000, 16
    G = np.zeros(256)
    G[5], G[200] = 3, 1
    pix, w = sample_gaussian(7, 3, [2], T, k, tile_pattern(T, G))
    assert set(np.unique(pix).tolist()) == {5, 200}
    frac = float(np.mean(pix == 5))
    assert abs(frac - 0.75) < 5 * math.sqrt(0.75 * 0.25 / pix.size)
    assert np.allclose(w[pix == 5], 4.0 / (3 * k), rtol=1e-15)
    assert np.allclose(w[pix == 200], 4.0 / k, rtol=1e-15)


def test_horvitz_thompson_estimate_is_unbiased():
    """E[sum_j w_j f(p_j)] = sum over pixels with G_p > 0 of f(p)."""
    rng = np.random.default_rng(1)
    T, k = 6000, 8
    G = rng.integers(0, 9, size=256).astype(np.float64)
    f = rng.normal(size=256) + 2.0
    pix, w = sample_gaussian(11, 0, [0], T, k, tile_pattern(T, G))
    est = (w * f[pix.astype(np.int64)]).sum(axis=-1).reshape(-1)
    se = est.std(ddof=1) / math.sqrt(est.size)
    assert abs(est.mean() - f[G > 0].sum()) < 5 * se


def test_empty_tile_is_sampled_uniformly():
    """No contribution anywhere in the tile: q = 1/256, weight 256/k, draws
    uniform (chi-square, 255 dof)."""
    T, k = 2000, 13
    pix, w = sample_gaussian(3, 1, [4], T, k, np.zeros((1, T, 256)))
    assert np.allclose(w, 256.0 / k, rtol=1e-15)
    counts = np.bincount(pix.reshape(-1), minlength=256)
    e = pix.size / 256
    assert float(((counts - e) ** 2 / e).sum()) < 255 + 6 * math.sqrt(2 * 255)


def test_uniform_counts_match_uniform_weights():
    """Equal counts: q = 1/256, weight 256/k exactly."""
    pix, w = sample_gaussian(5, 2, [1, 3], 40, 26, np.full((2, 40, 256), 17.0))
    assert np.allclose(w, 256.0 / 26, rtol=1e-15)


def test_draws_follow_the_counter():
    """Same (seed, iteration, camera) -> same draws; another iteration -> others."""
    G = np.random.default_rng(3).integers(1, 5, size=(2, 30, 256)).astype(np.float64)
    a = sample_gaussian(9, 4, [2, 7], 30, 13, G)[0]
    assert np.array_equal(a, sample_gaussian(9, 4, [2, 7], 30, 13, G)[0])
    assert not np.array_equal(a, sample_gaussian(9, 5, [2, 7], 30, 13, G)[0])


def test_contributor_count_of_opaque_stack():
    """Four Gaussians centred on pixel (16, 16) at depths 3.0..3.3, each with
    alpha 0.95 there: T goes 1 -> 0.05 -> 0.0025 -> 1.25e-4, and the fourth
    would take it to 6.25e-6 < 1e-4, so exactly 3 are blended at the centre."""
    f, W = 40.0, 32
    depths = [3.0, 3.1, 3.2, 3.3]
    means = [[0.5 * d / f, 0.5 * d / f, d - 3.0] for d in depths]
    n, beta = one_gaussian_scene(means, [math.log(0.2)] * 3, [1, 0, 0, 0], math.log(19.0), [0.8, 0.6, 0.4])
    orc = Oracle(n, 0, beta, axis_camera(f, W, W), W, W)
    G = contributor_counts(orc)
    v, x, y = orc.pixel_coords()
    i = int(np.flatnonzero((x == 16) & (y == 16))[0])
    assert G.reshape(-1)[i] == 3


def test_contributor_counts_match_brute_force():
    """G_p against a brute-force count: every visible Gaussian in depth order,
    opacity test, transmittance stop (the render's own rules, written out per
    pixel from the projection)."""
    rng = np.random.default_rng(4)
    n, W, f = 12, 32, 40.0
    means = np.column_stack([rng.uniform(-0.3, 0.3, n), rng.uniform(-0.3, 0.3, n), rng.uniform(-0.5, 0.5, n)])
    beta_n, beta = one_gaussian_scene(means.tolist(), [math.log(0.15)] * 3, [1, 0, 0, 0], 0.5, [0.5, 0.5, 0.5])
    orc = Oracle(beta_n, 0, beta, axis_camera(f, W, W), W, W)
    pr = orc.projection()
    G = contributor_counts(orc).reshape(-1)
    v, xs, ys = orc.pixel_coords()
    order = sorted(range(n), key=lambda g: (pr["depth"][0, g], g))
    amin, amax, tmin = orc_opts()
    for i in range(0, xs.size, 7):
        x, y = xs[i] + 0.5, ys[i] + 0.5
        tx, ty = int(xs[i]) // 16, int(ys[i]) // 16
        T, cnt = 1.0, 0
        for g in order:
            rc = pr["rect"][0, g]
            if not (pr["visible"][0, g] and rc[0] <= tx < rc[2] and rc[1] <= ty < rc[3]):
                continue
            u, vv, A, B, C, o = pr["rec"][0, g, :6]
            dx, dy = u - x, vv - y
            s = -0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy
            if s > 0:
                continue
            a = min(amax, o * math.exp(s))
            if a < amin:
                continue
            if T * (1 - a) < tmin:
                break
            T *= 1 - a
            cnt += 1
        assert G[i] == cnt, (i, G[i], cnt)


def orc_opts():
    from oracle import DEFAULT_OPTS
    return DEFAULT_OPTS["alpha_min"], DEFAULT_OPTS["alpha_max"], DEFAULT_OPTS["t_min"]
