"""Pins of the oracle's SSIM residual with the diagonal approximation
(Supp. B; Sec. 6): SSIM's fixed values (identical images, constant patches),
a brute-force window sum at single pixels, the diagonal derivative against
central differences in the centre pixel, and the Gauss-Newton right-hand side
against the exact gradient of the objective where the diagonal approximation
is exact (a 1 x 1 window)."""
import math

import numpy as np

from oracle import Oracle
from oracle.ssim import C1, C2, gaussian_window, residual_and_weights, ssim_terms
from paper_2504_12905_amd import synth


def rand_images(seed, V=2, H=24, W=20):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, 1, (V, H, W, 3)), rng.uniform(0, 1, (V, H, W, 3))


def test_identical_images_have_ssim_one_and_zero_slope():
    x, _ = rand_images(0)
    s, d = ssim_terms(x, x)
    np.testing.assert_allclose(s, 1.0, atol=1e-12)
    np.testing.assert_allclose(d, 0.0, atol=1e-10)


def test_constant_patches_closed_form():
    """Interior pixels of constant images a and b: SSIM = (2ab + C1)/(a^2 + b^2 + C1)."""
    a, b = 0.3, 0.7
    x = np.full((1, 30, 30, 3), a)
    y = np.full((1, 30, 30, 3), b)
    s, _ = ssim_terms(x, y)
    np.testing.assert_allclose(s[0, 5:25, 5:25], (2 * a * b + C1) / (a * a + b * b + C1), rtol=1e-12)


def brute_ssim(x, y, v, py, px, c):
    """SSIM at one pixel from explicit window sums (zero outside the image)."""
    win = gaussian_window()
    H, W = x.shape[1:3]
    sx = sy = sxx = syy = sxy = 0.0
    for dy in range(-5, 6):
        for dx in range(-5, 6):
            q, r = py + dy, px + dx
            if 0 <= q < H and 0 <= r < W:
                g = win[dy + 5, dx + 5]
                a, b = x[v, q, r, c], y[v, q, r, c]
                sx += g * a
                sy += g * b
                sxx += g * a * a
                syy += g * b * b
                sxy += g * a * b
    vx, vy, cxy = sxx - sx * sx, syy - sy * sy, sxy - sx * sy
    return ((2 * sx * sy + C1) * (2 * cxy + C2)) / ((sx * sx + sy * sy + C1) * (vx + vy + C2))


def test_window_sums_match_brute_force():
    x, y = rand_images(1)
    s, _ = ssim_terms(x, y)
    for (v, py, px, c) in [(0, 0, 0, 0), (1, 12, 9, 2), (0, 23, 19, 1), (1, 3, 17, 0), (0, 11, 2, 2)]:
        assert math.isclose(s[v, py, px, c], brute_ssim(x, y, v, py, px, c), rel_tol=1e-12)


def test_diagonal_derivative_matches_central_differences():
    """d SSIM_c(p) / d x_pc by moving pixel p only (interior and border)."""
    x, y = rand_images(2)
    _, d = ssim_terms(x, y)
    h = 1e-6
    for (v, py, px, c) in [(0, 10, 10, 0), (1, 0, 5, 1), (0, 23, 0, 2), (1, 7, 19, 0)]:
        xp, xm = x.copy(), x.copy()
        xp[v, py, px, c] += h
        xm[v, py, px, c] -= h
        fd = (brute_ssim(xp, y, v, py, px, c) - brute_ssim(xm, y, v, py, px, c)) / (2 * h)
        assert math.isclose(d[v, py, px, c], fd, rel_tol=1e-6, abs_tol=1e-9)


def test_rhs_is_half_gradient_where_the_diagonal_is_exact():
    """With a 1 x 1 window SSIM(p) depends on pixel p alone, so the
    approximation is exact: b = J^T (w (r + s delta rho)) must equal half the
    gradient of E = sum w (r^2 + s rho^2), checked along random directions by
    central differences of E (FP64 oracle renders, every pixel, w = 1)."""
    tw = synth.tiny(n=4, sh_degree=0, n_views=1, size=32, seed=3)
    orc = Oracle(tw.n, 0, tw.beta_init, tw.cams, tw.width, tw.height)
    target = Oracle(tw.n, 0, tw.beta_gt, tw.cams, tw.width, tw.height).render_image()

    def energy(beta):
        o = Oracle(tw.n, 0, beta, tw.cams, tw.width, tw.height)
        img = o.render_image()
        s1, _ = ssim_terms(img, target, size=1)
        return float(((img - target) ** 2).sum() + 0.2 * ((1 - s1) ** 2).sum())

    img = orc.render_image()
    u, _, _ = residual_and_weights(orc, img, target, np.ones(orc.S), size=1)
    b = orc.vjp(u)
    rng = np.random.default_rng(4)
    for _ in range(3):
        p = rng.normal(size=orc.P)
        p /= np.linalg.norm(p)
        h = 1e-5
        b0 = np.asarray(tw.beta_init, np.float64)
        fd = (energy(b0 + h * p) - energy(b0 - h * p)) / (2 * h)
        assert math.isclose(2 * float(b @ p), fd, rel_tol=1e-5, abs_tol=1e-9)


def test_channel_weighted_operator_against_dense_jacobian():
    """J^T diag(wc) J p + lambda p with per-channel weights equals the dense
    product from the dual-number Jacobian columns (tiny scene, every pixel)."""
    tw = synth.tiny(n=3, sh_degree=1, n_views=1, size=32, seed=5)
    orc = Oracle(tw.n, 1, tw.beta_init, tw.cams, tw.width, tw.height)
    orc.set_samples(256)
    rng = np.random.default_rng(6)
    wc = rng.uniform(0.5, 2.0, size=(orc.S, 3))
    J = np.stack([orc.jvp(e).reshape(-1) for e in np.eye(orc.P)], axis=1)   # [3S, P]
    p = rng.normal(size=orc.P)
    ref = J.T @ (wc.reshape(-1) * (J @ p)) + 0.1 * p
    orc.set_channel_weights(wc)
    np.testing.assert_allclose(orc.gn(p, 0.1), ref, rtol=1e-10, atol=1e-12)
    orc.set_channel_weights(None)
    np.testing.assert_allclose(orc.gn(p, 0.1), J.T @ (J @ p) + 0.1 * p, rtol=1e-10, atol=1e-12)


def _ssim_objective(tw, beta, target, s=0.2):
    img = Oracle(tw.n, tw.sh_degree, beta, tw.cams, tw.width, tw.height).render_image()
    ssim, _ = ssim_terms(img, target)
    return float(((img - target) ** 2).sum() + s * ((1 - ssim) ** 2).sum())


def test_lm_step_with_ssim_solves_the_weighted_system_and_descends():
    """The oracle's LM step with the SSIM residual: run to convergence, its x
    solves the dense system (J^T diag(wc) J + lambda I) x = J^T u built from
    the dual-number Jacobian columns; its preconditioner diagonal is the
    column sums of wbar J^2; and a short step along -x lowers the SSIM + colour
    objective (tiny scene, every pixel)."""
    from oracle.solver import lm_step
    tw = synth.tiny(n=3, sh_degree=1, n_views=1, size=32, seed=7)
    target = Oracle(tw.n, 1, tw.beta_gt, tw.cams, tw.width, tw.height).render_image()
    beta = np.asarray(tw.beta_init, np.float32)
    orc = Oracle(tw.n, 1, beta, tw.cams, tw.width, tw.height)
    lam = 0.1
    beta_next, info = lm_step(tw.n, 1, beta, tw.cams, target.astype(np.float32), [0], tw.width, tw.height,
                              256, 0, 0, lam, orc.P, ssim_weight=0.2)
    orc.set_samples(256)
    img = orc.render_image()
    u, wc, wbar = residual_and_weights(orc, img, target, np.ones(orc.S), s=0.2)
    J = np.stack([orc.jvp(e).reshape(-1) for e in np.eye(orc.P)], axis=1)   # [3S, P]
    A = J.T @ (wc.reshape(-1)[:, None] * J) + lam * np.eye(orc.P)
    x = np.linalg.solve(A, J.T @ u.reshape(-1))
    np.testing.assert_allclose(info["x"], x, rtol=1e-5, atol=1e-7 * np.abs(x).max())
    np.testing.assert_allclose(info["diag"], (np.repeat(wbar, 3)[:, None] * J ** 2).sum(axis=0),
                               rtol=1e-6, atol=1e-12)
    assert info["b"] @ info["x"] > 0
    e0 = _ssim_objective(tw, beta, target)
    e1 = _ssim_objective(tw, (beta.astype(np.float64) - 0.05 * info["x"]).astype(np.float32), target)
    assert e1 < e0
