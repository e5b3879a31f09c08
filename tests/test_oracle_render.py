"""Pins of the oracle's alpha-blended render (eq. 3, Alg. 2) by closed forms and brute force."""
import math

import numpy as np
import pytest

from oracle import DEFAULT_OPTS, Oracle
from paper_2504_12905_amd import synth

from test_oracle_geometry import axis_camera, one_gaussian_scene

LOWPASS = DEFAULT_OPTS["lowpass"]      # the FP32 low-pass 0.3 px^2 of the options block
ALPHA_MIN = DEFAULT_OPTS["alpha_min"]  # the FP32 alpha floor 1/255


def test_single_gaussian_closed_form():
    f, W = 40.0, 32
    sigma, o_logit = 0.1, 0.7
    rgb = np.array([0.9, 0.3, 0.1])
    n, beta = one_gaussian_scene([0, 0, 0], [math.log(sigma)] * 3, [1, 0, 0, 0], o_logit, rgb)
    orc = Oracle(n, 0, beta, axis_camera(f, W, W), W, W)
    img = orc.render_image()[0]
    s2 = (f * sigma / 3.0) ** 2 + LOWPASS
    r = math.ceil(3 * math.sqrt(s2))
    op = 1 / (1 + math.exp(-o_logit))
    ys, xs = np.mgrid[0:W, 0:W]
    d2 = (xs + 0.5 - W / 2) ** 2 + (ys + 0.5 - W / 2) ** 2
    a = np.minimum(op * np.exp(-0.5 * d2 / s2), 0.99)
    a[a < ALPHA_MIN] = 0.0
    # tiles outside the 3-sigma rectangle are not rendered
    tx0, tx1 = math.floor((W / 2 - r) / 16), math.floor((W / 2 + r) / 16)
    in_rect = ((xs // 16 >= tx0) & (xs // 16 <= tx1) & (ys // 16 >= tx0) & (ys // 16 <= tx1))
    ref = (a * in_rect)[..., None] * rgb
    np.testing.assert_allclose(img, ref, rtol=1e-12, atol=1e-15)


def test_two_gaussians_over_operator():
    f, W = 40.0, 32
    rgb1, rgb2 = np.array([1.0, 0.0, 0.2]), np.array([0.1, 0.8, 0.3])
    n, beta = one_gaussian_scene([[0, 0, 0], [0.01, -0.02, 0.5]], [math.log(0.1)] * 3, [1, 0, 0, 0],
                                 0.3, [0, 0, 0])
    K = 1
    sh = beta[synth.seg(n, "sh", 0)].reshape(K, 3, n)
    sh[0, :, 0] = (rgb1 - 0.5) / 0.28209479177387814
    sh[0, :, 1] = (rgb2 - 0.5) / 0.28209479177387814
    beta[synth.seg(n, "sh", 0)] = sh.reshape(-1)
    orc = Oracle(n, 0, beta, axis_camera(f, W, W), W, W)
    img = orc.render_image()[0]
    pr = orc.projection()["rec"][0]

    def alpha(rec, x, y):
        dx, dy = rec[0] - x, rec[1] - y
        s = -0.5 * (rec[2] * dx * dx + rec[4] * dy * dy) - rec[3] * dx * dy
        a = min(0.99, rec[5] * math.exp(s))
        return 0.0 if a < ALPHA_MIN else a

    for (x, y) in [(15, 15), (16, 17), (13, 18), (18, 12)]:
        a1, a2 = alpha(pr[0], x + 0.5, y + 0.5), alpha(pr[1], x + 0.5, y + 0.5)
        ref = rgb1 * a1 + rgb2 * a2 * (1 - a1)
        np.testing.assert_allclose(img[y, x], ref, rtol=1e-12)


def test_transmittance_stop_three_layers():
    """Opacity 0.95 centred on a pixel: T 1 -> 0.05 -> 0.0025 -> 1.25e-4; a fourth
    layer would take T to 6.25e-6 < 1e-4, so exactly three layers are blended."""
    f, W = 32.0, 32
    depths = [3.0, 3.1, 3.2, 3.3]
    # camera at z = -3: a mean at world z has depth z + 3; centre on pixel (16, 16)
    means = [[0.5 * (d) / f, 0.5 * (d) / f, d - 3.0] for d in depths]
    n, beta = one_gaussian_scene(means, [math.log(0.2)] * 3, [1, 0, 0, 0], math.log(19.0), [0.8, 0.6, 0.4])
    orc = Oracle(n, 0, beta, axis_camera(f, W, W), W, W)
    orc.set_samples(256)
    out = orc.render()
    v, x, y = orc.pixel_coords()
    i = int(np.where((x == 16) & (y == 16))[0][0])
    assert out["n_contrib"][i] == 3
    assert out["T"][i] == pytest.approx(0.05 ** 3, rel=1e-9)
    np.testing.assert_allclose(out["C"][i], np.array([0.8, 0.6, 0.4]) * (1 - 0.05 ** 3), rtol=1e-9)


def brute_force_pixel(rec, order, x, y):
    T, Cc = 1.0, np.zeros(3)
    for g in order:
        r = rec[g]
        dx, dy = r[0] - x, r[1] - y
        s = -0.5 * (r[2] * dx * dx + r[4] * dy * dy) - r[3] * dx * dy
        if s > 0:
            continue
        a = min(0.99, r[5] * math.exp(s))
        if a < ALPHA_MIN:
            continue
        if T * (1 - a) < 1e-4:
            break
        Cc += r[6:9] * a * T
        T *= 1 - a
    return Cc, T


def test_tile_render_matches_brute_force_pixels():
    w = synth.config0()
    orc = Oracle(w.n, 0, w.beta_gt, w.cams, w.width, w.height)
    pr = orc.projection()
    img = orc.render_image()
    rng = np.random.default_rng(3)
    for _ in range(60):
        v, x, y = rng.integers(0, orc.V), rng.integers(0, w.width), rng.integers(0, w.height)
        tx, ty = x // 16, y // 16
        members = [g for g in range(orc.n) if pr["visible"][v, g]
                   and pr["rect"][v, g, 0] <= tx < pr["rect"][v, g, 2]
                   and pr["rect"][v, g, 1] <= ty < pr["rect"][v, g, 3]]
        members.sort(key=lambda g: (pr["depth"][v, g], g))
        ref, _ = brute_force_pixel(pr["rec"][v], members, x + 0.5, y + 0.5)
        np.testing.assert_allclose(img[v, y, x], ref, rtol=1e-12, atol=1e-15)


def test_samples_select_pixels():
    w = synth.config0()
    orc = Oracle(w.n, 0, w.beta_gt, w.cams, w.width, w.height)
    full = orc.render_image()
    rng = np.random.default_rng(0)
    k = 13
    pix = np.stack([np.sort(rng.choice(256, k, replace=False)) for _ in range(orc.V * orc.T)])
    orc.set_samples(k, pix, np.full(pix.shape, 256 / k, np.float32))
    out = orc.render()
    v, x, y = orc.pixel_coords()
    np.testing.assert_array_equal(out["C"], full[v, y, x])


def test_decision_margin_flags_threshold_pixels():
    """A pixel whose alpha sits 1e-6 (relative) above the 1/255 floor is not
    decided at tau = 1e-4; with alpha 0.006 it is."""
    f, W = 40.0, 32
    sigma = 0.1
    s2 = (f * sigma / 3.0) ** 2 + LOWPASS
    x, y = 20, 16                        # pixel centre (20.5, 16.5), Gaussian at (16, 16)
    d2 = (x + 0.5 - W / 2) ** 2 + (y + 0.5 - W / 2) ** 2
    g = math.exp(-0.5 * d2 / s2)
    for target, expect in [((1 + 1e-6) / 255.0, False), (0.006, True)]:
        op = target / g
        n, beta = one_gaussian_scene([0, 0, 0], [math.log(sigma)] * 3, [1, 0, 0, 0], math.log(op / (1 - op)),
                                     [0.5, 0.5, 0.5])
        orc = Oracle(n, 0, beta, axis_camera(f, W, W), W, W)
        orc.set_samples(256)
        v, xs, ys = orc.pixel_coords()
        i = int(np.flatnonzero((xs == x) & (ys == y))[0])
        assert bool(orc.decided()[i]) is expect


def test_undecided_tiles_cover_a_radius_at_an_integer():
    """On the optical axis at depth 3, 3 sqrt((f sigma / 3)^2 + 0.3) is the
    footprint extent. At 16 + 1e-6 px the radius ceil() = 17 is not decided to
    within tau = 1e-4 px, an evaluation that loose may give 16: around the
    centre (32, 32) of a 64x64 image the
    radius-17 rectangle holds tiles 0..3 (32 - 17 = 15 lies in tile 0), the
    radius-16 one tiles 1..3 (the right edge 48 starts tile 3), so the flagged
    ring is every tile with tx == 0 or ty == 0; their pixels leave
    decided(tau_list=1e-4). At 16 - 1e-6 px the radius 16 may become 17: the
    same ring. At 16.5 px nothing is flagged, and at the default tau_list
    (two FP64 evaluations) the 1e-6 px cases are decided."""
    f, W = 40.0, 64
    ring = {(ty, tx) for ty in range(4) for tx in range(4) if tx == 0 or ty == 0}
    for ext, expect in [(16.0 + 1e-6, ring), (16.0 - 1e-6, ring), (16.5, set())]:
        sigma = 3.0 * math.sqrt((ext / 3.0) ** 2 - LOWPASS) / f
        n, beta = one_gaussian_scene([0, 0, 0], [math.log(sigma)] * 3, [1, 0, 0, 0], 0.5, [0.5, 0.5, 0.5])
        orc = Oracle(n, 0, beta, axis_camera(f, W, W), W, W)
        flags = orc.undecided_tiles(1e-4).reshape(W // 16, W // 16)
        assert {(int(ty), int(tx)) for ty, tx in zip(*np.nonzero(flags))} == expect
        orc.set_samples(256)
        ok = orc.decided(tau_list=1e-4).reshape(-1, 256)
        assert np.array_equal(~ok.all(axis=1), flags.reshape(-1).astype(bool)) or not expect
        assert not orc.undecided_tiles().any()


def test_only_tiles_setup_keeps_those_lists_and_renders():
    """An oracle that builds the lists of some tiles only has exactly the full
    oracle's lists and render there (and empty lists elsewhere)."""
    w = synth.config0()
    full = Oracle(w.n, 0, w.beta_init, w.cams, w.width, w.height)
    mask = (np.arange(full.V * full.T) % 3 == 1).astype(np.uint8)
    part = Oracle(w.n, 0, w.beta_init, w.cams, w.width, w.height, only_tiles=mask)
    ts_f, ids_f = full.lists()
    ts_p, ids_p = part.lists()
    for t in range(full.V * full.T):
        got = ids_p[ts_p[t]:ts_p[t + 1]]
        assert list(got) == (list(ids_f[ts_f[t]:ts_f[t + 1]]) if mask[t] else [])
    on = np.repeat(mask.astype(bool), 256)
    assert np.array_equal(part.render()["C"][on], full.render()["C"][on])
