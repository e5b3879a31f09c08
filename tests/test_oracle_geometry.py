"""Pins of the oracle's geometry against closed forms, library routines and brute force.

Oracle functions covered: real SH basis, projection (eq. 1-3, EWA), tile lists.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.special import sph_harm_y

import oracle
from oracle import DEFAULT_OPTS, Oracle
from paper_2504_12905_amd import synth

LOWPASS = DEFAULT_OPTS["lowpass"]      # the FP32 low-pass 0.3 px^2 of the options block
ALPHA_MIN = DEFAULT_OPTS["alpha_min"]  # the FP32 alpha floor 1/255


def one_gaussian_scene(means, log_scales, quats, ologit, rgb, sh_degree=0, sh_rest=None):
    """beta for hand-placed Gaussians; rgb is the colour seen at DC only."""
    means = np.atleast_2d(means).astype(np.float64)
    n = means.shape[0]
    K = (sh_degree + 1) ** 2
    beta = np.zeros(synth.n_params(n, sh_degree))
    beta[synth.seg(n, "mean")] = means.T.reshape(-1)
    beta[synth.seg(n, "log_scale")] = np.broadcast_to(np.atleast_2d(log_scales), (n, 3)).T.reshape(-1)
    beta[synth.seg(n, "quat")] = np.broadcast_to(np.atleast_2d(quats), (n, 4)).T.reshape(-1)
    beta[synth.seg(n, "opacity")] = np.broadcast_to(ologit, (n,))
    sh = np.zeros((K, 3, n))
    sh[0] = (np.broadcast_to(np.atleast_2d(rgb), (n, 3)).T - 0.5) / 0.28209479177387814
    if sh_rest is not None:
        sh[1:] = sh_rest
    beta[synth.seg(n, "sh", sh_degree)] = sh.reshape(-1)
    return n, beta


def axis_camera(f, W, H, z=3.0):
    """Camera at (0, 0, -z) looking along +z, focal f, principal point at the centre."""
    c = np.zeros(16, np.float32)
    c[0:9] = np.eye(3).reshape(-1)
    c[9:12] = [0.0, 0.0, z]
    c[12:16] = [f, f, W / 2, H / 2]
    return c[None, :]


# ----------------------------------------------------------------- SH basis
def real_sh_scipy(l, m, d):
    theta = math.acos(d[2])
    phi = math.atan2(d[1], d[0])
    if m == 0:
        return float(np.real(sph_harm_y(l, 0, theta, phi)))
    y = sph_harm_y(l, abs(m), theta, phi)
    return float(math.sqrt(2.0) * (np.real(y) if m > 0 else np.imag(y)))


def test_sh_basis_matches_scipy():
    rng = np.random.default_rng(0)
    for _ in range(20):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        Y = oracle.sh_basis(3, d)
        ref = [real_sh_scipy(l, m, d) for l in range(4) for m in range(-l, l + 1)]
        np.testing.assert_allclose(Y, ref, rtol=1e-12, atol=1e-14)


def test_sh_basis_orthonormal():
    # Gauss-Legendre in cos(theta) x uniform phi integrates degree <= 6 products exactly.
    xs, ws = np.polynomial.legendre.leggauss(8)
    phis = np.linspace(0, 2 * np.pi, 16, endpoint=False)
    G = np.zeros((16, 16))
    for x, w in zip(xs, ws):
        s = math.sqrt(1 - x * x)
        for ph in phis:
            Y = oracle.sh_basis(3, np.array([s * math.cos(ph), s * math.sin(ph), x]))
            G += w * (2 * np.pi / len(phis)) * np.outer(Y, Y)
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)
    assert oracle.sh_basis(0, np.array([0, 0, 1.0]))[0] == pytest.approx(0.5 / math.sqrt(math.pi))


# ---------------------------------------------------------------- projection
def test_on_axis_isotropic_closed_form():
    f, W = 40.0, 64
    sigma = 0.1
    n, beta = one_gaussian_scene([0, 0, 0], [math.log(sigma)] * 3, [1, 0, 0, 0], 0.0, [0.2, 0.4, 0.6])
    o = Oracle(n, 0, beta, axis_camera(f, W, W), W, W)
    pr = o.projection()
    rec = pr["rec"][0, 0]
    s2 = (f * sigma / 3.0) ** 2 + LOWPASS
    np.testing.assert_allclose(rec[:2], [W / 2, W / 2], atol=1e-12)
    np.testing.assert_allclose(rec[2:5], [1 / s2, 0.0, 1 / s2], rtol=1e-12, atol=1e-15)
    assert rec[5] == pytest.approx(0.5)                      # sigmoid(0)
    np.testing.assert_allclose(rec[6:9], [0.2, 0.4, 0.6], rtol=1e-12)
    assert pr["radius"][0, 0] == math.ceil(3 * math.sqrt(s2))
    assert pr["depth"][0, 0] == np.float32(3.0)


def test_projection_matches_independent_ewa():
    """Conic and mean from scipy rotations + a finite-difference pinhole Jacobian."""
    w = synth.config0()
    o = Oracle(w.n, 0, w.beta_gt, w.cams, w.width, w.height)
    pr = o.projection()
    b = w.beta_gt.astype(np.float64)
    n = w.n
    rng = np.random.default_rng(1)
    checked = 0
    for g in rng.choice(n, 40, replace=False):
        mu = b[synth.seg(n, "mean")].reshape(3, n)[:, g]
        ls = b[synth.seg(n, "log_scale")].reshape(3, n)[:, g]
        q = b[synth.seg(n, "quat")].reshape(4, n)[:, g]
        Rg = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        Sig = Rg @ np.diag(np.exp(2 * ls)) @ Rg.T
        for v in range(w.cams.shape[0]):
            if not pr["visible"][v, g]:
                continue
            c = w.cams[v].astype(np.float64)
            Rw, tw, (fx, fy, cx, cy) = c[:9].reshape(3, 3), c[9:12], c[12:16]
            t = Rw @ mu + tw

            def pi(tt):
                return np.array([fx * tt[0] / tt[2] + cx, fy * tt[1] / tt[2] + cy])

            h = 1e-6
            Jp = np.stack([(pi(t + h * e) - pi(t - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
            S2 = Jp @ Rw @ Sig @ Rw.T @ Jp.T + LOWPASS * np.eye(2)
            Q = np.linalg.inv(S2)
            rec = pr["rec"][v, g]
            np.testing.assert_allclose(rec[:2], pi(t), rtol=1e-12)
            np.testing.assert_allclose(rec[2:5], [Q[0, 0], Q[0, 1], Q[1, 1]], rtol=1e-6)
            checked += 1
    assert checked > 50


def test_quaternion_sign_and_scale_invariance():
    w = synth.config0()
    n = w.n
    b2 = w.beta_gt.astype(np.float64).copy()
    b2[synth.seg(n, "quat")] *= -2.5
    r1 = Oracle(n, 0, w.beta_gt, w.cams, w.width, w.height).projection()["rec"]
    r2 = Oracle(n, 0, b2, w.cams, w.width, w.height).projection()["rec"]
    np.testing.assert_allclose(r1, r2, rtol=1e-10, atol=1e-12)


def test_projection_jacobian_matches_central_differences():
    w = synth.tiny(n=3, sh_degree=3, n_views=2, size=32)
    o = Oracle(w.n, 3, w.beta_init, w.cams, w.width, w.height)
    b = w.beta_init.astype(np.float64)
    h = 1e-6
    for v in range(2):
        for g in range(w.n):
            J = o.proj_jacobian(v, g)
            for j in range(o.Pg):
                e = np.zeros(o.P)
                e[j * w.n + g] = h
                rp = Oracle(w.n, 3, b + e, w.cams, w.width, w.height).projection()["rec"][v, g]
                rm = Oracle(w.n, 3, b - e, w.cams, w.width, w.height).projection()["rec"][v, g]
                np.testing.assert_allclose(J[:, j], (rp - rm) / (2 * h), rtol=1e-6, atol=1e-7)


# --------------------------------------------------------------- tile lists
def test_lists_match_brute_force():
    w = synth.config0()
    o = Oracle(w.n, 0, w.beta_gt, w.cams, w.width, w.height)
    pr = o.projection()
    ts, ids = o.lists()
    for v in range(o.V):
        for t in range(o.T):
            tx, ty = t % o.TX, t // o.TX
            members = [g for g in range(o.n) if pr["visible"][v, g]
                       and pr["rect"][v, g, 0] <= tx < pr["rect"][v, g, 2]
                       and pr["rect"][v, g, 1] <= ty < pr["rect"][v, g, 3]]
            members.sort(key=lambda g: (pr["depth"][v, g], g))
            got = ids[ts[v * o.T + t]: ts[v * o.T + t + 1]]
            assert list(got) == members


def test_rect_definition_and_visibility():
    """Rectangles from the FP64 centre and the integer radius: a tile is in the
    rectangle iff its pixel span [16t, 16t+16) meets [u - r, u + r]."""
    w = synth.config0()
    o = Oracle(w.n, 0, w.beta_gt, w.cams, w.width, w.height)
    pr = o.projection()
    assert pr["visible"].sum() > 0.9 * pr["visible"].size
    for v in range(o.V):
        for g in range(o.n):
            if not pr["visible"][v, g]:
                continue
            u, vv = pr["rec"][v, g, :2]
            r = pr["radius"][v, g]
            xs = [t for t in range(o.TX) if 16 * t <= u + r and 16 * t + 16 > u - r]
            ys = [t for t in range(o.TY) if 16 * t <= vv + r and 16 * t + 16 > vv - r]
            rc = pr["rect"][v, g]
            assert (rc[0], rc[2] - 1, rc[1], rc[3] - 1) == (xs[0], xs[-1], ys[0], ys[-1])
            assert pr["depth"][v, g] > 0.2


def test_near_plane_culls():
    n, beta = one_gaussian_scene([[0, 0, -2.9], [0, 0, 0]], [math.log(0.1)] * 3, [1, 0, 0, 0], 0.0,
                                 [0.5, 0.5, 0.5])
    o = Oracle(n, 0, beta, axis_camera(40.0, 64, 64), 64, 64)
    vis = o.projection()["visible"][0]
    assert list(vis) == [0, 1]


def test_dense_jacobian_size_arithmetic():
    """Sec. 4.1: 100 images of 800x800, 10k Gaussians, 14 parameters each, FP32:
    the dense Jacobian exceeds 100 TB and a 99 % sparse one still exceeds 1 TB."""
    rows = 100 * 800 * 800 * 3
    cols = 10_000 * synth.n_params(1, 0)
    assert synth.n_params(1, 0) == 14
    dense = rows * cols * 4
    assert dense > 100e12 and 0.01 * dense > 1e12
