"""Pins of the oracle's derivatives and operators.

* J p (dual numbers, Supp. A Alg. 3) against central finite differences of the
  primal render, excluding pixels whose discrete decisions change between
  beta - h e_j and beta + h e_j (the derivative is taken with decisions frozen);
* J^T u (reverse accumulation) against the dense J built column by column, and
  the adjoint identity <J p, u> = <p, J^T u>;
* the Gauss-Newton operator J^T W J + lam d (eq. 8, eq. 14): equal to the dense
  product, symmetric, and with eigenvalues >= lam min(d) (PSD Gauss-Newton part);
* diag(J^T W J) against the dense column sums.
"""
import numpy as np
import pytest

from oracle import Oracle
from paper_2504_12905_amd import synth


def tiny_problem(sh_degree=0, n=4, views=2, size=32, seed=0, k=None):
    w = synth.tiny(n=n, sh_degree=sh_degree, n_views=views, size=size, seed=seed)
    o = Oracle(w.n, sh_degree, w.beta_init, w.cams, w.width, w.height)
    if k is not None:
        rng = np.random.default_rng(seed + 100)
        pix = np.stack([np.sort(rng.choice(256, k, replace=False)) for _ in range(o.V * o.T)])
        wt = rng.uniform(0.5, 3.0, size=pix.shape).astype(np.float32)
        o.set_samples(k, pix, wt)
    return w, o


def fd_jacobian(w, o, h=1e-5):
    """Central differences with the same sample set; returns (J_fd, valid rows)."""
    b = w.beta_init.astype(np.float64)
    base = o.render()
    J = np.zeros((3 * o.S, o.P))
    valid = np.ones(3 * o.S, bool)
    for j in range(o.P):
        outs = []
        for s in (+1, -1):
            bb = b.copy()
            bb[j] += s * h
            oo = Oracle(w.n, w.sh_degree, bb, w.cams, w.width, w.height)
            oo.set_samples(o.k, o.pix, o.w)
            outs.append(oo.render())
        J[:, j] = ((outs[0]["C"] - outs[1]["C"]) / (2 * h)).reshape(-1)
        same = (outs[0]["trace"] == base["trace"]) & (outs[1]["trace"] == base["trace"])
        valid &= np.repeat(same, 3)
    return J, valid


@pytest.mark.parametrize("deg", [0, 1, 3])
def test_dual_jvp_matches_central_differences(deg):
    w, o = tiny_problem(sh_degree=deg, n=3, views=2, size=32, seed=deg)
    Jd = o.dense_jacobian()
    Jf, valid = fd_jacobian(w, o)
    assert valid.mean() > 0.97
    assert np.abs(Jd).max() > 0.1
    scale = np.abs(Jd[valid]).max()
    np.testing.assert_allclose(Jd[valid], Jf[valid], rtol=1e-5, atol=1e-6 * scale)


def test_vjp_is_transpose_of_dense_jacobian():
    w, o = tiny_problem(sh_degree=1, n=4, views=2, seed=5, k=64)
    J = o.dense_jacobian()
    rng = np.random.default_rng(1)
    u = rng.normal(size=(o.S, 3))
    np.testing.assert_allclose(o.vjp(u), J.T @ u.reshape(-1), rtol=1e-10, atol=1e-12)


def test_screen_adjoint_matches_dense_screen_jacobian():
    """Per-(view, Gaussian) screen gradients, checked through the chain rule."""
    w, o = tiny_problem(sh_degree=0, n=3, views=1, seed=2)
    rng = np.random.default_rng(2)
    u = rng.normal(size=(o.S, 3))
    gs = o.vjp_screen(u)
    full = o.vjp(u)
    acc = np.zeros(o.P)
    for v in range(o.V):
        for g in range(o.n):
            Jp = o.proj_jacobian(v, g)
            acc[np.arange(o.Pg) * o.n + g] += Jp.T @ gs[v, g]
    np.testing.assert_allclose(acc, full, rtol=1e-12, atol=1e-14)


def test_adjoint_identity_config0():
    w = synth.config0()
    o = Oracle(w.n, 0, w.beta_init, w.cams, w.width, w.height)
    rng = np.random.default_rng(7)
    p = rng.normal(size=o.P)
    u = rng.normal(size=(o.S, 3))
    lhs = float(np.sum(o.jvp(p) * u))
    rhs = float(p @ o.vjp(u))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_gn_operator_dense_symmetric_psd():
    w, o = tiny_problem(sh_degree=1, n=4, views=2, seed=3, k=48)
    lam = 0.05
    J = o.dense_jacobian()
    wt = np.repeat(o.weights(), 3)
    A_dense = J.T @ (wt[:, None] * J) + lam * np.eye(o.P)
    A = np.stack([o.gn(e, lam) for e in np.eye(o.P)], axis=1)
    np.testing.assert_allclose(A, A_dense, rtol=1e-10, atol=1e-12 * np.abs(A_dense).max())
    np.testing.assert_allclose(A, A.T, rtol=1e-10, atol=1e-12 * np.abs(A).max())
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev.min() >= lam - 1e-10 * ev.max()
    d = np.random.default_rng(0).uniform(0.5, 2.0, o.P)
    p = np.random.default_rng(1).normal(size=o.P)
    np.testing.assert_allclose(o.gn(p, lam, d), (A_dense - lam * np.eye(o.P)) @ p + lam * d * p,
                               rtol=1e-10, atol=1e-12)


def test_diag_matches_dense_column_sums():
    w, o = tiny_problem(sh_degree=2, n=3, views=2, seed=4, k=40)
    J = o.dense_jacobian()
    wt = np.repeat(o.weights(), 3)
    np.testing.assert_allclose(o.diag(), np.sum(wt[:, None] * J * J, axis=0), rtol=1e-10, atol=1e-14)


def test_tile_mask_restricts_to_listed_gaussians():
    """Restricting the pixel work to the tiles that list a Gaussian leaves that
    Gaussian's entries of the GN product unchanged (used for sampled parity at scale)."""
    w = synth.config0()
    o = Oracle(w.n, 0, w.beta_init, w.cams, w.width, w.height)
    rng = np.random.default_rng(0)
    p = rng.normal(size=o.P)
    full = o.gn(p, 1e-3)
    ts, ids = o.lists()
    sel = np.array([5, 77, 400])
    mask = np.zeros(o.V * o.T, np.uint8)
    for i in range(o.V * o.T):
        if np.isin(ids[ts[i]:ts[i + 1]], sel).any():
            mask[i] = 1
    assert 0 < mask.sum() < mask.size
    o.set_tile_mask(mask)
    part = o.gn(p, 1e-3)
    idx = (np.arange(o.Pg)[:, None] * o.n + sel[None, :]).reshape(-1)
    np.testing.assert_allclose(part[idx], full[idx], rtol=1e-12, atol=1e-14)


def test_vjp_term_magnitudes():
    """|J^T u| term scale (oracle.vjp_abs) bounds both |J^T u| and |J|^T |u|
    (dense J by dual numbers) from above, entry by entry."""
    w, o = tiny_problem(sh_degree=1, n=3, views=1, seed=4, k=16)
    rng = np.random.default_rng(9)
    u = rng.normal(size=(o.S, 3))
    got = o.vjp_abs(u)
    J = o.dense_jacobian()
    absju = np.abs(J).T @ np.abs(u.reshape(-1))
    assert np.all(got >= absju * (1 - 1e-12) - 1e-14)
    assert np.all(got >= np.abs(o.vjp(u)) * (1 - 1e-12) - 1e-14)
    assert np.abs(got).max() > 0
    # a term mis-signed into a cancellation would leave the bound on some entry
    assert np.max(got - absju) > 0


def test_vjp_term_magnitudes_without_cancellation():
    """One Gaussian, black background, u >= 0: every pixel's derivative with
    respect to the opacity logit and to the DC colour coefficients is a
    single non-negative product (nothing behind, one record component), so
    the term scale equals |J^T u| there exactly."""
    from test_oracle_geometry import axis_camera, one_gaussian_scene
    n, beta = one_gaussian_scene([[0.02, -0.03, 0.0]], [np.log(0.15)] * 3, [1, 0, 0, 0], 0.3, [0.6, 0.4, 0.8])
    o = Oracle(n, 0, beta, axis_camera(40.0, 32, 32), 32, 32)
    u = np.random.default_rng(3).uniform(0.1, 1.0, size=(o.S, 3))
    got, exact = o.vjp_abs(u), o.vjp(u)
    idx = [synth.seg(n, "opacity").start] + list(range(synth.seg(n, "sh", 0).start, synth.seg(n, "sh", 0).start + 3))
    assert np.all(exact[idx] > 0)
    np.testing.assert_allclose(got[idx], exact[idx], rtol=1e-12)
