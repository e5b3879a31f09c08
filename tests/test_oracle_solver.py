"""Pins of the oracle's PCG (Alg. 1), LM step, learning-rate rule and residual sampling."""
import os

import numpy as np
import pytest

from oracle import Oracle
from oracle.sampling import philox4x32_10, sample_uniform, tile_keys
from oracle.solver import full_loss, learning_rate, lm_step, pcg
from paper_2504_12905_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------- PCG
def spd(n, cond=50.0, seed=0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    ev = np.geomspace(1.0, cond, n)
    return (Q * ev) @ Q.T


def test_pcg_solves_spd_system_in_n_steps():
    n = 40
    A = spd(n)
    b = np.random.default_rng(1).normal(size=n)
    m_inv = 1.0 / np.diag(A)
    # exact in n steps in exact arithmetic; a few more absorb FP64 loss of orthogonality
    x, norms, done = pcg(lambda p: A @ p, b, m_inv, 2 * n)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-8, atol=1e-10)
    x, _, _ = pcg(lambda p: A @ p, b, m_inv, n)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-4)


def test_pcg_unpreconditioned_is_textbook_cg_and_a_norm_error_decreases():
    n = 30
    A = spd(n, cond=200.0, seed=2)
    b = np.random.default_rng(3).normal(size=n)
    xs = np.linalg.solve(A, b)
    errs = []
    for it in range(1, n + 1):
        x, _, _ = pcg(lambda p: A @ p, b, np.ones(n), it)
        e = x - xs
        errs.append(float(e @ A @ e))
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-9) for i in range(len(errs) - 1))
    # textbook CG (Hestenes-Stiefel) written independently
    x = np.zeros(n); r = b.copy(); p = r.copy()
    for _ in range(5):
        Ap = A @ p; a = (r @ r) / (p @ Ap); x += a * p; rn = r - a * Ap
        p = rn + (rn @ rn) / (r @ r) * p; r = rn
    x5, _, _ = pcg(lambda q: A @ q, b, np.ones(n), 5)
    np.testing.assert_allclose(x5, x, rtol=1e-10)


def test_pcg_iterates_have_positive_model_decrease():
    """x_0 = 0 and A SPD: every iterate minimises the quadratic model over its
    Krylov space, so b^T x_i >= x_i^T A x_i / 2 > 0 (the LM step descends)."""
    A = spd(25, seed=4)
    b = np.random.default_rng(5).normal(size=25)
    for it in range(1, 10):
        x, _, _ = pcg(lambda p: A @ p, b, 1.0 / np.diag(A), it)
        assert b @ x >= 0.5 * x @ A @ x > 0


# --------------------------------------------------------- learning rate
def test_learning_rate_rule():
    n = 10
    x = np.zeros(n * 14)
    assert learning_rate(x, n, 3) == 0.05
    assert learning_rate(x, n, 12) == 0.2
    x[11 * n + 4] = -20.0
    assert learning_rate(x, n, 12) == pytest.approx(1 / 20)
    x[11 * n + 4] = 2.0
    assert learning_rate(x, n, 12) == 0.2
    x[0] = 1e6  # a non-colour entry does not bound the step
    assert learning_rate(x, n, 12) == 0.2


# -------------------------------------------------------------- sampling
def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = philox4x32_10(np.array(v[:4], np.uint32), (v[4], v[5]))
        assert [int(x) for x in out] == v[6:10]


def test_uniform_sampler_shape_and_full_case():
    pix, w = sample_uniform(7, 3, [5, 9], 12, 26)
    assert pix.shape == (2, 12, 26) and np.all(w == np.float32(256 / 26))
    assert np.all(np.diff(pix.astype(int), axis=-1) > 0)
    full, wf = sample_uniform(7, 3, [5], 4, 256)
    assert np.all(full == np.arange(256)) and np.all(wf == 1.0)
    again, _ = sample_uniform(7, 3, [5, 9], 12, 26)
    assert np.array_equal(pix, again)
    other, _ = sample_uniform(7, 4, [5, 9], 12, 26)
    assert not np.array_equal(pix, other)


def test_uniform_sampler_chi_square():
    from scipy.stats import chi2
    pix, _ = sample_uniform(0, 0, np.arange(40), 100, 26)
    counts = np.bincount(pix.reshape(-1), minlength=256)
    expected = pix.size / 256
    stat = ((counts - expected) ** 2 / expected).sum()
    assert chi2.sf(stat, 255) > 1e-3
    keys = tile_keys(0, 0, [0], 64).reshape(-1)
    hist = np.bincount((keys >> np.uint32(28)).astype(int), minlength=16)
    stat = ((hist - keys.size / 16) ** 2 / (keys.size / 16)).sum()
    assert chi2.sf(stat, 15) > 1e-3


def test_sampled_gn_product_is_unbiased():
    """eq. 12-14: with weights 256/k the sampled J^T W J p averages to the full one."""
    w = synth.tiny(n=3, sh_degree=0, n_views=1, size=32, seed=1)
    o = Oracle(w.n, 0, w.beta_init, w.cams, w.width, w.height)
    p = np.random.default_rng(0).normal(size=o.P)
    o.set_samples(256)
    full = o.gn(p, 0.0)
    k, R = 32, 400
    acc = []
    for s in range(R):
        pix, wt = sample_uniform(s, 0, [0], o.T, k)
        o.set_samples(k, pix, wt)
        acc.append(o.gn(p, 0.0))
    acc = np.array(acc)
    mean, se = acc.mean(0), acc.std(0) / np.sqrt(R)
    big = np.abs(full) > 1e-3 * np.abs(full).max()
    z = np.abs(mean - full)[big] / (se[big] + 1e-12)
    assert np.mean(z < 4.0) > 0.99


# --------------------------------------------------------------------- LM
@pytest.fixture(scope="module")
def cfg0_targets():
    w = synth.config0()
    o = Oracle(w.n, 0, w.beta_gt, w.cams, w.width, w.height)
    return w, o.render_image().astype(np.float32)


def test_lm_steps_descend_on_config0(cfg0_targets):
    w, tg = cfg0_targets
    beta = w.beta_init
    losses = [full_loss(w.n, 0, beta, w.cams, tg, w.width, w.height)]
    for it in range(4):
        beta, info = lm_step(w.n, 0, beta, w.cams, tg, np.arange(4), w.width, w.height, 256, 0, it,
                             w.lam, w.cg_iters)
        assert float(info["b"] @ info["x"]) > 0
        assert info["cg_done"] == w.cg_iters
        losses.append(full_loss(w.n, 0, beta, w.cams, tg, w.width, w.height))
    assert all(losses[i + 1] < losses[i] for i in range(len(losses) - 1)), losses


def test_lm_step_with_sampling_descends(cfg0_targets):
    w, tg = cfg0_targets
    l0 = full_loss(w.n, 0, w.beta_init, w.cams, tg, w.width, w.height)
    beta, info = lm_step(w.n, 0, w.beta_init, w.cams, tg, np.arange(4), w.width, w.height, 64, 3, 0,
                         w.lam, 6)
    assert np.all(info["weights"] == 4.0)
    assert full_loss(w.n, 0, beta, w.cams, tg, w.width, w.height) < l0


def test_residual_scores_follow_tile_major_pixel_order(cfg0_targets):
    """scores[v, t, p] is the L1 residual of image pixel (x, y) with
    t = (y // 16) * (W / 16) + x // 16 and p = 16 (y % 16) + x % 16."""
    from oracle.solver import residual_scores
    w, tg = cfg0_targets
    orc = Oracle(w.n, 0, w.beta_init, w.cams, w.width, w.height)
    sc = residual_scores(orc, tg)
    img = orc.render_image()
    ref = np.abs(img - tg).sum(axis=-1)                      # [V, H, W]
    TX = w.width // 16
    for (v, y, x) in [(0, 0, 0), (1, 17, 5), (3, 63, 63), (2, 40, 22)]:
        t, p = (y // 16) * TX + x // 16, 16 * (y % 16) + x % 16
        assert sc[v, t, p] == pytest.approx(ref[v, y, x], rel=1e-12, abs=1e-15)


def test_lm_step_with_residual_sampling_descends(cfg0_targets):
    w, tg = cfg0_targets
    l0 = full_loss(w.n, 0, w.beta_init, w.cams, tg, w.width, w.height)
    beta, info = lm_step(w.n, 0, w.beta_init, w.cams, tg, np.arange(4), w.width, w.height, 32, 3, 0,
                         w.lam, 6, sampler="residual")
    assert float(info["b"] @ info["x"]) > 0
    assert info["weights"].min() > 0
    assert full_loss(w.n, 0, beta, w.cams, tg, w.width, w.height) < l0
