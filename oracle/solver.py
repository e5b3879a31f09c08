"""Matrix-free PCG and one LM step for the oracle (test infrastructure only).

Written in the order of Alg. 1 (one LM step with a matrix-free preconditioned
CG solver) of arXiv 2504.12905, in FP64 numpy over the C++ oracle's operator
products. Readings of the paper that this code fixes:

* sign: with r = I_hat - I (eq. 7) and (J^T J + lam I) dbeta = J^T r (eq. 8),
  the descent update is beta - eta * x (Alg. 1 writes "+"); see ``lm_step``;
* "for i = 0 to PCG_iters" runs exactly ``iters`` operator products;
* the loop stops early (keeping x) if p^T A p <= 0 or r^T z has collapsed;
* learning rate (Sec. 4.5, Supp. D): eta = 0.05 for the first 10 LM
  iterations, afterwards min(0.2, 1 / max |x_dc|) with x_dc the DC colour
  coefficients of the solution (so the largest colour change is at most 1);
* residual-weighted sampling (Supp. E, q_residual): the distribution comes
  from a render of every pixel of the batch views at the current parameters,
  with |r_p| = |r_p,R| + |r_p,G| + |r_p,B|; see ``residual_scores``;
* contribution-weighted sampling (Supp. E, q_Gaussian): the counts G_p come
  from the same full render; see ``contributor_counts``;
* SSIM residual (Supp. B, Sec. 6; ``ssim_weight`` > 0): the SSIM terms come
  from full renders of the batch views, and the Gauss-Newton system of the
  step is that of ``ssim.residual_and_weights``: b = J^T u, the operator
  weighted per channel by wc, the preconditioner's diagonal by wbar.
"""
from __future__ import annotations

import numpy as np

from . import Oracle
from .sampling import sample_gaussian, sample_residual, sample_uniform
from .ssim import residual_and_weights, ssim_terms


def pcg(apply_A, b: np.ndarray, m_inv: np.ndarray, iters: int):
    """Alg. 1, PCG part: solve A x = b from x0 = 0 with Jacobi preconditioner m_inv.

    Returns (x, residual norms ||r_i|| for i = 0..done, number of products)."""
    r = b.copy()                       # r0 = J^T r   (the right-hand side)
    z = m_inv * r                      # z0 = M^-1 r0
    p = z.copy()                       # p0 = z0
    x = np.zeros_like(b)               # x0 = 0
    rz = float(r @ z)
    rz0 = rz
    norms = [float(np.linalg.norm(r))]
    done = 0
    for _ in range(iters):
        u = apply_A(p)                 # u = (J^T J + lam I) p
        done += 1
        pu = float(p @ u)
        if not (pu > 0.0) or not (rz > 1e-30 * rz0):
            break
        alpha = rz / pu
        x = x + alpha * p
        r = r - alpha * u
        z = m_inv * r
        rz_new = float(r @ z)
        beta = rz_new / rz
        p = z + beta * p
        rz = rz_new
        norms.append(float(np.linalg.norm(r)))
    return x, np.array(norms), done


def learning_rate(x: np.ndarray, n: int, it: int, cap: float = 0.2, warm: float = 0.05,
                  warm_iters: int = 10) -> float:
    """Sec. 4.5 / Supp. D: bound the largest DC-colour change of eta*x by 1."""
    if it < warm_iters:
        return warm
    m = float(np.max(np.abs(x[11 * n: 14 * n]))) if n else 0.0
    return cap if m == 0.0 else min(cap, 1.0 / m)


def gather_targets(targets: np.ndarray, orc: Oracle) -> np.ndarray:
    """Target colours [S, 3] at the oracle's sampled pixels; targets is [V, H, W, 3]."""
    v, x, y = orc.pixel_coords()
    return targets[v, y, x].astype(np.float64)


def residual_scores(orc: Oracle, targets: np.ndarray) -> np.ndarray:
    """|r_p| = sum over channels of |I_hat_p - I_p| at every pixel of the
    oracle's views (targets [V, H, W, 3] of those views), as [V, T, 256] in
    tile-major pixel order. Leaves the oracle sampling every pixel."""
    orc.set_samples(256)
    res = orc.render()["C"] - gather_targets(targets, orc)
    return np.abs(res).sum(axis=1).reshape(orc.V, orc.T, 256)


def contributor_counts(orc: Oracle) -> np.ndarray:
    """G_p = the number of Gaussians blended into pixel p (Supp. E, q_Gaussian:
    skipped transparent ones and those behind the transmittance stop are not
    counted) at every pixel of the oracle's views, as [V, T, 256] in tile-major
    pixel order. Leaves the oracle sampling every pixel."""
    orc.set_samples(256)
    return orc.render()["n_contrib"].reshape(orc.V, orc.T, 256).astype(np.float64)


def lm_step(n, sh_degree, beta, cams_all, targets_all, view_ids, width, height, k, seed, it, lam,
            cg_iters, d=None, opts=None, sampler="uniform", ssim_weight=0.0):
    """Alg. 1 for one LM iteration. Returns (beta_next float32, info dict).

    sampler: "uniform" (Sec. 4.4; k = 256 takes every pixel), "residual"
    (Supp. E q_residual) or "gaussian" (Supp. E q_Gaussian), the last two with
    k draws per tile with replacement."""
    view_ids = np.asarray(view_ids, dtype=np.int64)
    cams = cams_all[view_ids]                                   # getBatch (view sampling)
    orc = Oracle(n, sh_degree, beta, cams, width, height, opts)  # splatting: project + bin
    margin = None
    if sampler == "residual":
        scores = residual_scores(orc, targets_all[view_ids])
        pix, w, margin = sample_residual(seed, it, view_ids, orc.T, k, scores)
        orc.set_samples(k, pix, w)
    elif sampler == "gaussian":
        pix, w = sample_gaussian(seed, it, view_ids, orc.T, k, contributor_counts(orc))
        orc.set_samples(k, pix, w)
    elif k >= 256:
        orc.set_samples(256)
    else:
        pix, w = sample_uniform(seed, it, view_ids, orc.T, k)
        orc.set_samples(k, pix, w)
    fwd = orc.render()
    res = fwd["C"] - gather_targets(targets_all[view_ids], orc)  # r = I_hat - I  (eq. 7)
    wts = orc.weights()
    if ssim_weight > 0:
        k_s, pix_s, w_s = orc.k, orc.pix, orc.w
        img = orc.render_image()                                # every pixel of the batch views
        orc.set_samples(k_s, pix_s, w_s)
        tg = np.asarray(targets_all[view_ids], np.float64)
        u, wc, wbar = residual_and_weights(orc, img, tg, wts, s=ssim_weight)
        b = orc.vjp(u)                                          # r0 = J^T u
        orc.set_samples(k_s, pix_s, wbar)
        D = orc.diag()                                          # diag(J^T diag(wbar) J)
        orc.set_channel_weights(wc)                             # operator J^T diag(wc) J
        v, px, py = orc.pixel_coords()
        rho = 1.0 - ssim_terms(img, tg)[0][v, py, px]
        loss = float(np.sum(wts[:, None] * (res ** 2 + ssim_weight * rho ** 2)))
    else:
        b = orc.vjp(wts[:, None] * res)                         # r0 = J^T W r
        D = orc.diag()                                          # diag(J^T W J)
        loss = float(np.sum(wts[:, None] * res ** 2))
    dd = np.ones(orc.P) if d is None else np.asarray(d, np.float64)
    m_inv = 1.0 / (D + lam * dd)                                # M^-1 = 1 / diag(J^T W J + lam d)
    x, norms, done = pcg(lambda p: orc.gn(p, lam, dd), b, m_inv, cg_iters)
    eta = learning_rate(x, n, it)
    beta_next = (beta.astype(np.float64) - eta * x).astype(np.float32)
    info = dict(loss_sampled=loss, b=b, diag=D, x=x, eta=eta,
                cg_norms=norms, cg_done=done, residual=res, weights=wts, samples=orc.pix,
                sample_margin=margin)
    return beta_next, info


def full_loss(n, sh_degree, beta, cams, targets, width, height, opts=None) -> float:
    """Sum of squared residuals over every pixel and channel of the given views (eq. 6, unnormalised)."""
    orc = Oracle(n, sh_degree, beta, cams, width, height, opts)
    img = orc.render_image()
    return float(np.sum((img - targets) ** 2))
