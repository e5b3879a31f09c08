"""SSIM residual with the diagonal approximation, for the oracle (test
infrastructure only).

Supp. B ("Results with SSIM loss") and Sec. 6 (Limitations) of arXiv
2504.12905: the SSIM term is added to the MSE loss with weights 1.0 and 0.2,
and its Jacobian is approximated diagonally: the SSIM of pixel p depends on
the colours of the whole window around p, and only its dependence on the
colour of p itself is kept. The paper gives no formula; the readings here:

* SSIM (Wang et al. 2004) per colour channel, an 11 x 11 Gaussian window of
  sigma 1.5 (weights summing to 1), zero padding outside the image,
  C1 = 0.01^2, C2 = 0.03^2 (dynamic range 1);
* the SSIM term enters the least-squares objective of Alg. 1 as a second
  residual per sampled pixel and channel, rho = 1 - SSIM_c(p), weighted by
  s = 0.2 relative to the colour residual r = I_hat - I:
      E = sum_{sampled p, c} w_p [ r_pc^2 + s rho_pc^2 ];
* diagonal approximation: d rho_pc / d I_hat_qc' = delta_pc if q = p and
  c' = c, else 0, with delta_pc = -d SSIM_c(p) / d I_hat_pc, so the
  Jacobian of rho is diag(delta) J and the Gauss-Newton system is
      b = J^T (w (r + s delta rho)),   A = J^T diag(w (1 + s delta^2)) J + lambda d;
* the Jacobi preconditioner uses one weight per pixel, the mean over the
  channels of w (1 + s delta^2).
"""
from __future__ import annotations

import numpy as np
from scipy.ndimage import correlate

WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2
WEIGHT = 0.2


def gaussian_window(size: int = WINDOW, sigma: float = SIGMA) -> np.ndarray:
    x = np.arange(size, dtype=np.float64) - (size - 1) / 2
    g = np.exp(-x ** 2 / (2 * sigma ** 2))
    g /= g.sum()
    return np.outer(g, g)


def _filter(img: np.ndarray, win: np.ndarray) -> np.ndarray:
    """Window-weighted local sums of [V, H, W, C] images, zero outside (a library correlation)."""
    out = np.empty_like(img)
    for v in range(img.shape[0]):
        for c in range(img.shape[3]):
            out[v, :, :, c] = correlate(img[v, :, :, c], win, mode="constant", cval=0.0)
    return out


def ssim_terms(x: np.ndarray, y: np.ndarray, size: int = WINDOW, sigma: float = SIGMA):
    """x: rendered images, y: targets, [V, H, W, 3] (FP64). Returns
    (ssim, dssim_dx_center): the SSIM map per pixel and channel and its
    derivative with respect to the rendered colour of the window's centre
    pixel (the diagonal term)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    win = gaussian_window(size, sigma)
    g0 = win[size // 2, size // 2]
    mx, my = _filter(x, win), _filter(y, win)
    sxx = _filter(x * x, win) - mx * mx
    syy = _filter(y * y, win) - my * my
    sxy = _filter(x * y, win) - mx * my
    a1, a2 = 2 * mx * my + C1, 2 * sxy + C2
    b1, b2 = mx * mx + my * my + C1, sxx + syy + C2
    ssim = (a1 * a2) / (b1 * b2)
    # d/dx_p of mu_x, sigma_x^2 and sigma_xy (p the centre, weight g0):
    #   g0, 2 g0 (x_p - mu_x), g0 (y_p - mu_y)
    da1 = 2 * g0 * my
    da2 = 2 * g0 * (y - my)
    db1 = 2 * g0 * mx
    db2 = 2 * g0 * (x - mx)
    dssim = (da1 * a2 + a1 * da2) / (b1 * b2) - ssim * (db1 / b1 + db2 / b2)
    return ssim, dssim


def residual_and_weights(orc, img: np.ndarray, target: np.ndarray, w: np.ndarray, s: float = WEIGHT,
                         size: int = WINDOW):
    """For the oracle's sampled pixels (img, target: [V, H, W, 3] of its
    views; w: [S] sample weights): (u [S, 3] = w (r + s delta rho),
    wc [S, 3] = w (1 + s delta^2), wbar [S] = mean over channels of wc)."""
    ssim, dssim = ssim_terms(img, target, size)
    v, px, py = orc.pixel_coords()
    r = img[v, py, px] - target[v, py, px]
    rho = 1.0 - ssim[v, py, px]
    delta = -dssim[v, py, px]
    w = np.asarray(w, np.float64)[:, None]
    u = w * (r + s * delta * rho)
    wc = w * (1.0 + s * delta ** 2)
    return u, wc, wc.mean(axis=1)
