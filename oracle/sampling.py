"""Residual sampling for the oracle (test infrastructure only).

Stratified uniform sampling of Sec. 4.4: k pixels drawn per 16x16 tile, without
replacement, each with weight 256 / k (the importance weight 1 / (N q) of
eq. 12 with q uniform inside the tile, scaled so that k = 256 gives weight 1).

The random numbers come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC 2011): a counter-based
generator, so the oracle and the GPU draw identical keys from the same
(seed, LM iteration, view, tile, pixel) counter without sharing state.
Pixel p of tile t in camera c at LM iteration it gets the first 32-bit output
word of Philox(counter = (p, t, c, it), key = (seed_lo, seed_hi)); the k pixels
with the smallest (word, p) are taken and listed in ascending pixel order.

The residual-weighted sampler (Supp. E, q_residual) draws k pixels per tile
with replacement from the softmax of the pixels' residual magnitudes inside
the tile; see ``sample_residual``. The contribution-weighted sampler (Supp. E,
q_Gaussian) draws them in proportion to the number of Gaussians blended into
each pixel; see ``sample_gaussian``.
"""
from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint32(0x9E3779B9)
_W1 = np.uint32(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr: np.ndarray, key: tuple[int, int]) -> np.ndarray:
    """ctr: uint32 [..., 4]; returns uint32 [..., 4]."""
    c = [ctr[..., i].astype(np.uint64) for i in range(4)]
    k0 = np.uint64(key[0] & 0xFFFFFFFF)
    k1 = np.uint64(key[1] & 0xFFFFFFFF)
    for r in range(10):
        if r > 0:
            k0 = (k0 + np.uint64(_W0)) & _MASK
            k1 = (k1 + np.uint64(_W1)) & _MASK
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack([x.astype(np.uint32) for x in c], axis=-1)


def tile_keys(seed: int, it: int, cam_ids: np.ndarray, n_tiles: int) -> np.ndarray:
    """uint32 keys [V, T, 256] for every pixel of every tile of the listed cameras."""
    cam_ids = np.asarray(cam_ids, dtype=np.uint32)
    V = cam_ids.size
    ctr = np.zeros((V, n_tiles, 256, 4), dtype=np.uint32)
    ctr[..., 0] = np.arange(256, dtype=np.uint32)[None, None, :]
    ctr[..., 1] = np.arange(n_tiles, dtype=np.uint32)[None, :, None]
    ctr[..., 2] = cam_ids[:, None, None]
    ctr[..., 3] = np.uint32(it)
    return philox4x32_10(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))[..., 0]


def sample_uniform(seed: int, it: int, cam_ids, n_tiles: int, k: int):
    """(pix uint8 [V, T, k] ascending, w float32 [V, T, k] = 256/k)."""
    keys = tile_keys(seed, it, cam_ids, n_tiles).astype(np.uint64)
    order_key = (keys << np.uint64(8)) | np.arange(256, dtype=np.uint64)[None, None, :]
    chosen = np.sort(np.argsort(order_key, axis=-1, kind="stable")[..., :k], axis=-1)
    w = np.full(chosen.shape, 256.0 / k, dtype=np.float32)
    return chosen.astype(np.uint8), w


def draw_words(seed: int, it: int, cam_ids, n_tiles: int, k: int) -> np.ndarray:
    """int64 [V, T, k] in [0, 2^24): draw j of tile t in camera c at LM iteration
    it is the first Philox4x32-10 word of counter (256 + j, t, c, it) (counters
    0..255 belong to the uniform sampler's pixel keys), cut to its top 24 bits."""
    cam_ids = np.asarray(cam_ids, dtype=np.uint32)
    V = cam_ids.size
    ctr = np.zeros((V, n_tiles, k, 4), dtype=np.uint32)
    ctr[..., 0] = 256 + np.arange(k, dtype=np.uint32)[None, None, :]
    ctr[..., 1] = np.arange(n_tiles, dtype=np.uint32)[None, :, None]
    ctr[..., 2] = cam_ids[:, None, None]
    ctr[..., 3] = np.uint32(it)
    word = philox4x32_10(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))[..., 0]
    return (word >> np.uint32(8)).astype(np.int64)


def draw_uniforms(seed: int, it: int, cam_ids, n_tiles: int, k: int) -> np.ndarray:
    """float64 [V, T, k] in [0, 1): the draw words scaled by 2^-24 (exact in
    FP32 as well)."""
    return draw_words(seed, it, cam_ids, n_tiles, k).astype(np.float64) * 2.0 ** -24


def sample_residual(seed: int, it: int, cam_ids, n_tiles: int, k: int, scores: np.ndarray):
    """Residual-weighted stratified sampling (Supp. E, q_residual, eq. 16),
    restricted to each 16x16 tile (Sec. 4.4): inside a tile pixel p has
    probability q(p) = exp(s_p) / sum_q exp(s_q), with s_p = |r_p| the pixel's
    residual magnitude (scores, [V, T, 256]); k independent draws per tile, with
    replacement, each weighted 1 / (k q(p)) so that the weighted sum over the
    draws estimates the tile's sum (eq. 11, 12).

    Draw j takes the pixel whose interval [Q_{p-1}, Q_p) of the cumulative
    distribution Q_p = q(0) + ... + q(p) holds the draw's uniform number.
    Returns (pix uint8 [V, T, k] in draw order, w float64 [V, T, k],
    margin float64 [V, T, k] = distance of the uniform number to the nearer
    end of its interval, the room the decision has for rounding)."""
    s = np.asarray(scores, dtype=np.float64)
    e = np.exp(s - s.max(axis=-1, keepdims=True))         # softmax numerator (shift-invariant)
    q = e / e.sum(axis=-1, keepdims=True)
    Q = np.cumsum(q, axis=-1)
    Q[..., -1] = 1.0
    u = draw_uniforms(seed, it, cam_ids, n_tiles, k)
    # smallest p with Q_p > u = the number of p with Q_p <= u (Q is non-decreasing)
    pix = np.empty(u.shape, dtype=np.int64)
    for v in range(u.shape[0]):
        pix[v] = (Q[v][:, None, :] <= u[v][:, :, None]).sum(axis=-1)
    pix = np.minimum(pix, 255)
    qp = np.take_along_axis(q, pix, axis=-1)
    hi = np.take_along_axis(Q, pix, axis=-1)
    lo = hi - qp
    margin = np.minimum(u - lo, hi - u)
    return pix.astype(np.uint8), 1.0 / (k * qp), margin


def sample_gaussian(seed: int, it: int, cam_ids, n_tiles: int, k: int, counts: np.ndarray):
    """Contribution-weighted stratified sampling (Supp. E, q_Gaussian, eq. 17),
    restricted to each 16x16 tile (Sec. 4.4): inside a tile pixel p has
    probability q(p) = G_p / sum_q G_q, with G_p the number of Gaussians
    blended into pixel p (counts, [V, T, 256]). A tile where no pixel has a
    contribution is sampled uniformly (G_p taken as 1). k independent draws per
    tile, with replacement, each weighted 1 / (k q(p)) = Z / (k G_p), Z = sum G.

    Draw j takes the smallest p with Q_p > u_j Z, Q_p = G_0 + ... + G_p and
    u_j = d_j 2^-24 with d_j the draw's 24-bit word: in integers,
    Q_p 2^24 > d_j Z, so the draws are exact. A pixel with G_p = 0 (in a tile
    with contributions) is never drawn; its Jacobian row is zero, so it adds
    nothing to J^T W r or J^T W J either.
    Returns (pix uint8 [V, T, k] in draw order, w float64 [V, T, k])."""
    G = np.rint(np.asarray(counts, dtype=np.float64)).astype(np.int64)
    assert np.all(G >= 0)
    empty = G.sum(axis=-1, keepdims=True) == 0
    G = np.where(empty, 1, G)
    Q = np.cumsum(G, axis=-1)
    Z = Q[..., -1:]
    d = draw_words(seed, it, cam_ids, n_tiles, k)
    pix = np.empty(d.shape, dtype=np.int64)
    for v in range(d.shape[0]):
        # smallest p with Q_p 2^24 > d Z = the number of p with Q_p 2^24 <= d Z
        pix[v] = ((Q[v][:, None, :] << 24) <= (d[v] * Z[v])[:, :, None]).sum(axis=-1)
    assert np.all(pix < 256)
    gp = np.take_along_axis(G, pix, axis=-1)
    return pix.astype(np.uint8), Z.astype(np.float64) / (k * gp)
