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
