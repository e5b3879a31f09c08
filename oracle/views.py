"""View batches by camera clustering for the oracle (test infrastructure only).

Sec. 4.3 of arXiv 2504.12905: each camera gets the 6-D feature
f_i = (x, y, z, dx, dy, dz), its normalised location and its viewing
direction; K-means splits the features into B clusters (B = batch size) and
one camera is drawn at random from every cluster.

Readings (the paper names the method only):
* location: the camera centre -R^T t, minus the mean of all centres, divided
  by the largest resulting distance (positions in the unit ball, the scale of
  the unit directions); direction: the camera's +z axis in world coordinates;
* K-means is Lloyd's algorithm from D^2 ("k-means++") seeding, run until no
  assignment changes (at most 100 rounds); ties go to the lower cluster index;
  a cluster left empty takes the camera farthest from its own centre;
* random numbers are Philox4x32-10 words (top 24 bits) of fixed counters
  under key = seed: seeding draw s uses counter (s, 0, B, 0x4b4d0001), the
  draw of cluster j at LM iteration it counter (j, it, B, 0x4b4d0002), which
  picks member floor(d m / 2^24) of the cluster's m members in ascending
  camera index.
"""
from __future__ import annotations

import numpy as np

from .sampling import philox4x32_10

SEED_TAG = 0x4B4D0001
PICK_TAG = 0x4B4D0002


def _word24(c0: int, c1: int, c2: int, c3: int, seed: int) -> int:
    ctr = np.array([[c0, c1, c2, c3]], dtype=np.uint32)
    return int(philox4x32_10(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))[0, 0]) >> 8


def camera_features(cams: np.ndarray) -> np.ndarray:
    """[N, 6] features of the cameras (float32 rows R[9] t[3] fx fy cx cy)."""
    cams = np.asarray(cams, dtype=np.float32).astype(np.float64)
    R = cams[:, 0:9].reshape(-1, 3, 3)
    t = cams[:, 9:12]
    centres = -np.einsum("nji,nj->ni", R, t)          # -R^T t
    pos = centres - centres.mean(axis=0)
    rmax = np.sqrt((pos ** 2).sum(axis=1)).max()
    if rmax > 0:
        pos = pos / rmax
    return np.hstack([pos, R[:, 2, :]])               # forward axis = third row of world->camera R


def kmeans(f: np.ndarray, B: int, seed: int, max_rounds: int = 100):
    """Returns (labels [N], centres [B, 6]) of Lloyd's algorithm from D^2 seeding."""
    N = f.shape[0]
    assert 0 < B <= N
    sq = lambda a, b: float(((a - b) ** 2).sum())
    first = (_word24(0, 0, B, SEED_TAG, seed) * N) >> 24
    centres = [f[first].copy()]
    chosen = {first}
    d2 = np.array([sq(f[i], centres[0]) for i in range(N)])
    for s in range(1, B):
        total = float(d2.sum())
        if total > 0:
            target = _word24(s, 0, B, SEED_TAG, seed) * 2.0 ** -24 * total
            run, pick = 0.0, N - 1
            for i in range(N):
                run += d2[i]
                if run > target:
                    pick = i
                    break
        else:
            pick = min(i for i in range(N) if i not in chosen)
        centres.append(f[pick].copy())
        chosen.add(pick)
        d2 = np.minimum(d2, [sq(f[i], centres[-1]) for i in range(N)])
    C = np.array(centres)
    labels = np.full(N, -1)
    for _ in range(max_rounds):
        D = np.array([[sq(f[i], C[c]) for c in range(B)] for i in range(N)])
        new = D.argmin(axis=1)                       # first minimum: lower cluster index on ties
        changed = bool(np.any(new != labels))
        labels = new
        count = np.bincount(labels, minlength=B)
        reseeded = False
        for c in range(B):
            if count[c] > 0:
                continue
            cand = [i for i in range(N) if count[labels[i]] >= 2]
            dist = [sq(f[i], C[labels[i]]) for i in cand]
            far = cand[int(np.argmax(dist))]         # first maximum: lower camera index on ties
            count[labels[far]] -= 1
            labels[far] = c
            count[c] = 1
            reseeded = True
        C = np.array([f[labels == c].mean(axis=0) for c in range(B)])
        if not changed and not reseeded:
            break
    return labels, C


def view_batch(labels: np.ndarray, B: int, seed: int, it: int) -> np.ndarray:
    """One camera per cluster for LM iteration it: int [B]."""
    out = np.empty(B, dtype=np.int64)
    for j in range(B):
        members = np.flatnonzero(labels == j)
        out[j] = members[(_word24(j, it, B, PICK_TAG, seed) * members.size) >> 24]
    return out
