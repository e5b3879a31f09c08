"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
compare with the FP64 oracle on the same seeded inputs."""
from __future__ import annotations

import sys

import numpy as np
import torch

from oracle import TAU_LIST, Oracle

DEV = "cuda:0"


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b) -> float:
    """Norm-wise relative difference ||a - b|| / ||b|| in FP64."""
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def elem(a, b) -> float:
    """Element-wise relative difference max_i |a_i - b_i| / (|b_i| + 1e-3 max|b|)
    in FP64: a few wrong entries among millions, which the norm-wise figure
    would average away, show up here."""
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    if b.size == 0:
        return 0.0
    return float(np.max(np.abs(a - b) / (np.abs(b) + 1e-3 * np.max(np.abs(b)) + 1e-300)))


def elem_scaled(a, b, scale) -> float:
    """Entry-wise error against the magnitude of the terms each entry is summed
    from: max_i |a_i - b_i| / scale_i over entries with scale_i > 0 (FP64).
    With scale = oracle.vjp_abs(u) a wrong term, sign or index shows as O(1);
    FP32 rounding of the sums shows as ~1e-6."""
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    s = np.asarray(scale, np.float64).reshape(-1)
    on = s > 0
    if not np.any(on):
        return float(np.max(np.abs(a - b))) if a.size else 0.0
    assert np.all(a[~on] == 0.0) or np.max(np.abs(a[~on])) < 1e-30, "entry with no terms is non-zero"
    return float(np.max(np.abs(a[on] - b[on]) / s[on]))


def lib():
    from paper_2504_12905_amd import lmrs
    return lmrs


def gpu_frame(n, deg, beta, cams, W, H, k=256, pix=None, wts=None, view_ids=None, render=True, ssim=False):
    L = lib()
    V = int(cams.shape[0]) if view_ids is None else len(view_ids)
    fr = L.Frame(n, deg, torch.tensor(np.asarray(beta, np.float32), device=DEV),
                 torch.tensor(np.asarray(cams, np.float32), device=DEV), W, H, V,
                 view_ids=None if view_ids is None else torch.tensor(np.asarray(view_ids, np.int32), device=DEV),
                 k=k, sampled=pix is not None, ssim=ssim)
    L.lmrs_project(fr)
    L.lmrs_bin_tiles(fr)
    if pix is not None:
        fr.pix.copy_(torch.tensor(np.asarray(pix, np.uint8).reshape(fr.pix.shape), device=DEV))
        fr.w.copy_(torch.tensor(np.asarray(wts, np.float32).reshape(fr.w.shape), device=DEV))
    if render:
        L.lmrs_render(fr)
    torch.cuda.synchronize()
    return fr


def oracle_for(n, deg, beta, cams, W, H, k=256, pix=None, wts=None) -> Oracle:
    # the same FP32 parameters the GPU frame is given (gpu_frame)
    o = Oracle(n, deg, np.asarray(beta, np.float32), cams, W, H)
    o.set_samples(k, pix, wts)
    return o


def np_(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def lists_of(fr):
    torch.cuda.synchronize()
    ni = int(fr.n_instances.item())
    return np_(fr.tile_start), np_(fr.ids[:ni])


def compare_lists(gts, gids, ots, oids, margin, T, tau=TAU_LIST):
    """Tile lists must match exactly. Both sides decide membership and depth
    order in FP64, so a difference is allowed only for a Gaussian one of whose
    list decisions (radius extent, rectangle edge, near plane) lies within tau
    of its threshold, where two FP64 evaluations may differ; common members
    must keep the same order. Returns the number of such exceptions."""
    if np.array_equal(gts, ots) and np.array_equal(gids, oids):
        return 0
    exceptions = 0
    for i in range(len(ots) - 1):
        a = gids[gts[i]:gts[i + 1]]
        b = oids[ots[i]:ots[i + 1]]
        if np.array_equal(a, b):
            continue
        sa, sb = set(a.tolist()), set(b.tolist())
        diff = sa ^ sb
        v = i // T
        for g in diff:
            assert margin[v, g] < tau, f"tile {i}: Gaussian {g} differs with list-decision margin {margin[v, g]}"
        exceptions += len(diff)
        ca = [x for x in a.tolist() if x in sb]
        cb = [x for x in b.tolist() if x in sa]
        assert ca == cb, f"tile {i}: order differs"
    return exceptions
