"""GPU parity of the residual-weighted sampler (Supp. E q_residual, stratified
per tile as in Sec. 4.4) through the C ABI: lmrs_residual_scores,
lmrs_sample and lmrs_lm_step with the residual sampler, against the oracle.

A draw is an integer decided by floating point: the GPU forms the tile's
cumulative distribution in FP32, the oracle in FP64, so a draw may differ
only where the oracle puts its uniform number within 1e-5 (in probability)
of an end of the chosen pixel's interval; every other draw must be
identical, and its weight within 1e-5 relative."""
import math

import numpy as np
import pytest
import torch

from gpu_util import DEV, gpu_frame, lib, log, np_, oracle_for, rel
from oracle.sampling import sample_residual
from oracle.solver import lm_step as oracle_lm_step
from oracle.solver import residual_scores
from paper_2504_12905_amd import synth

pytestmark = pytest.mark.gpu
MARGIN = 1e-5


def empty_frame(V, W, H, k, view_ids=None):
    """A frame used only for its sample buffers (one Gaussian, no projection)."""
    L = lib()
    beta = torch.zeros(synth.n_params(1, 0), device=DEV)
    cams = torch.tensor(synth.sphere_cameras(max(V, 8), 3.0, W, H, 60.0, 0), device=DEV)
    vid = None if view_ids is None else torch.tensor(np.asarray(view_ids, np.int32), device=DEV)
    return L.Frame(1, 0, beta, cams, W, H, V, view_ids=vid, k=k, sampled=True)


def compare_draws(gpix, gw, opix, ow, margin):
    same = gpix == opix
    near = margin < MARGIN
    assert np.all(same | near), f"{np.sum(~same & ~near)} draws differ away from an interval end"
    e = rel(gw[same], ow[same])
    assert e < 1e-5, e
    return int(np.sum(~same)), int(np.sum(near))


@pytest.mark.parametrize("k", [1, 13, 64, 256])
def test_residual_sampler_matches_oracle(k):
    V, W, H = 3, 160, 80
    view_ids = [5, 0, 7]
    fr = empty_frame(V, W, H, k, view_ids)
    T = fr.T
    rng = np.random.default_rng(k)
    scores = rng.uniform(0.0, 3.0, size=(V, T, 256)).astype(np.float32)
    scores[0, 3] = 0.0                                   # a flat tile
    scores[1, 7, 100] = 60.0                             # one dominant pixel
    L = lib()
    L.lmrs_sample(fr, L.SAMPLER_RESIDUAL, 987654321, 4, torch.tensor(scores, device=DEV))
    torch.cuda.synchronize()
    opix, ow, m = sample_residual(987654321, 4, view_ids, T, k, scores.astype(np.float64))
    diff, near = compare_draws(np_(fr.pix), np_(fr.w), opix, ow, m)
    log(f"  k={k}: {opix.size} draws, {near} within {MARGIN} of an interval end, {diff} differ")
    assert np.all(np_(fr.pix)[1, 7] == 100)


def test_residual_sampler_hot_pixel_frequency():
    """|r| = ln 255 on one pixel and 0 elsewhere: the GPU draws it with
    probability 1/2 (closed form), weight 2/k; others weight 510/k."""
    k = 64
    fr = empty_frame(1, 1024, 1024, k)
    sc = np.zeros((1, fr.T, 256), np.float32)
    sc[..., 31] = math.log(255.0)
    L = lib()
    L.lmrs_sample(fr, L.SAMPLER_RESIDUAL, 5, 0, torch.tensor(sc, device=DEV))
    pix, w = np_(fr.pix), np_(fr.w)
    frac = float(np.mean(pix == 31))
    log(f"  hot-pixel frequency {frac:.5f} over {pix.size} draws")
    assert abs(frac - 0.5) < 5 * math.sqrt(0.25 / pix.size)
    assert np.allclose(w[pix == 31], 2.0 / k, rtol=1e-5)
    assert np.allclose(w[pix != 31], 510.0 / k, rtol=1e-5)


@pytest.fixture(scope="module")
def cfg0():
    w = synth.config0()
    tg = oracle_for(w.n, 0, w.beta_gt, w.cams, w.width, w.height).render_image().astype(np.float32)
    return w, tg


def test_residual_scores_match_oracle(cfg0):
    w, tg = cfg0
    fr = gpu_frame(w.n, 0, w.beta_init, w.cams, w.width, w.height, render=False)
    sc = np_(lib().lmrs_residual_scores(fr, torch.tensor(tg, device=DEV)))
    ref = residual_scores(oracle_for(w.n, 0, w.beta_init, w.cams, w.width, w.height), tg)
    log(f"  scores rel {rel(sc, ref):.2e}")
    assert rel(sc, ref) < 1e-4


def test_residual_scores_medium_sh3():
    n, deg, W = 20000, 3, 256
    gt = synth.make_scene(n, deg, 21, means="ball")
    beta = synth.perturb_init(gt, n, deg, 21)
    cams = synth.sphere_cameras(5, 4.0, W, W, 60.0, 21)
    view_ids = [4, 1]
    tg = oracle_for(n, deg, gt, cams, W, W).render_image().astype(np.float32)
    fr = gpu_frame(n, deg, beta, cams, W, W, view_ids=view_ids, render=False)
    sc = np_(lib().lmrs_residual_scores(fr, torch.tensor(tg, device=DEV)))
    ref = residual_scores(oracle_for(n, deg, beta, cams[view_ids], W, W), tg[view_ids])
    log(f"  scores rel {rel(sc, ref):.2e}")
    assert rel(sc, ref) < 1e-4


def _seed_without_near_draws(w, tg, k, it):
    """First seed whose oracle draws all sit farther than MARGIN from an
    interval end (decided by the oracle alone)."""
    scores = residual_scores(oracle_for(w.n, 0, w.beta_init, w.cams, w.width, w.height), tg)
    for seed in range(200):
        _, _, m = sample_residual(seed, it, np.arange(4), 16, k, scores)
        if m.min() > MARGIN:
            return seed
    pytest.fail("no seed without near-boundary draws")


@pytest.mark.parametrize("k,it", [(4, 0), (4, 12)])
def test_lm_step_residual_sampler_cfg0(cfg0, k, it):
    w, tg = cfg0
    L = lib()
    seed = _seed_without_near_draws(w, tg, k, it)
    fr = L.Frame(w.n, 0, torch.tensor(w.beta_init, device=DEV), torch.tensor(w.cams, device=DEV), w.width,
                 w.height, 4, view_ids=torch.arange(4, dtype=torch.int32, device=DEV), k=k, sampled=True)
    rep = torch.zeros(L.REPORT_FLOATS, device=DEV)
    L.lmrs_lm_step(fr, torch.tensor(tg, device=DEV),
                   L.lm_params(it, 10, w.lam, seed=seed, sampler=L.SAMPLER_RESIDUAL), report=rep)
    b_gpu = np_(fr.beta)
    b_ref, info = oracle_lm_step(w.n, 0, w.beta_init, w.cams, tg, np.arange(4), w.width, w.height, k, seed,
                                 it, w.lam, 10, sampler="residual")
    assert np.array_equal(np_(fr.pix).reshape(-1), info["samples"])
    assert rel(np_(fr.w), info["weights"]) < 1e-5
    r = np_(rep)
    d_gpu = b_gpu.astype(np.float64) - w.beta_init
    d_ref = b_ref.astype(np.float64) - w.beta_init
    log(f"  seed {seed} k={k} it={it}: step rel {rel(d_gpu, d_ref):.2e}  eta {r[1]:.4f}/{info['eta']:.4f}  "
        f"loss {r[0]:.6e}/{info['loss_sampled']:.6e}")
    assert abs(r[0] - info["loss_sampled"]) <= 1e-4 * info["loss_sampled"]
    assert abs(r[1] - info["eta"]) <= 1e-3 * info["eta"]
    assert rel(d_gpu, d_ref) < 1e-3
