"""The SSIM residual with the diagonal approximation (Supp. B; Sec. 6)
through the C ABI against the FP64 oracle (oracle/ssim.py, oracle/solver.py):

* lmrs_ssim_residual: the full render of the batch views, and at the samples
  u = w (r + s delta rho) and wc = w (1 + s delta^2), for every pixel and for
  26 samples per tile, with windows clipped at the image border;
* the Gauss-Newton operator with per-channel weights (over the blend table
  and over the lists) and its diagonal with their channel mean;
* LM steps with ssim_weight 0.2 from identical parameters, and ssim_weight 0
  on a frame holding the SSIM buffers (the colour residual alone)."""
import numpy as np
import pytest
import torch
from scipy.ndimage import maximum_filter

from gpu_util import DEV, elem, gpu_frame, lib, log, np_, oracle_for, rel
from oracle.sampling import sample_uniform
from oracle.solver import lm_step as oracle_lm_step
from oracle.ssim import WINDOW, residual_and_weights, ssim_terms
from paper_2504_12905_amd import synth

pytestmark = pytest.mark.gpu

S_W = 0.2


def _scene(k, seed=11, n=3000, deg=2, W=128, H=96, V=2):
    gt = synth.make_scene(n, deg, seed, means="ball")
    beta = synth.perturb_init(gt, n, deg, seed)
    cams = synth.sphere_cameras(V, 4.0, W, H, 60.0, seed)
    T = (W // 16) * (H // 16)
    pix, wts = (None, None) if k == 256 else sample_uniform(seed, 0, np.arange(V), T, k)
    target = oracle_for(n, deg, gt, cams, W, H).render_image()
    return n, deg, beta, cams, W, H, pix, wts, target.astype(np.float32)


def _window_decided(n, deg, beta, cams, W, H, orc):
    """Samples of orc whose whole SSIM window holds pixels with decided blends
    (their FP32 and FP64 colours agree to rounding)."""
    full = oracle_for(n, deg, beta, cams, W, H)
    dec = full.decided()
    v, x, y = full.pixel_coords()
    und = np.zeros((full.V, H, W), bool)
    und[v, y, x] = ~dec
    und = maximum_filter(und, size=(1, WINDOW, WINDOW), mode="constant", cval=False)
    sv, sx, sy = orc.pixel_coords()
    return ~und[sv, sy, sx]


@pytest.mark.parametrize("k", [256, 26])
def test_ssim_residual_matches_oracle(k):
    L = lib()
    n, deg, beta, cams, W, H, pix, wts, target = _scene(k)
    fr = gpu_frame(n, deg, beta, cams, W, H, k, pix, wts, ssim=True)
    tg = torch.tensor(target, device=DEV)
    tile_loss = torch.zeros(fr.n_views * fr.T, dtype=torch.float64, device=DEV)
    u = np_(L.lmrs_ssim_residual(fr, tg, S_W, tile_loss=tile_loss))
    wc = np_(fr.wc)
    img = np_(fr.image)
    orc = oracle_for(n, deg, beta, cams, W, H, k, pix, wts)
    img_ref = oracle_for(n, deg, beta, cams, W, H).render_image()
    u_ref, wc_ref, _ = residual_and_weights(orc, img_ref, target.astype(np.float64), orc.weights(), s=S_W)
    ok = _window_decided(n, deg, beta, cams, W, H, orc)
    e_img, e_u, e_wc = rel(img, img_ref), rel(u, u_ref), rel(wc, wc_ref)
    eu_d, ewc_d = elem(u[ok], u_ref[ok]), elem(wc[ok], wc_ref[ok])
    v, x, y = orc.pixel_coords()
    tg64 = target.astype(np.float64)
    rho = 1.0 - ssim_terms(img_ref, tg64)[0][v, y, x]
    r = img_ref[v, y, x] - tg64[v, y, x]
    loss_ref = float(np.sum(orc.weights()[:, None] * (r ** 2 + S_W * rho ** 2)))
    loss = float(np_(tile_loss).sum())
    log(f"  k={k}: image rel {e_img:.2e}; u rel {e_u:.2e} (decided windows {ok.mean():.4f}: element-wise "
        f"{eu_d:.2e}); wc rel {e_wc:.2e} (element-wise {ewc_d:.2e}); objective {loss:.6e}/{loss_ref:.6e}")
    assert e_img < 1e-5
    assert e_u < 1e-4 and e_wc < 1e-5
    assert eu_d < 1e-3 and ewc_d < 1e-5
    assert abs(loss - loss_ref) <= 1e-5 * loss_ref


@pytest.mark.parametrize("k", [256, 26])
def test_channel_weighted_operator_and_diagonal(k):
    L = lib()
    n, deg, beta, cams, W, H, pix, wts, target = _scene(k, seed=12)
    fr = gpu_frame(n, deg, beta, cams, W, H, k, pix, wts, ssim=True)
    L.lmrs_ssim_residual(fr, torch.tensor(target, device=DEV), S_W)
    lam = 0.05
    p = torch.tensor(np.random.default_rng(k).normal(size=fr.P).astype(np.float32), device=DEV)
    out_walk = np_(L.lmrs_gn_product(fr, p, lam))
    diag = np_(L.lmrs_gn_diag(fr))
    assert fr.blend_built()   # the diagonal pass wrote the table
    out_tab = np_(L.lmrs_gn_product(fr, p, lam))
    orc = oracle_for(n, deg, beta, cams, W, H, k, pix, wts)
    img_ref = oracle_for(n, deg, beta, cams, W, H).render_image()
    _, wc_ref, wbar_ref = residual_and_weights(orc, img_ref, target.astype(np.float64), orc.weights(), s=S_W)
    orc.set_samples(k, pix, wbar_ref)
    diag_ref = orc.diag()
    orc.set_channel_weights(wc_ref)
    ref = orc.gn(np_(p).astype(np.float64), lam)
    e_t, e_w, e_tw, e_d = rel(out_tab, ref), rel(out_walk, ref), rel(out_tab, out_walk), rel(diag, diag_ref)
    log(f"  k={k}: GN with wc: table {e_t:.2e}, walk {e_w:.2e}, table vs walk {e_tw:.2e}; diag(wbar) {e_d:.2e}")
    assert e_t < 1e-4 and e_w < 1e-4 and e_tw < 2e-5 and e_d < 1e-4


@pytest.mark.parametrize("k", [256, 64])
def test_lm_step_with_ssim_cfg0(k):
    w = synth.config0()
    L = lib()
    tg = oracle_for(w.n, 0, w.beta_gt, w.cams, w.width, w.height).render_image().astype(np.float32)
    for it in (0, 12):
        fr = L.Frame(w.n, 0, torch.tensor(w.beta_init, device=DEV), torch.tensor(w.cams, device=DEV),
                     w.width, w.height, 4, view_ids=torch.arange(4, dtype=torch.int32, device=DEV), k=k,
                     sampled=k < 256, ssim=True)
        rep = torch.zeros(L.REPORT_FLOATS, device=DEV)
        L.lmrs_lm_step(fr, torch.tensor(tg, device=DEV), L.lm_params(it, 10, w.lam, seed=3, ssim_weight=S_W),
                       report=rep)
        b_ref, info = oracle_lm_step(w.n, 0, w.beta_init, w.cams, tg, np.arange(4), w.width, w.height, k, 3,
                                     it, w.lam, 10, ssim_weight=S_W)
        d_gpu = np_(fr.beta).astype(np.float64) - w.beta_init
        d_ref = b_ref.astype(np.float64) - w.beta_init
        r = np_(rep)
        log(f"  k={k} it={it}: step rel {rel(d_gpu, d_ref):.2e}  eta {r[1]:.4f}/{info['eta']:.4f}  "
            f"loss {r[0]:.6e}/{info['loss_sampled']:.6e}")
        assert abs(r[0] - info["loss_sampled"]) <= 1e-4 * info["loss_sampled"]
        assert abs(r[1] - info["eta"]) <= 1e-3 * info["eta"]
        assert rel(d_gpu, d_ref) < 1e-3


def test_zero_ssim_weight_is_the_colour_residual():
    """ssim_weight 0 on a frame holding SSIM buffers (wc left from an SSIM
    step) takes the plain colour-residual step, bit for bit (both frames with
    deterministic accumulation, so float-atomic order cannot tell them apart);
    lmrs_ssim_residual with s = 0 gives u = w r and wc = w."""
    w = synth.config0()
    L = lib()
    tg = oracle_for(w.n, 0, w.beta_gt, w.cams, w.width, w.height).render_image().astype(np.float32)
    tgt = torch.tensor(tg, device=DEV)
    steps = []
    for ssim in (False, True):
        fr = L.Frame(w.n, 0, torch.tensor(w.beta_init, device=DEV), torch.tensor(w.cams, device=DEV),
                     w.width, w.height, 4, view_ids=torch.arange(4, dtype=torch.int32, device=DEV), k=64,
                     sampled=True, ssim=ssim, deterministic=True)
        if ssim:
            fr.wc.fill_(7.0)   # stale weights of an earlier step must not enter
        L.lmrs_lm_step(fr, tgt, L.lm_params(0, 10, w.lam, seed=3))
        steps.append(np_(fr.beta).astype(np.float64) - w.beta_init)
    log(f"  ssim_weight 0 with and without SSIM buffers: identical steps {np.array_equal(steps[1], steps[0])} "
        f"(step rel {rel(steps[1], steps[0]):.2e})")
    assert np.array_equal(steps[1], steps[0])
    n, deg, beta, cams, W, H, pix, wts, target = _scene(26, seed=13)
    fr = gpu_frame(n, deg, beta, cams, W, H, 26, pix, wts, ssim=True)
    u = np_(L.lmrs_ssim_residual(fr, torch.tensor(target, device=DEV), 0.0))
    orc = oracle_for(n, deg, beta, cams, W, H, 26, pix, wts)
    v, x, y = orc.pixel_coords()
    r = np_(fr.image)[v, y, x].astype(np.float64) - target[v, y, x]
    wv = np.asarray(wts, np.float64).reshape(-1)
    np.testing.assert_allclose(u, wv[:, None] * r, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(np_(fr.wc), np.repeat(wv[:, None], 3, axis=1), rtol=1e-7)
