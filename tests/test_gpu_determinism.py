"""Deterministic accumulation (lmrs_frame.deterministic = 1): the sums over
tiles (screen gradients of J^T u and of b, Gram blocks of the diagonal) and
the blend table's per-pixel sums of J p are fixed-point integer sums, so the
order of the adds no longer shows in the result. Through the C ABI:

* GN products over the list walk and over the blend table: repeated calls
  give the same bits; the result matches the float-atomic mode (FP32 noise)
  and the FP64 oracle (1e-4 norm-wise, like every GN parity test);
* J^T u and diag(J^T W J): the same bits on repeat; oracle bars as above;
* LM steps at lambda = 1e-3 from the same state give the same parameters bit
  for bit after every step (the float mode's run-to-run spread is logged);
* a term beyond the fixed-point range (|term| >= 2^30) turns its rows into
  NaN instead of wrapping, so the non-finite checks downstream see it.
The scene is the 20k-Gaussian SH-3 one of the autograd tests (4 views of
256x256, 26 samples per tile)."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, gpu_frame, lib, log, np_, oracle_for, rel
from oracle.sampling import sample_uniform
from paper_2504_12905_amd import synth

pytestmark = pytest.mark.gpu

N, DEG, W, V, K = 20000, 3, 256, 4, 26


@pytest.fixture(scope="module")
def scene():
    gt = synth.make_scene(N, DEG, 9, means="ball")
    beta = synth.perturb_init(gt, N, DEG, 9)
    cams = synth.sphere_cameras(V, 4.0, W, W, 60.0, 9)
    T = (W // 16) ** 2
    pix, wts = sample_uniform(9, 0, np.arange(V), T, K)
    return gt, beta, cams, pix, wts


def same_bits(a: torch.Tensor, b: torch.Tensor) -> bool:
    return torch.equal(a.view(torch.int32), b.view(torch.int32))


def test_gn_product_repeats_bit_for_bit(scene):
    L = lib()
    _, beta, cams, pix, wts = scene
    fr = gpu_frame(N, DEG, beta, cams, W, W, K, pix, wts)
    orc = oracle_for(N, DEG, beta, cams, W, W, K, pix, wts)
    lam = 0.05
    p = torch.tensor(np.random.default_rng(4).normal(size=fr.P).astype(np.float32), device=DEV)
    ref = orc.gn(np_(p).astype(np.float64), lam)
    for path in ("walk", "table"):
        if path == "table":
            L.lmrs_linearize(fr)
            assert fr.blend_built()
        else:
            assert not fr.blend_built()
        fr.deterministic = False
        flt = [L.lmrs_gn_product(fr, p, lam).clone() for _ in range(3)]
        fr.deterministic = True
        det = [L.lmrs_gn_product(fr, p, lam).clone() for _ in range(3)]
        torch.cuda.synchronize()
        flt_same = all(same_bits(flt[0], x) for x in flt[1:])
        e_ref, e_flt = rel(np_(det[0]), ref), rel(np_(det[0]), np_(flt[0]))
        log(f"  {path}: deterministic vs oracle {e_ref:.2e}, vs float atomics {e_flt:.2e}; "
            f"float-atomic repeats identical: {flt_same}")
        assert all(same_bits(det[0], x) for x in det[1:])
        assert e_ref < 1e-4 and e_flt < 2e-5
    fr.deterministic = False


def test_vjp_and_diag_repeat_bit_for_bit(scene):
    L = lib()
    _, beta, cams, pix, wts = scene
    fr = gpu_frame(N, DEG, beta, cams, W, W, K, pix, wts)
    orc = oracle_for(N, DEG, beta, cams, W, W, K, pix, wts)
    u = torch.tensor(np.random.default_rng(6).normal(size=(fr.S, 3)).astype(np.float32), device=DEV)
    fr.deterministic = True
    g = [L.lmrs_vjp(fr, u).clone() for _ in range(2)]
    dg = [L.lmrs_gn_diag(fr).clone() for _ in range(2)]
    torch.cuda.synchronize()
    assert same_bits(g[0], g[1]) and same_bits(dg[0], dg[1])
    e_g = rel(np_(g[0]), orc.vjp(np_(u).astype(np.float64)))
    e_d = rel(np_(dg[0]), orc.diag())
    fr.deterministic = False
    e_gf = rel(np_(g[0]), np_(L.lmrs_vjp(fr, u)))
    e_df = rel(np_(dg[0]), np_(L.lmrs_gn_diag(fr)))
    log(f"  J^T u vs oracle {e_g:.2e} (vs float {e_gf:.2e}); diag vs oracle {e_d:.2e} (vs float {e_df:.2e})")
    assert e_g < 1e-4 and e_d < 1e-4 and e_gf < 2e-5 and e_df < 2e-5


def _targets(gt, cams):
    L = lib()
    tf = L.Frame(N, DEG, torch.tensor(gt, device=DEV), torch.tensor(cams, device=DEV), W, W, V, blend=False)
    L.lmrs_project(tf)
    L.lmrs_bin_tiles(tf)
    L.lmrs_render(tf)
    TX = W // 16
    t = torch.arange(tf.T, device=DEV)
    q = torch.arange(256, device=DEV)
    y = ((t // TX) * 16)[:, None] + (q // 16)[None, :]
    x = ((t % TX) * 16)[:, None] + (q % 16)[None, :]
    col = tf.color.view(V, tf.T, 256, 3)
    tg = torch.empty((V, W, W, 3), device=DEV)
    for v in range(V):
        tg[v, y, x] = col[v]
    return tg


def test_lm_steps_repeat_bit_for_bit(scene):
    L = lib()
    gt, beta, cams, _, _ = scene
    tg = _targets(gt, cams)
    lam, steps = 1e-3, 5

    def run(det):
        fr = L.Frame(N, DEG, torch.tensor(beta, device=DEV), torch.tensor(cams, device=DEV), W, W, V,
                     view_ids=torch.arange(V, dtype=torch.int32, device=DEV), k=K, sampled=True,
                     deterministic=det)
        rep = torch.zeros(L.REPORT_FLOATS, device=DEV)
        out = []
        for it in range(steps):
            L.lmrs_lm_step(fr, tg, L.lm_params(it, 8, lam, seed=11), report=rep)
            out.append(fr.beta.clone())
        torch.cuda.synchronize()
        L.check_report(rep)
        return out, float(rep[0].item())

    a, loss = run(True)
    b, _ = run(True)
    f1, _ = run(False)
    f2, _ = run(False)
    spread = [rel(np_(x), np_(y)) for x, y in zip(f1, f2)]
    gap = rel(np_(a[-1]), np_(f1[-1]))
    log(f"  {steps} LM steps at lambda {lam}: last sampled loss {loss:.4e}; deterministic runs identical: "
        f"{all(same_bits(x, y) for x, y in zip(a, b))}; float-atomic runs apart by {spread[-1]:.2e} "
        f"(per step {', '.join(f'{s:.1e}' for s in spread)}); deterministic vs float {gap:.2e}")
    assert all(same_bits(x, y) for x, y in zip(a, b))
    assert np.all(np.isfinite(np_(a[-1])))


def test_out_of_range_terms_poison_their_rows(scene):
    L = lib()
    _, beta, cams, pix, wts = scene
    fr = gpu_frame(N, DEG, beta, cams, W, W, K, pix, wts)
    u = torch.full((fr.S, 3), 1e12, device=DEV)
    fr.deterministic = False
    big = np_(L.lmrs_vjp(fr, u))
    fr.deterministic = True
    det = np_(L.lmrs_vjp(fr, u))
    ok = np.isfinite(det)
    log(f"  u = 1e12: float mode finite {np.isfinite(big).all()}, deterministic mode NaN entries "
        f"{(~ok).sum()} of {det.size}")
    assert np.isfinite(big).all()
    assert (~ok).any()
    # poisoned entries are NaN (no wrapped or infinite values), and only
    # where the float mode accumulated something
    assert np.all(np.isnan(det[~ok])) and np.all(big[~ok] != 0)
    fr.deterministic = False


def test_noalloc_and_ssim_products_repeat_bit_for_bit(scene):
    """The no-workspace entry point gives the workspace entry point's bits in
    deterministic mode (same kernels, same fixed-point rows, in its static
    array); with the SSIM residual's per-channel operator weights the product
    repeats bit for bit too."""
    L = lib()
    gt, beta, cams, pix, wts = scene
    fr = gpu_frame(N, DEG, beta, cams, W, W, K, pix, wts)
    L.lmrs_linearize(fr)
    p = torch.tensor(np.random.default_rng(8).normal(size=fr.P).astype(np.float32), device=DEV)
    fr.deterministic = True
    a = L.lmrs_gn_product(fr, p, 0.05).clone()
    b = L.lmrs_gn_product_noalloc(fr, p, 0.05, torch.empty_like(p)).clone()
    torch.cuda.synchronize()
    assert same_bits(a, b)
    fs = gpu_frame(N, DEG, beta, cams, W, W, K, pix, wts, ssim=True)
    L.lmrs_ssim_residual(fs, _targets(gt, cams), 0.2)   # sets the operator weights wc
    L.lmrs_linearize(fs)
    fs.deterministic = True
    c = L.lmrs_gn_product(fs, p, 0.05).clone()
    d = L.lmrs_gn_product(fs, p, 0.05).clone()
    fs.deterministic = False
    f = L.lmrs_gn_product(fs, p, 0.05).clone()
    torch.cuda.synchronize()
    e = rel(np_(c), np_(f))
    log(f"  no-alloc = workspace bits: True; SSIM-weighted product repeats identical {same_bits(c, d)}, "
        f"vs float atomics {e:.2e}, vs unweighted {rel(np_(c), np_(a)):.2e}")
    assert same_bits(c, d) and e < 2e-5 and not same_bits(c, a)
