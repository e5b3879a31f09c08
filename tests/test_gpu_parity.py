"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bar (FP32 path vs FP64 oracle, norm-wise relative error ||a-b||/||b||):
* tile lists and depth order: bit-exact (both sides decide them in FP64; an
  exception is allowed only for a decision within 1e-9 of its threshold, and
  there are none);
* projection, render, J p, J^T u, GN product, diagonal: <= 1e-4 (J p per pixel on
  the pixels whose skip / cap / stop decisions are farther than 1e-4 from their
  thresholds, the rest having no unique derivative at FP32 precision);
* PCG solution: <= 1e-3 (FP32 CG recurrences drift from FP64 over iterations);
* sampler: bit-exact.
"""
import numpy as np
import pytest
import torch

from gpu_util import DEV, TAU_LIST, compare_lists, gpu_frame, lib, lists_of, log, np_, oracle_for, rel
from oracle.sampling import sample_uniform
from oracle.solver import lm_step as oracle_lm_step
from oracle.solver import pcg as oracle_pcg
from paper_2504_12905_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-4


class Case:
    def __init__(self, name, n, deg, beta, cams, W, H, k=256, pix=None, wts=None):
        self.name, self.n, self.deg, self.beta, self.cams, self.W, self.H = name, n, deg, beta, cams, W, H
        self.k, self.pix, self.wts = k, pix, wts
        log(f"[case] {name}: n={n} deg={deg} V={cams.shape[0]} {W}x{H} k={k}")
        self.fr = gpu_frame(n, deg, beta, cams, W, H, k, pix, wts)
        self.orc = oracle_for(n, deg, beta, cams, W, H, k, pix, wts)
        self.P = self.orc.P


def case_cfg0():
    w = synth.config0()
    return Case("cfg0-init", w.n, 0, w.beta_init, w.cams, w.width, w.height)


def case_medium_sampled():
    n, deg = 20000, 3
    gt = synth.make_scene(n, deg, 5, means="ball")
    beta = synth.perturb_init(gt, n, deg, 5)
    cams = synth.sphere_cameras(3, 4.0, 256, 256, 60.0, 5)
    T = 16 * 16
    pix, wts = sample_uniform(11, 0, np.arange(3), T, 26)
    return Case("medium-20k-sh3-3x256-k26", n, deg, beta, cams, 256, 256, 26, pix, wts)


@pytest.fixture(scope="module", params=["cfg0", "medium"])
def case(request):
    return case_cfg0() if request.param == "cfg0" else case_medium_sampled()


def test_projection(case):
    pr = case.orc.projection()
    rec = np_(case.fr.rec)
    vis = pr["visible"] > 0
    rect = np_(case.fr.rect)
    gvis = rect[..., 0] < rect[..., 2]
    # the FP64 camera depth (record words 9 = low, 11 = high): the oracle's
    # within a few FP64 spacings (both FP64, different operation order)
    z = ((rec[..., 11].view(np.uint32).astype(np.uint64) << np.uint64(32)) |
         rec[..., 9].view(np.uint32).astype(np.uint64)).view(np.float64)
    assert np.all(np.abs(z[vis] - pr["depth"][vis]) <= 4 * np.spacing(pr["depth"][vis]))
    bad = (vis != gvis) & (pr["margin"] >= TAU_LIST)
    assert not bad.any(), f"{bad.sum()} visibility mismatches"
    both = vis & gvis
    # the GPU record holds the conic's Cholesky factor (f11, f12, f22):
    # conic = F^T F = [[f11^2, f11 f12], [f11 f12, f12^2 + f22^2]]
    g = rec.astype(np.float64)
    conic = np.stack([g[..., 2] ** 2, g[..., 2] * g[..., 3], g[..., 3] ** 2 + g[..., 4] ** 2], axis=-1)
    g = np.concatenate([g[..., :2], conic, g[..., 5:9]], axis=-1)
    for q, name in enumerate(["u", "v", "A", "B", "C", "opacity", "r", "g", "b"]):
        e = rel(g[..., q][both], pr["rec"][..., q][both])
        log(f"  rec[{name}] rel {e:.2e}")
        assert e < TOL, name
    same_r = (rec[..., 10][both] == pr["radius"][both])
    assert np.all(same_r | (pr["margin"][both] < TAU_LIST))


def test_tile_lists(case):
    gts, gids = lists_of(case.fr)
    ots, oids = case.orc.lists()
    ex = compare_lists(gts, gids, ots, oids, case.orc.projection()["margin"], case.orc.T)
    log(f"  {case.name}: {oids.size} list entries, {ex} margin exceptions")
    assert ex == 0


def test_render(case):
    out = case.orc.render()
    C = np_(case.fr.color)
    T = np_(case.fr.trans)
    last = np_(case.fr.last)
    log(f"  color rel {rel(C, out['C']):.2e}  T rel {rel(T, out['T']):.2e}  "
        f"last equal {np.mean(last == out['last']):.6f}")
    assert rel(C, out["C"]) < TOL
    assert rel(T, out["T"]) < TOL
    assert np.mean(last == out["last"]) > 0.999


def test_jvp(case):
    rng = np.random.default_rng(1)
    p = rng.normal(size=case.P).astype(np.float32)
    jp = np_(lib().lmrs_jvp(case.fr, torch.tensor(p, device=DEV)))
    ref = case.orc.jvp(p)
    ok = case.orc.decided()
    log(f"  jvp rel {rel(jp[ok], ref[ok]):.2e} on decided pixels ({1 - ok.mean():.4%} within 1e-4 of a threshold)")
    assert rel(jp[ok], ref[ok]) < TOL


def test_vjp(case):
    rng = np.random.default_rng(2)
    u = rng.normal(size=(case.orc.S, 3)).astype(np.float32)
    out = np_(lib().lmrs_vjp(case.fr, torch.tensor(u, device=DEV)))
    ref = case.orc.vjp(u)
    log(f"  vjp rel {rel(out, ref):.2e}")
    assert rel(out, ref) < TOL


def test_adjoint_identity_on_gpu(case):
    L = lib()
    g = torch.Generator(device="cpu").manual_seed(3)
    p = torch.randn(case.P, generator=g).to(DEV)
    u = torch.randn(case.orc.S, 3, generator=g).to(DEV)
    jp = L.lmrs_jvp(case.fr, p)
    jtu = L.lmrs_vjp(case.fr, u)
    lhs = float((jp.double() * u.double()).sum())
    rhs = float((p.double() * jtu.double()).sum())
    log(f"  <Jp,u>={lhs:.8e} <p,J^T u>={rhs:.8e}")
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_gn_product(case):
    rng = np.random.default_rng(4)
    p = rng.normal(size=case.P).astype(np.float32)
    lam = 0.1
    d = rng.uniform(0.5, 2.0, size=case.P).astype(np.float32)
    L = lib()
    out = np_(L.lmrs_gn_product(case.fr, torch.tensor(p, device=DEV), lam))
    ref = case.orc.gn(p, lam)
    log(f"  gn rel {rel(out, ref):.2e}")
    assert rel(out, ref) < TOL
    out_d = np_(L.lmrs_gn_product(case.fr, torch.tensor(p, device=DEV), lam, torch.tensor(d, device=DEV)))
    assert rel(out_d, case.orc.gn(p, lam, d)) < TOL


def test_gn_diag(case):
    D = np_(lib().lmrs_gn_diag(case.fr))
    ref = case.orc.diag()
    log(f"  diag rel {rel(D, ref):.2e}")
    assert rel(D, ref) < TOL


def test_pcg(case):
    rng = np.random.default_rng(5)
    lam = 0.1
    b = (case.orc.vjp(rng.normal(size=(case.orc.S, 3)))).astype(np.float32)
    iters = 8
    rep = torch.zeros(8, device=DEV)
    x = np_(lib().lmrs_pcg(case.fr, torch.tensor(b, device=DEV), lam, iters, report=rep))
    D = case.orc.diag()
    xr, norms, done = oracle_pcg(lambda q: case.orc.gn(q, lam), b.astype(np.float64), 1.0 / (D + lam), iters)
    r = np_(rep)
    log(f"  pcg rel {rel(x, xr):.2e}  done {r[3]:.0f}/{done}  r0 {r[4]:.4e}/{norms[0]:.4e}  "
        f"rN {r[5]:.4e}/{norms[-1]:.4e}")
    assert rel(x, xr) < 1e-3
    assert r[3] == done
    assert abs(r[4] - norms[0]) <= 1e-4 * norms[0]
    assert float(b @ x) > 0


def test_pcg_unaligned_output(case):
    """x at an address that is not 16-byte aligned takes the scalar PCG vector
    kernels; the result matches the vectorised run (both FP32 recurrences with
    FP64 dot products, in different summation orders)."""
    rng = np.random.default_rng(6)
    b = torch.tensor(case.orc.vjp(rng.normal(size=(case.orc.S, 3))).astype(np.float32), device=DEV)
    x_al = np_(lib().lmrs_pcg(case.fr, b, 0.1, 8))
    buf = torch.zeros(case.P + 1, device=DEV)
    x_un = buf[1:]
    assert x_un.data_ptr() % 16 != 0
    lib().lmrs_pcg(case.fr, b, 0.1, 8, x=x_un)
    e = rel(np_(x_un), x_al)
    log(f"  unaligned vs aligned PCG rel {e:.2e}")
    assert e < 1e-4


def test_sampler_bit_exact():
    L = lib()
    cams = synth.sphere_cameras(6, 4.0, 128, 96, 60.0, 0)
    view_ids = np.array([5, 0, 3], np.int32)
    n, deg = 10, 0
    beta = synth.make_scene(n, deg, 0)
    fr = L.Frame(n, deg, torch.tensor(beta, device=DEV), torch.tensor(cams, device=DEV), 128, 96, 3,
                 view_ids=torch.tensor(view_ids, device=DEV), k=26, sampled=True)
    targets = torch.zeros((6, 96, 128, 3), device=DEV)
    prm = L.lm_params(7, 0, 0.1, seed=123456789012)
    L.lmrs_lm_step(fr, targets, prm)
    torch.cuda.synchronize()
    pix, w = sample_uniform(123456789012, 7, view_ids, fr.T, 26)
    assert np.array_equal(np_(fr.pix), pix)
    assert np.array_equal(np_(fr.w), w)


def targets_of(n, deg, beta_gt, cams, W, H):
    o = oracle_for(n, deg, beta_gt, cams, W, H)
    return o.render_image().astype(np.float32)


@pytest.mark.parametrize("k", [256, 64])
def test_lm_step_cfg0(k):
    w = synth.config0()
    L = lib()
    tg = targets_of(w.n, 0, w.beta_gt, w.cams, w.width, w.height)
    for it in (0, 12):
        fr = L.Frame(w.n, 0, torch.tensor(w.beta_init, device=DEV), torch.tensor(w.cams, device=DEV),
                     w.width, w.height, 4, view_ids=torch.arange(4, dtype=torch.int32, device=DEV), k=k,
                     sampled=k < 256)
        rep = torch.zeros(8, device=DEV)
        L.lmrs_lm_step(fr, torch.tensor(tg, device=DEV), L.lm_params(it, 10, w.lam, seed=3), report=rep)
        b_gpu = np_(fr.beta)
        b_ref, info = oracle_lm_step(w.n, 0, w.beta_init, w.cams, tg, np.arange(4), w.width, w.height, k, 3,
                                     it, w.lam, 10)
        d_gpu = b_gpu.astype(np.float64) - w.beta_init
        d_ref = b_ref.astype(np.float64) - w.beta_init
        r = np_(rep)
        log(f"  k={k} it={it}: step rel {rel(d_gpu, d_ref):.2e}  eta {r[1]:.4f}/{info['eta']:.4f}  "
            f"loss {r[0]:.6e}/{info['loss_sampled']:.6e}")
        assert abs(r[0] - info["loss_sampled"]) <= 1e-4 * info["loss_sampled"]
        assert abs(r[1] - info["eta"]) <= 1e-3 * info["eta"]
        assert rel(d_gpu, d_ref) < 1e-3
