"""lmrs_gn_product_noalloc (the GN product without a workspace, for callers
that cannot allocate) against lmrs_gn_product on the same frames, through
the C ABI: two calls in a row on the same GPU, the second on a smaller
frame (the static scratch then still holds the first call's values), each
checked against the workspace entry point and against the FP64 oracle; and
a frame larger than the static array is rejected on the host."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, gpu_frame, lib, log, np_, oracle_for, rel
from oracle.sampling import sample_uniform
from paper_2504_12905_amd import synth

pytestmark = pytest.mark.gpu


def _medium():
    """20k Gaussians, SH 3, 3 views 256x256, 26 samples per tile."""
    n, deg = 20000, 3
    gt = synth.make_scene(n, deg, 5, means="ball")
    beta = synth.perturb_init(gt, n, deg, 5)
    cams = synth.sphere_cameras(3, 4.0, 256, 256, 60.0, 5)
    pix, wts = sample_uniform(11, 0, np.arange(3), 16 * 16, 26)
    return "medium-20k-sh3-3x256-k26", n, deg, beta, cams, 256, 256, 26, pix, wts, 0.1


def _small():
    w = synth.config0()
    return w.name, w.n, 0, w.beta_init, w.cams, w.width, w.height, 256, None, None, w.lam


def test_noalloc_matches_workspace_entry_point_twice():
    """The larger frame first, then the smaller one: the second call finds the
    first call's values in the scratch array and must not depend on them."""
    L = lib()
    for name, n, deg, beta, cams, W, H, k, pix, wts, lam in (_medium(), _small()):
        fr = gpu_frame(n, deg, beta, cams, W, H, k, pix, wts)
        p = torch.tensor(np.random.default_rng(5).normal(size=fr.P).astype(np.float32), device=DEV)
        out_ws = L.lmrs_gn_product(fr, p, lam)
        out_na = torch.full((fr.P,), float("nan"), device=DEV)
        L.lmrs_gn_product_noalloc(fr, p, lam, out_na)
        torch.cuda.synchronize()
        a, b = np_(out_na), np_(out_ws)
        orc = oracle_for(n, deg, beta, cams, W, H, k, pix, wts)
        ref = orc.gn(np_(p).astype(np.float64), lam)
        e_ws, e_or = rel(a, b), rel(a, ref)
        log(f"  {name}: no-alloc vs workspace entry point {e_ws:.2e}, vs oracle {e_or:.2e}")
        assert np.all(np.isfinite(a))
        assert e_ws < 1e-5 and e_or < 1e-4


def test_noalloc_rejects_frames_beyond_the_array():
    L = lib()
    w = synth.config0()
    fr = gpu_frame(w.n, w.sh_degree, w.beta_init, w.cams, w.width, w.height)
    fs = fr.struct()
    fs.n = 2_000_000  # 4 views x 2M Gaussians: ~900 MB of scratch; rejected before any launch
    import ctypes as C
    p = torch.zeros(fr.P, device=DEV)
    st = L._lib.lmrs_gn_product_noalloc(C.byref(fs), C.byref(L.default_opts()), L._ptr(p), 0.1, None, L._ptr(p + 1),
                                        L._stream(None))
    assert st == L.LMRS_EWORKSPACE
    assert b"static array" in L._lib.lmrs_last_error()
