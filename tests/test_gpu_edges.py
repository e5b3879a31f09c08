"""GPU edge cases against the oracle: culled scenes, a single Gaussian, one
sample per tile, a tile list longer than one LDS sort chunk (merge path) and
empty tiles."""
import math

import numpy as np
import pytest
import torch

from gpu_util import DEV, compare_lists, gpu_frame, lib, lists_of, log, np_, oracle_for, rel
from oracle.sampling import sample_uniform
from paper_2504_12905_amd import synth
from test_oracle_geometry import axis_camera, one_gaussian_scene

pytestmark = pytest.mark.gpu


def check_all(name, n, deg, beta, cams, W, H, k=256, pix=None, wts=None, lam=0.05):
    log(f"[edge] {name}")
    fr = gpu_frame(n, deg, beta, cams, W, H, k, pix, wts)
    orc = oracle_for(n, deg, beta, cams, W, H, k, pix, wts)
    gts, gids = lists_of(fr)
    ots, oids = orc.lists()
    assert compare_lists(gts, gids, ots, oids, orc.projection()["margin"], orc.T) == 0
    ref = orc.render()
    assert rel(np_(fr.color), ref["C"]) < 1e-4 or np.linalg.norm(ref["C"]) == 0
    p = np.random.default_rng(0).normal(size=orc.P).astype(np.float32)
    out = np_(lib().lmrs_gn_product(fr, torch.tensor(p, device=DEV), lam))
    e = rel(out, orc.gn(p, lam))
    log(f"  lists {oids.size}  gn rel {e:.2e}")
    assert e < 1e-4
    return fr, orc


def test_everything_culled():
    # all Gaussians behind the camera or off-screen: empty lists, background render, out = lam p
    n, beta = one_gaussian_scene([[0, 0, -3.5], [50, 0, 0], [0, 0, -3.0]], [math.log(0.1)] * 3,
                                 [1, 0, 0, 0], 0.0, [0.5, 0.5, 0.5])
    fr, orc = check_all("culled", n, 0, beta, axis_camera(40.0, 32, 32), 32, 32)
    assert int(fr.n_instances.item()) == 0
    assert np.all(np_(fr.last) == -1) and np.all(np_(fr.trans) == 1.0)


def test_single_gaussian_sh2():
    rng = np.random.default_rng(0)
    n, beta = one_gaussian_scene([0.05, -0.02, 0.1], [-2.0, -2.3, -1.9], [0.9, 0.1, -0.3, 0.2], 0.4,
                                 [0.7, 0.2, 0.4], sh_degree=2, sh_rest=rng.normal(0, 0.1, size=(8, 3, 1)))
    check_all("single-sh2", n, 2, beta, axis_camera(60.0, 48, 48), 48, 48)


def test_one_sample_per_tile():
    w = synth.config0()
    pix, wts = sample_uniform(4, 2, np.arange(4), 16, 1)
    check_all("cfg0-k1", w.n, 0, w.beta_init, w.cams, w.width, w.height, 1, pix, wts)


def test_long_tile_list():
    # 6000 small Gaussians in front of one tile: a long list, sorted by several radix passes whose
    # four wave parts each hold 1,500 entries
    rng = np.random.default_rng(7)
    n, f = 6000, 120.0
    zc = rng.uniform(2.0, 4.0, n)                 # camera depth
    u, v = rng.uniform(35.0, 45.0, n), rng.uniform(35.0, 45.0, n)   # inside tile (2, 2) with margin
    mu = np.stack([(u - 32.0) * zc / f, (v - 32.0) * zc / f, zc - 3.0], 1)
    n, beta = one_gaussian_scene(mu, [math.log(0.004)] * 3, [1, 0, 0, 0], -1.0, [0.3, 0.6, 0.9])
    beta[synth.seg(n, "log_scale")] += rng.normal(0, 0.1, size=3 * n)
    fr, orc = check_all("long-list", n, 0, beta, axis_camera(f, 64, 64), 64, 64)
    ts = np_(fr.tile_start)
    assert np.diff(ts).max() > 4096


def _one_tile_cloud(n, seed, f=120.0, W=64):
    """n small Gaussians whose footprints all fall inside tile (2, 2) of a WxW view."""
    rng = np.random.default_rng(seed)
    zc = rng.uniform(2.0, 4.0, n)
    u, v = rng.uniform(35.0, 45.0, n), rng.uniform(35.0, 45.0, n)
    mu = np.stack([(u - 32.0) * zc / f, (v - 32.0) * zc / f, zc - 3.0], 1)
    n, beta = one_gaussian_scene(mu, [math.log(0.004)] * 3, [1, 0, 0, 0], -1.0, [0.3, 0.6, 0.9])
    return n, beta, axis_camera(f, W, W)


def test_list_of_twelve_thousand():
    """12,000 entries in one tile (14-bit depth ranks: two radix passes, the
    second on 6-bit digits)."""
    n, beta, cams = _one_tile_cloud(12000, 8)
    fr, orc = check_all("three-chunk list", n, 0, beta, cams, 64, 64)
    assert np.diff(np_(fr.tile_start)).max() == 12000


def test_four_million_entry_tile_lists():
    """4.2 M entries in one tile: a 4.2M-Gaussian view sort and 23-bit depth
    ranks (three radix passes of a 4.2M-entry segment). Lists only (bit-exact
    against the oracle)."""
    n, beta, cams = _one_tile_cloud(4_200_000, 9)
    log("[edge] 4.2M-entry tile")
    fr = gpu_frame(n, 0, beta, cams, 64, 64, render=False)
    gts, gids = lists_of(fr)
    orc = oracle_for(n, 0, beta, cams, 64, 64)
    ots, oids = orc.lists()
    assert np.diff(ots).max() == n
    assert compare_lists(gts, gids, ots, oids, orc.projection()["margin"], orc.T) == 0


def test_equal_depths_keep_id_order():
    """Gaussians at exactly the same depth (identical FP64 depths): the lists
    order them by ascending id (the stable view sort keeps id order and the
    tie pass leaves such runs alone)."""
    rng = np.random.default_rng(11)
    n, f = 300, 120.0
    u, v = rng.uniform(35.0, 45.0, n), rng.uniform(35.0, 45.0, n)
    zc = np.where(np.arange(n) % 3 == 0, 2.5, 3.25)  # two depth classes, each shared by many Gaussians
    mu = np.stack([(u - 32.0) * zc / f, (v - 32.0) * zc / f, zc - 3.0], 1)
    n, beta = one_gaussian_scene(mu, [math.log(0.004)] * 3, [1, 0, 0, 0], -1.0, [0.3, 0.6, 0.9])
    fr, orc = check_all("equal depths", n, 0, beta, axis_camera(f, 64, 64), 64, 64)
    rec = np_(fr.rec)[0]
    vis = np_(fr.rect)[0][:, 0] < np_(fr.rect)[0][:, 2]
    z = ((rec[vis, 11].view(np.uint32).astype(np.uint64) << np.uint64(32)) |
         rec[vis, 9].view(np.uint32).astype(np.uint64)).view(np.float64)
    assert len(np.unique(z)) == 2


@pytest.mark.parametrize("k", [13, 16, 24, 27, 32, 40, 64])
def test_multi_wave_paths(k):
    """Samples per tile at which the derivative walks run several waves per
    tile: 13 and 16 (2 waves, 7 and 8 pixels each) and 24, 27 and 32 (4
    waves, 6 to 8 pixels each), pixels dealt to the waves by depth with
    per-lane colour-tangent accumulators; 40 and 64 (4 waves, pixels beyond
    32 per tile: dealt by slot, one wave sum per step). Against the oracle
    (GN product in check_all, J p, J^T u and the diagonal here)."""
    n, deg = 3000, 2
    gt = synth.make_scene(n, deg, 12, means="ball")
    beta = synth.perturb_init(gt, n, deg, 12)
    cams = synth.sphere_cameras(2, 4.0, 128, 96, 60.0, 12)
    pix, wts = sample_uniform(13, 0, np.arange(2), (128 // 16) * (96 // 16), k)
    fr, orc = check_all(f"k={k}", n, deg, beta, cams, 128, 96, k, pix, wts)
    p = np.random.default_rng(1).normal(size=orc.P).astype(np.float32)
    jp = np_(lib().lmrs_jvp(fr, torch.tensor(p, device=DEV)))
    ok = orc.decided()
    e = rel(jp[ok], orc.jvp(p)[ok])
    log(f"  k={k} jvp rel {e:.2e} on decided pixels")
    assert e < 1e-4
    u = np.random.default_rng(2).normal(size=(orc.S, 3)).astype(np.float32)
    e = rel(np_(lib().lmrs_vjp(fr, torch.tensor(u, device=DEV))), orc.vjp(u))
    log(f"  k={k} vjp rel {e:.2e}")
    assert e < 1e-4
    d = np_(lib().lmrs_gn_diag(fr))
    e = rel(d, orc.diag())
    log(f"  k={k} diag rel {e:.2e}")
    assert e < 1e-4


def test_maximum_tiles_per_view():
    """A 2048x2048 view has 16,384 tiles, the most one view may have (the
    binning histogram of a view lives in LDS); one sample per tile."""
    w = synth.config0()
    W = 2048
    cams = synth.sphere_cameras(1, 3.0, W, W, 60.0, 5)
    pix, wts = sample_uniform(6, 0, np.arange(1), (W // 16) ** 2, 1)
    check_all("2048x2048", w.n, 0, w.beta_init, cams, W, W, 1, pix, wts)
