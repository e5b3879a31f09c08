"""GPU: the tile schedule that lmrs_render writes into lmrs_frame.sched.

The schedule is bookkeeping, not arithmetic of the method, so it is checked
against its definition on the host, bit-exact: the walk length of a tile is the
sum over its sampled pixels of the 64-entry chunks up to the pixel's last
blended entry (computed here from the `last` the render wrote), the order is a
permutation of the tiles by non-increasing walk length (bins of 16 above 512),
and the persistent splat launches leave the work counters as they found them
(ticket 0, finished 0, busy = tiles with a non-empty walk).
"""
import numpy as np
import pytest
import torch

from gpu_util import gpu_frame, lib, log, np_
from oracle.sampling import sample_uniform
from paper_2504_12905_amd import synth

pytestmark = pytest.mark.gpu


def walk_lengths(last: np.ndarray) -> np.ndarray:
    last = last.astype(np.int64)
    return np.where(last >= 0, last // 64 + 1, 0).sum(axis=1)


def bin_key(length: np.ndarray) -> np.ndarray:
    return np.where(length < 512, length, np.minimum(1023, 512 + (length - 512) // 16))


def check_schedule(fr, where):
    torch.cuda.synchronize()
    VT = fr.n_views * fr.T
    sched = np_(fr.sched).astype(np.int64)
    assert sched.shape == (2 * VT + 4,)
    order, length, ctr = sched[:VT], sched[VT:2 * VT], sched[2 * VT:]
    expect = walk_lengths(np_(fr.last).reshape(VT, fr.k))
    busy = int((expect > 0).sum())
    log(f"  [{where}] tiles {VT}, busy {busy}, longest walk {expect.max()}, counters {ctr.tolist()}")
    assert np.array_equal(length, expect), "walk lengths"
    assert np.array_equal(np.sort(order), np.arange(VT)), "order is not a permutation of the tiles"
    assert np.all(np.diff(bin_key(length[order])) <= 0), "order not by decreasing walk length"
    assert ctr.tolist() == [0, 0, busy, 0], "work counters"


@pytest.mark.parametrize("name", ["cfg0-all-pixels", "medium-k26"])
def test_schedule_after_render_and_each_walk(name):
    L = lib()
    if name == "cfg0-all-pixels":
        w = synth.config0()
        fr = gpu_frame(w.n, 0, w.beta_init, w.cams, w.width, w.height)
    else:
        n, deg = 20000, 3
        gt = synth.make_scene(n, deg, 5, means="ball")
        beta = synth.perturb_init(gt, n, deg, 5)
        cams = synth.sphere_cameras(3, 4.0, 256, 256, 60.0, 5)
        pix, wts = sample_uniform(11, 0, np.arange(3), 256, 26)
        fr = gpu_frame(n, deg, beta, cams, 256, 256, 26, pix, wts)
    check_schedule(fr, "render")
    p = torch.randn(fr.P, generator=torch.Generator().manual_seed(1)).to(fr.beta.device)
    jp = L.lmrs_jvp(fr, p)
    check_schedule(fr, "jvp")
    L.lmrs_vjp(fr, jp)
    check_schedule(fr, "vjp")
    L.lmrs_gn_product(fr, p, 0.1)
    check_schedule(fr, "gn")
    L.lmrs_gn_diag(fr)
    check_schedule(fr, "diag")


def test_schedule_empty_frame():
    """No Gaussian in front of the camera: every walk is empty, nothing is busy,
    and the derivative calls still return zeros with the counters intact."""
    L = lib()
    w = synth.config0()
    cams = w.cams.copy()
    cams[:, 9:12] = 0.0
    cams[:, 11] = -10.0  # every Gaussian behind the camera
    fr = gpu_frame(w.n, 0, w.beta_init, cams, w.width, w.height)
    check_schedule(fr, "render")
    p = torch.ones(fr.P, device=fr.beta.device)
    assert float(L.lmrs_jvp(fr, p).abs().max()) == 0.0
    assert float(L.lmrs_gn_product(fr, p, 0.0).abs().max()) == 0.0
    check_schedule(fr, "gn")
