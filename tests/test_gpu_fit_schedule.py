"""The LM driver's schedules (Sec. 5) and camera-clustering view batches
(Sec. 4.3) on the GPU: batch 4 -> 8 views and CG 3 -> 6 steps from iteration 3
on, on 12 cameras of the 1k-Gaussian scene, every pixel. Checked: each
iteration's views are one camera per K-means cluster of the scheduled batch
size, the reported CG steps follow the schedule, the full loss decreases, and
a scheduled step matches the oracle's LM step from the same parameters."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, log, np_, oracle_for, rel
from oracle.solver import full_loss
from oracle.solver import lm_step as oracle_lm_step
from oracle.views import camera_features, kmeans
from paper_2504_12905_amd import fit, synth

pytestmark = pytest.mark.gpu


def test_schedule_and_cluster_views():
    w = synth.config0()
    cams = synth.sphere_cameras(12, 3.0, w.width, w.height, 60.0, 5)
    tg_np = oracle_for(w.n, 0, w.beta_gt, cams, w.width, w.height).render_image().astype(np.float32)
    tg = torch.tensor(tg_np, device=DEV)
    beta = torch.tensor(w.beta_init, device=DEV)
    sch = fit.Schedule(batch=4, batch_late=8, cg_iters=3, cg_iters_late=6, late_iter=3)
    f = fit.Fitter(w.n, 0, beta, cams, tg, w.width, w.height, sch, lam=w.lam, seed=2)
    loss0 = full_loss(w.n, 0, w.beta_init, cams, tg_np, w.width, w.height)
    hist = f.run(3)
    # the first late iteration, checked against the oracle from the same parameters
    b_before = np_(beta).copy()
    ids = f.step(3)
    rep = f.report.cpu().numpy()
    b_ref, info = oracle_lm_step(w.n, 0, b_before, cams, tg_np, ids, w.width, w.height, 256, 2, 3, w.lam, 6)
    d_gpu = np_(beta).astype(np.float64) - b_before
    d_ref = b_ref.astype(np.float64) - b_before
    log(f"  late step: views {ids.tolist()}, cg {int(rep[3])}/{info['cg_done']}, step rel {rel(d_gpu, d_ref):.2e}")
    assert len(ids) == 8 and int(rep[3]) == info["cg_done"] == 6
    assert rel(d_gpu, d_ref) < 1e-3
    hist += f.run(2, start=4)
    for h in hist:
        B = 4 if h["iter"] < 3 else 8
        labels, _ = kmeans(camera_features(cams), B, 2)
        assert len(h["views"]) == B and sorted(labels[h["views"]].tolist()) == list(range(B))
        assert h["cg_done"] == (3 if h["iter"] < 3 else 6)
    loss1 = full_loss(w.n, 0, np_(beta), cams, tg_np, w.width, w.height)
    log(f"  full loss {loss0:.4e} -> {loss1:.4e} over 6 iterations")
    assert loss1 < loss0
