"""A whole LM fit of the 1k-Gaussian workload (4 views 64x64, all pixels,
lambda 1e-3, 20 LM iterations x 10 CG steps) on the GPU, beside the FP64
oracle running the same 20 iterations from the same start.

Each run follows its own trajectory (FP32 and FP64 steps differ in the last
bits and LM iterations amplify that), so the runs are compared by what they
achieve: the full-objective loss after every iteration (within 1 %) and
the final PSNR (within 0.1 dB). Per-iteration parity from identical
parameters is checked in test_gpu_parity.test_lm_step_cfg0."""
import math

import numpy as np
import pytest
import torch

from gpu_util import DEV, lib, log, np_, oracle_for
from oracle.solver import full_loss
from oracle.solver import lm_step as oracle_lm_step
from paper_2504_12905_amd import synth

pytestmark = pytest.mark.gpu


def test_lm_run_cfg0_loss_curve_and_psnr():
    w = synth.config0()
    L = lib()
    tg = oracle_for(w.n, 0, w.beta_gt, w.cams, w.width, w.height).render_image().astype(np.float32)
    tg_dev = torch.tensor(tg, device=DEV)
    fr = L.Frame(w.n, 0, torch.tensor(w.beta_init, device=DEV), torch.tensor(w.cams, device=DEV), w.width,
                 w.height, 4, view_ids=torch.arange(4, dtype=torch.int32, device=DEV), k=256)
    b_ref = w.beta_init.copy()
    M = tg.size
    l0 = full_loss(w.n, 0, w.beta_init, w.cams, tg, w.width, w.height)
    curve_gpu, curve_ref = [l0], [l0]
    for it in range(w.lm_iters):
        L.lmrs_lm_step(fr, tg_dev, L.lm_params(it, w.cg_iters, w.lam, seed=0))
        b_ref, _ = oracle_lm_step(w.n, 0, b_ref, w.cams, tg, np.arange(4), w.width, w.height, 256, 0, it, w.lam,
                                  w.cg_iters)
        curve_gpu.append(full_loss(w.n, 0, np_(fr.beta), w.cams, tg, w.width, w.height))
        curve_ref.append(full_loss(w.n, 0, b_ref, w.cams, tg, w.width, w.height))
    psnr = [10 * math.log10(M / c[-1]) for c in (curve_gpu, curve_ref)]
    log("  it   loss GPU       loss oracle    rel diff")
    for i, (a, b) in enumerate(zip(curve_gpu, curve_ref)):
        log(f"  {i:2d}  {a:.6e}  {b:.6e}  {abs(a - b) / b:.2e}")
    log(f"  final PSNR GPU {psnr[0]:.4f} dB, oracle {psnr[1]:.4f} dB")
    assert all(abs(a - b) <= 0.01 * b for a, b in zip(curve_gpu, curve_ref))
    assert abs(psnr[0] - psnr[1]) <= 0.1
    assert curve_gpu[-1] < 0.5 * curve_gpu[0]
