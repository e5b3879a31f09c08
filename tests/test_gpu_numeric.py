"""Numeric failures surface as a status (LMRS_ENUMERIC through the report's
LMRS_REP_STATUS word) instead of corrupting the parameters: NaN in a visible
Gaussian's colour, or in the target image, makes b = J^T W r non-finite; the
LM step then records LMRS_FAIL_NONFINITE, leaves beta bit-for-bit as it was,
and lmrs_report_status turns the report into LMRS_ENUMERIC. A clean step
reports 0. The NaNs are data, not faults: every kernel runs to its end."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, lib, log, np_
from paper_2504_12905_amd import synth

pytestmark = pytest.mark.gpu


def frame_and_targets(beta):
    w = synth.config0()
    L = lib()
    fr = L.Frame(w.n, 0, torch.tensor(beta, device=DEV), torch.tensor(w.cams, device=DEV), w.width, w.height, 4,
                 view_ids=torch.arange(4, dtype=torch.int32, device=DEV))
    gt = L.Frame(w.n, 0, torch.tensor(w.beta_gt, device=DEV), torch.tensor(w.cams, device=DEV), w.width, w.height, 4)
    L.lmrs_project(gt)
    L.lmrs_bin_tiles(gt)
    L.lmrs_render(gt)
    tg = torch.empty((4, w.height, w.width, 3), device=DEV)
    TX = w.width // 16
    t = torch.arange(gt.T, device=DEV)
    p = torch.arange(256, device=DEV)
    y = ((t // TX) * 16)[:, None] + (p // 16)[None, :]
    x = ((t % TX) * 16)[:, None] + (p % 16)[None, :]
    col = gt.color.view(4, gt.T, 256, 3)
    for v in range(4):
        tg[v, y, x] = col[v]
    return w, fr, tg


def visible_gaussian(w):
    from oracle import Oracle
    vis = Oracle(w.n, 0, w.beta_init, w.cams, w.width, w.height).projection()["visible"]
    return int(np.flatnonzero(vis.all(axis=0))[0])


def run_step(fr, tg, w, it=0):
    L = lib()
    rep = torch.zeros(L.REPORT_FLOATS, device=DEV)
    L.lmrs_lm_step(fr, tg, L.lm_params(it, 10, w.lam), report=rep)
    torch.cuda.synchronize()
    return rep


def test_clean_step_reports_no_failure():
    w = synth.config0()
    w, fr, tg = frame_and_targets(w.beta_init)
    rep = run_step(fr, tg, w)
    L = lib()
    assert float(rep[L.REP["status"]]) == 0.0
    L.check_report(rep)  # does not raise


@pytest.mark.parametrize("where", ["colour", "target"])
def test_nan_input_sets_status_and_keeps_beta(where):
    L = lib()
    w = synth.config0()
    beta = w.beta_init.astype(np.float32).copy()
    if where == "colour":
        g = visible_gaussian(w)
        beta[synth.seg(w.n, "sh", 0).start + g] = np.nan   # DC red coefficient of a Gaussian every view sees
    w, fr, tg = frame_and_targets(beta)
    if where == "target":
        tg[1, 30, 30, 2] = float("nan")
    before = np_(fr.beta).copy()
    log(f"[numeric] NaN in the {where}")
    rep = run_step(fr, tg, w)
    st = int(float(rep[L.REP["status"]]))
    log(f"  status bits {st}, loss {float(rep[0])}")
    assert st & L.FAIL_NONFINITE
    after = np_(fr.beta)
    assert np.array_equal(before.view(np.uint32), after.view(np.uint32))  # unchanged, NaN included
    with pytest.raises(L.LmrsError) as e:
        L.check_report(rep)
    assert e.value.status == L.LMRS_ENUMERIC
