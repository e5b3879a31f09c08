"""LM fitting driver over the C ABI (Alg. 1 iterated; host choices only).

Each LM iteration picks the iteration's view batch on the host, then runs one
lmrs_lm_step on the device (projection, binning, sampling, render, residuals,
b, preconditioner, PCG, learning rate and update all in the library's
kernels). The host side holds the two choices the paper makes around the step:

* the view batch (Sec. 4.3): "kmeans" clusters the cameras into as many
  clusters as the batch size and draws one camera from each
  (lmrs_view_clusters / lmrs_view_batch, native host code of the library);
  "uniform" draws the batch without replacement from a seeded generator;
* the schedules of Sec. 5: the batch size rises from `batch` to `batch_late`
  and the CG steps from `cg_iters` to `cg_iters_late` at iteration
  `late_iter` (the paper: 16 -> 32 views and 5 -> 8 CG steps after the 50th
  iteration for real scenes; 8 views and 3 -> 8 CG steps for synthetic ones).
  The CG schedule travels in lmrs_lm_params; a batch-size change switches to a
  frame allocated for the larger batch (the parameters are shared).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import lmrs as L


@dataclass
class Schedule:
    batch: int = 8
    batch_late: int = 0          # 0: keep `batch`
    cg_iters: int = 8
    cg_iters_late: int = 0       # 0: keep `cg_iters`
    late_iter: int = 50          # first iteration of the late values

    def batch_at(self, it: int) -> int:
        return self.batch_late if (self.batch_late > 0 and it >= self.late_iter) else self.batch

    def cg_at(self, it: int) -> int:
        return self.cg_iters_late if (self.cg_iters_late > 0 and it >= self.late_iter) else self.cg_iters


class Fitter:
    """Fits the parameters `beta` (device float32 [P], updated in place) to the
    targets (device float32 [n_cams, H, W, 3]) of the cameras (host float32
    [n_cams, 16])."""

    def __init__(self, n: int, sh_degree: int, beta: torch.Tensor, cams: np.ndarray, targets: torch.Tensor,
                 width: int, height: int, schedule: Schedule, lam: float = 0.1, k: int = 256,
                 sampler: int = L.SAMPLER_UNIFORM, view_sampler: str = "kmeans", seed: int = 0):
        assert view_sampler in ("kmeans", "uniform")
        self.n, self.sh_degree, self.beta = n, sh_degree, beta
        self.cams_host = np.ascontiguousarray(cams, dtype=np.float32)
        self.cams = torch.tensor(self.cams_host, device=beta.device)
        self.targets, self.width, self.height = targets, width, height
        self.schedule, self.lam, self.k, self.sampler = schedule, lam, k, sampler
        self.view_sampler, self.seed = view_sampler, seed
        self._rng = np.random.default_rng(seed)
        self._frames: dict[int, L.Frame] = {}
        self._labels: dict[int, np.ndarray] = {}
        self.report = torch.zeros(L.REPORT_FLOATS, device=beta.device)
        self.history: list[dict] = []

    def _frame(self, B: int) -> L.Frame:
        fr = self._frames.get(B)
        if fr is None:
            ids = torch.zeros(B, dtype=torch.int32, device=self.beta.device)
            fr = L.Frame(self.n, self.sh_degree, self.beta, self.cams, self.width, self.height, B, view_ids=ids,
                         k=self.k, sampled=self.k < 256 or self.sampler != L.SAMPLER_UNIFORM)
            self._frames[B] = fr
        return fr

    def views(self, it: int) -> np.ndarray:
        """The view batch of LM iteration `it` (camera indices)."""
        B = self.schedule.batch_at(it)
        n_cams = self.cams_host.shape[0]
        if self.view_sampler == "uniform":
            return self._rng.choice(n_cams, B, replace=False).astype(np.int32)
        labels = self._labels.get(B)
        if labels is None:
            labels = L.view_clusters(self.cams_host, B, self.seed)
            self._labels[B] = labels
        return L.view_batch(labels, B, self.seed, it)

    def step(self, it: int, stream=None) -> np.ndarray:
        ids = self.views(it)
        fr = self._frame(len(ids))
        fr.view_ids.copy_(torch.from_numpy(ids))
        s = self.schedule
        prm = L.lm_params(it, s.cg_iters, self.lam, seed=self.seed, sampler=self.sampler,
                          cg_iters_late=s.cg_iters_late, late_iter=s.late_iter if s.cg_iters_late else 0)
        L.lmrs_lm_step(fr, self.targets, prm, report=self.report, stream=stream)
        return ids

    def run(self, iters: int, start: int = 0, check: bool = True) -> list[dict]:
        """`iters` LM iterations from `start`; keeps one report per iteration
        and raises LmrsError(LMRS_ENUMERIC) on a numeric failure when check."""
        for it in range(start, start + iters):
            ids = self.step(it)
            rep = self.report.cpu()
            if check:
                L.check_report(rep, f"LM iteration {it}")
            self.history.append({"iter": it, "views": ids.tolist(), "loss": float(rep[L.REP["loss"]]),
                                 "eta": float(rep[L.REP["eta"]]), "cg_done": int(rep[L.REP["cg_done"]])})
        return self.history
