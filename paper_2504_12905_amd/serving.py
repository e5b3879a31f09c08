"""Serving loop for scene-fit requests over the C ABI (host scheduling only;
every step of every fit runs in the library's kernels).

A fit request is a synthetic scene (Gaussians, cameras, target images
rendered from its ground truth) to be fitted by `lm_iters` LM iterations of
Alg. 1 with `cg_iters` GN products each, every pixel of every view per
iteration (weights 1), damping lambda.

`Server` does continuous batching on one GPU:
* admission by HBM footprint: a request is admitted when it has arrived, a
  slot is free and its footprint (parameters, targets, screen records, tile
  lists with their sort keys, per-pixel buffers and the solver workspace; the
  list size bounded from the scene on the host) fits next to the footprints
  of the fits already resident;
* requests are admitted in arrival order without overtaking (policy "fifo",
  the default), or, with policy "sjf", the arrived request with the least
  estimated work first. With the device saturated by the large fits of a
  stream, shortest-first lets the small ones finish early instead of waiting
  behind large ones, which lowers the median latency, but starts the largest
  fits last, which lengthens the tail and the makespan;
* an admitted fit keeps its parameters, lists, CG state and targets in device
  memory until it retires, and runs on its own HIP stream (default
  priority), so the kernels of different fits overlap on the device;
* one LM iteration of a fit is one lmrs_lm_iterate call (projection, binning
  into an id buffer sized from the host bound, sampling, render, residuals,
  b, preconditioner, the PCG loop's GN products and vector recurrences,
  learning rate, update: about a hundred launches), which never waits on the
  host. It is captured once per learning-rate branch into a HIP graph and
  replayed. A fit's iterations are enqueued CHUNK_ITERS at a time; when a
  chunk has run, the host reads its failure bits. The host bound on the list
  size holds for the parameters at admission, but a fit can grow its
  Gaussians past it: an iteration whose lists overflow the id buffer leaves
  the parameters alone and flags the overflow. The server then grows the id
  buffer (and the binning workspace) to the largest count any iteration of
  the chunk asked for, restores the parameters saved at the chunk's start and
  runs the chunk again, so every iteration index runs once on complete
  lists, as in the sequential solver;
* each fit keeps a blend table (the linearization of its render, 44 bytes per
  blending (pixel, Gaussian) pair; lmrs_frame), sized at admission from the
  pair count of the target render with a 30 % margin and within what is left
  of the HBM budget (at most TABLE_CAP_BYTES): an iteration whose pairs fit
  takes its GN products from the table, one whose pairs do not walks the tile
  lists (decided on the device, so graph replays need no host check);
* a fit retires when its last iteration's event has completed: final PSNR
  over all views at full resolution, and its status: "ok", or "numeric" /
  "capacity" when any iteration flagged a numeric failure or an overflow of
  its list buffer (the failure bits of every iteration are OR-ed on the
  device). A failed fit does not disturb the others: every buffer it touches
  is its own.

`run_sequential` is the plain baseline: the same requests one at a time in
arrival order, eager lmrs_lm_step calls on one stream (which wait for each
iteration's tile-list count), no graphs, the same blend-table sizing.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import lmrs as L
from . import synth


TABLE_CAP_BYTES = 48 << 30   # largest blend table of one fit
TABLE_MARGIN = 1.3           # table pairs per pair of the target render
CHUNK_ITERS = 5              # LM iterations a served fit enqueues between host checks
MAX_REGROWTHS = 8            # list-buffer regrowths per fit before an overflow is reported


@dataclass
class FitRequest:
    seed: int
    n: int
    sh_degree: int
    n_views: int
    res: int
    lm_iters: int = 30
    cg_iters: int = 8
    lam: float = 0.1
    arrival_t: float = 0.0       # seconds after the start of the run
    id: int = 0
    deterministic: bool = False  # fixed-point accumulation: the same bits alone, in a mix and on every run

    @staticmethod
    def from_stream(d: dict) -> "FitRequest":
        return FitRequest(seed=d["seed"], n=d["n"], sh_degree=d["sh_degree"], n_views=d["n_views"], res=d["res"],
                          lm_iters=d["lm_iters"], cg_iters=d["cg_iters"], lam=d["lam"], arrival_t=d["arrival_s"],
                          id=d["id"])


@dataclass
class FitResult:
    beta: np.ndarray
    final_psnr: float
    latency_s: float
    status: str
    start_s: float = 0.0
    end_s: float = 0.0


@dataclass
class Problem:
    """Host data of one request: scene and cameras per the 1k-Gaussian
    workload's priors (means in [-1,1]^3, cameras at radius 3, FOV 60)."""
    req: FitRequest
    beta_gt: np.ndarray
    beta_init: np.ndarray
    cams: np.ndarray
    instances_bound: int
    footprint: int


def instances_bound(beta: np.ndarray, n: int, cams: np.ndarray, W: int, H: int) -> int:
    """Upper bound on the tile-list entries of a scene: per (view, Gaussian)
    the tiles of the square of half-side ceil(3 sqrt(l) ) + 1 px around the
    projected mean, l >= lambda_max of the screen covariance bounded by
    (f/z)^2 (1 + (x^2 + y^2)/z^2) s_max^2 + 0.3 (spectral norm of the
    projection Jacobian times the largest scale)."""
    mu = beta[0:3 * n].reshape(3, n).astype(np.float64)
    smax = np.exp(beta[3 * n:6 * n].reshape(3, n).max(axis=0).astype(np.float64))
    TX, TY = W // 16, H // 16
    total = 0
    for c in cams:
        R = c[0:9].reshape(3, 3).astype(np.float64)
        t = c[9:12].astype(np.float64)
        fx, fy, cx, cy = (float(x) for x in c[12:16])
        tc = R @ mu + t[:, None]
        z = tc[2]
        ok = z > 0.15
        zs = np.where(ok, z, 1.0)
        jn2 = (max(fx, fy) / zs) ** 2 * (1.0 + (tc[0] ** 2 + tc[1] ** 2) / zs ** 2)
        r = np.ceil(3.0 * np.sqrt(jn2 * smax ** 2 + 0.3)) + 1.0
        u = fx * tc[0] / zs + cx
        v = fy * tc[1] / zs + cy
        x0 = np.clip(np.floor((u - r) / 16), 0, TX)
        x1 = np.clip(np.floor((u + r) / 16) + 1, 0, TX)
        y0 = np.clip(np.floor((v - r) / 16), 0, TY)
        y1 = np.clip(np.floor((v + r) / 16) + 1, 0, TY)
        total += int(np.sum(np.where(ok, np.maximum(x1 - x0, 0) * np.maximum(y1 - y0, 0), 0)))
    return total


def _frame_struct_bytes(op: int, n: int, deg: int, V: int, W: int, H: int, k: int, capacity: int,
                        deterministic: bool = False) -> int:
    fs = L._Frame(n, deg, V, W, H, k, None, None, None, None, None, None, None, capacity, None, None, None, None,
                  None, None)
    fs.deterministic = 1 if deterministic else 0
    return int(L._lib.lmrs_workspace_bytes(op, L.C.byref(fs)))


def work_estimate(req: FitRequest) -> float:
    """Relative GPU time of a fit: every LM iteration renders and
    differentiates every pixel of every view and projects every Gaussian into
    every view (a least-squares fit of the solve times of the serving stream:
    about 0.16 us per view-pixel and 0.34 us per view-Gaussian for 30
    iterations)."""
    return req.lm_iters * req.n_views * (req.res * req.res + 2.1 * req.n)


def footprint_bytes(req: FitRequest, instances: int) -> int:
    """Device bytes a fit holds while resident (see the module docstring)."""
    n, V, W = req.n, req.n_views, req.res
    K = (req.sh_degree + 1) ** 2
    P = n * (11 + 3 * K)
    T = (W // 16) ** 2
    S = V * T * 256
    cap = int(instances * 1.05) + 1024
    frame = (V * n * (4 * L.LMRS_REC + 16) + 8 * (V * T + 1) + 4 * cap + S * (12 + 4 + 4)
             + 4 * L.sched_ints(V * T))
    ws = max(_frame_struct_bytes(L.OP_BIN, n, req.sh_degree, V, W, W, 256, cap),
             _frame_struct_bytes(L.OP_LM, n, req.sh_degree, V, W, W, 256, cap, req.deterministic))
    return 4 * P + 16 * V * 4 + 12 * V * W * W + frame + ws + 64 * 4


def make_problem(req: FitRequest) -> Problem:
    gt = synth.make_scene(req.n, req.sh_degree, req.seed, means="cube")
    init = synth.perturb_init(gt, req.n, req.sh_degree, req.seed)
    cams = synth.sphere_cameras(req.n_views, 3.0, req.res, req.res, 60.0, req.seed)
    ib = max(instances_bound(gt, req.n, cams, req.res, req.res), instances_bound(init, req.n, cams, req.res, req.res))
    return Problem(req, gt, init, cams, ib, footprint_bytes(req, ib))


def _image_index(fr: L.Frame, dev) -> torch.Tensor:
    """Flat image index (v H W + y W + x) of every all-pixel sample."""
    t = torch.arange(fr.T, device=dev)
    p = torch.arange(256, device=dev)
    y = ((t // fr.TX) * 16)[:, None] + (p // 16)[None, :]
    x = ((t % fr.TX) * 16)[:, None] + (p % 16)[None, :]
    pix = (y * fr.width + x).reshape(-1)
    v = torch.arange(fr.n_views, device=dev)[:, None] * (fr.width * fr.height)
    return (v + pix[None, :]).reshape(-1)


class _Fit:
    """Device state of one resident fit."""

    def __init__(self, prob: Problem, stream: torch.cuda.Stream, use_graphs: bool, dev, ws_op: int = L.OP_LM,
                 table_bytes_max: int = TABLE_CAP_BYTES):
        req = prob.req
        self.prob, self.req, self.stream, self.use_graphs = prob, req, stream, use_graphs
        self.it = 0
        self.dev, self.ws_op = dev, ws_op
        self.graphs: dict[bool, torch.cuda.CUDAGraph] = {}
        self.chunk_start = 0
        self.chunk_event: torch.cuda.Event | None = None
        self.regrowths = 0
        self.grown_bytes = 0          # id buffer and workspace added since admission
        with torch.cuda.stream(stream):
            self.beta = torch.tensor(prob.beta_gt, device=dev)
            self.cams = torch.tensor(prob.cams, device=dev)
            cap = int(prob.instances_bound * 1.05) + 1024
            self.fr = L.Frame(req.n, req.sh_degree, self.beta, self.cams, req.res, req.res, req.n_views, k=256,
                              capacity=cap, blend=True, deterministic=req.deterministic)
            nbytes = max(L.workspace_bytes(L.OP_BIN, self.fr), L.workspace_bytes(ws_op, self.fr))
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
            self.rep = torch.zeros(L.REPORT_FLOATS, device=dev)
            self.fail = torch.zeros(1, dtype=torch.int32, device=dev)   # failure bits of every iteration, OR-ed
            self.chunk_fail = torch.zeros(1, dtype=torch.int32, device=dev)  # ... of the current chunk
            self.need = torch.zeros(1, dtype=torch.int64, device=dev)   # largest list count of the chunk
            self.idx = _image_index(self.fr, dev)
            # targets: the ground truth rendered at every pixel
            self.targets = torch.empty((req.n_views, req.res, req.res, 3), dtype=torch.float32, device=dev)
            self._render_all(self.targets)
            # the blend table, sized from the target render's pairs
            self.table_want = min(int(self.fr.blend_pairs() * TABLE_MARGIN) + 4096,
                                  TABLE_CAP_BYTES // L.BLEND_BYTES_PER_PAIR)
            room = max(min(table_bytes_max, TABLE_CAP_BYTES), 0) // L.BLEND_BYTES_PER_PAIR
            self.fr.set_blend_capacity(min(self.table_want, room))
            self.table_bytes = self.fr.blend_capacity * L.BLEND_BYTES_PER_PAIR
            self.beta.copy_(torch.tensor(prob.beta_init, device=dev))
            self.snapshot = self.beta.clone()   # parameters at the start of the current chunk

    def _render_all(self, out: torch.Tensor):
        L.lmrs_project(self.fr, stream=self.stream)
        L.lmrs_bin_tiles(self.fr, stream=self.stream, ws=self.ws)
        L.lmrs_render(self.fr, stream=self.stream, grow_blend=False)
        out.view(-1, 3)[self.idx] = self.fr.color

    def params(self) -> L.LmParams:
        return L.lm_params(self.it, self.req.cg_iters, self.req.lam)

    def _iterate(self):
        L.lmrs_lm_iterate(self.fr, self.targets, self.params(), self.ws, report=self.rep, stream=self.stream)
        self.chunk_fail.bitwise_or_(self.rep[L.REP["status"]:L.REP["status"] + 1].to(torch.int32))
        torch.maximum(self.need, self.fr.n_instances, out=self.need)

    def step(self):
        """Enqueue one LM iteration on the fit's stream (never waits on the host)."""
        req = self.req
        with torch.cuda.stream(self.stream):
            warm = self.it < 10
            if not self.use_graphs:
                self._iterate()
            else:
                g = self.graphs.get(warm)
                if g is None:
                    g = torch.cuda.CUDAGraph()
                    with torch.cuda.graph(g, stream=self.stream):
                        self._iterate()
                    self.graphs[warm] = g
                g.replay()
            self.it += 1

    def table_short(self) -> int:
        """Bytes the blend table lacks against its wanted size (the budget was short at admission)."""
        return max(self.table_want - self.fr.blend_capacity, 0) * L.BLEND_BYTES_PER_PAIR

    def grow_table(self) -> bool:
        """The wanted blend table, before the first iteration; False (and the
        table as it was) when the device cannot hold it after all."""
        have = self.fr.blend_capacity
        try:
            with torch.cuda.stream(self.stream):
                self.fr.set_blend_capacity(self.table_want)
        except torch.OutOfMemoryError:
            torch.cuda.empty_cache()   # cached blocks of retired fits
            try:
                with torch.cuda.stream(self.stream):
                    self.fr.set_blend_capacity(self.table_want)
            except torch.OutOfMemoryError:
                with torch.cuda.stream(self.stream):
                    self.fr.set_blend_capacity(have)
                self.table_want = have
                return False
        self.table_bytes = self.fr.blend_capacity * L.BLEND_BYTES_PER_PAIR
        return True

    def _enqueue_chunk(self):
        with torch.cuda.stream(self.stream):
            self.snapshot.copy_(self.beta)
            self.chunk_fail.zero_()
            self.need.zero_()
            self.chunk_start = self.it
            end = min(self.it + CHUNK_ITERS, self.req.lm_iters)
            while self.it < end:
                self.step()
            self.chunk_event = torch.cuda.Event()
            self.chunk_event.record(self.stream)

    def _grow(self, needed: int):
        """Id buffer for `needed` list entries (with the binding's margin) and a
        workspace to match; the graphs hold the old buffers and are dropped."""
        old = 4 * self.fr.capacity + self.ws.numel()
        self.graphs.clear()
        with torch.cuda.stream(self.stream):
            self.fr.grow_ids(needed)
            nbytes = max(L.workspace_bytes(L.OP_BIN, self.fr), L.workspace_bytes(self.ws_op, self.fr))
            if nbytes > self.ws.numel():
                self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.dev)
        self.grown_bytes += 4 * self.fr.capacity + self.ws.numel() - old
        self.regrowths += 1

    def poll(self) -> bool:
        """Advance the fit without waiting: enqueue its next chunk when the last
        one has run (again, after growing the lists, if it overflowed them).
        True once every iteration has run."""
        if self.chunk_event is not None:
            if not self.chunk_event.query():
                return False
            with torch.cuda.stream(self.stream):   # the chunk has run: these reads do not wait
                bits = int(self.chunk_fail.item())
                need = int(self.need.item())
            if bits & L.FAIL_CAPACITY and self.regrowths < MAX_REGROWTHS:
                self._grow(need)
                with torch.cuda.stream(self.stream):
                    self.beta.copy_(self.snapshot)
                self.it = self.chunk_start
            else:
                with torch.cuda.stream(self.stream):
                    self.fail.bitwise_or_(self.chunk_fail)
                if self.it >= self.req.lm_iters:
                    return True
        self._enqueue_chunk()
        return False

    def status(self) -> str:
        bits = int(self.fail.item())
        if bits & L.FAIL_CAPACITY:
            return "capacity"
        return "numeric" if bits else "ok"

    def finalize(self) -> tuple[np.ndarray, float]:
        """Final PSNR over every pixel of every view, and the parameters."""
        with torch.cuda.stream(self.stream):
            img = torch.empty_like(self.targets)
            self._render_all(img)
            mse = float(((img - self.targets) ** 2).mean().item())
            beta = self.beta.cpu().numpy()
        self.graphs.clear()
        if not math.isfinite(mse):
            return beta, float("nan")
        return beta, (10.0 * math.log10(1.0 / mse) if mse > 0 else float("inf"))


@dataclass
class Server:
    hbm_budget_bytes: int
    max_slots: int = 8
    use_graphs: bool = True
    device: str = "cuda:0"
    policy: str = "fifo"           # "fifo": arrival order; "sjf": least estimated work first among the arrived
    _pending: list = field(default_factory=list)
    _results: dict = field(default_factory=dict)
    log: list = field(default_factory=list)
    table_bytes: dict = field(default_factory=dict)   # blend-table bytes of each admitted fit
    regrowths: dict = field(default_factory=dict)     # list-buffer regrowths of each retired fit
    progress: object = None        # optional callable(str), called as each fit retires

    def submit(self, req: FitRequest, problem: Problem | None = None) -> int:
        """Queue a request (host data prepared now, off the device). Returns its handle."""
        prob = problem or make_problem(req)
        if prob.footprint > self.hbm_budget_bytes:
            raise ValueError(f"request {req.id}: footprint {prob.footprint} B exceeds the budget")
        self._pending.append(prob)
        return req.id

    def _pick(self, pending: list, now: float, used: int) -> int | None:
        """Index in `pending` (sorted by arrival) of the request to admit next, or None."""
        if self.policy == "fifo":
            ok = pending and pending[0].req.arrival_t <= now and used + pending[0].footprint <= self.hbm_budget_bytes
            return 0 if ok else None
        best = None
        for i, prob in enumerate(pending):
            if prob.req.arrival_t > now:
                break
            if used + prob.footprint > self.hbm_budget_bytes:
                continue
            if best is None or work_estimate(prob.req) < work_estimate(pending[best].req):
                best = i
        return best

    def result(self, handle: int) -> FitResult:
        return self._results[handle]

    def run_until_idle(self) -> dict[int, FitResult]:
        """Serve every submitted request; arrival times are seconds after this call."""
        pending = sorted(self._pending, key=lambda p: p.req.arrival_t)
        self._pending = []
        streams = [torch.cuda.Stream(device=self.device) for _ in range(self.max_slots)]
        free_streams = list(range(self.max_slots))
        active: list[tuple[_Fit, int, float]] = []   # (fit, stream index, start time)
        used = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while pending or active:
            now = time.perf_counter() - t0
            # admission: arrived, a free slot, and room in the footprint budget
            while free_streams:
                pick = self._pick(pending, now, used)
                if pick is None:
                    break
                prob = pending.pop(pick)
                si = free_streams.pop(0)
                fit = _Fit(prob, streams[si], self.use_graphs, self.device,
                           table_bytes_max=self.hbm_budget_bytes - used - prob.footprint)
                used += prob.footprint + fit.table_bytes
                self.table_bytes[prob.req.id] = fit.table_bytes
                start = time.perf_counter() - t0
                active.append((fit, si, start))
                self.log.append(("admit", prob.req.id, start, used))
            if not active:
                if pending:
                    time.sleep(max(0.0, min(0.01, pending[0].req.arrival_t - (time.perf_counter() - t0))))
                continue
            still = []
            running = sum(1 for fit, _, _ in active if fit.chunk_event is not None)
            for fit, si, start in active:
                if fit.chunk_event is None and fit.table_short():
                    # a fit admitted while the budget was short of its blend table waits
                    # for the room (its GN products would otherwise walk the lists where
                    # alone they take the table, a different summation order), unless
                    # nothing is running to free memory
                    short = fit.table_short()
                    if used + short <= self.hbm_budget_bytes:
                        before = fit.table_bytes
                        fit.grow_table()
                        used += fit.table_bytes - before
                        self.table_bytes[fit.req.id] = fit.table_bytes
                    elif running:
                        still.append((fit, si, start))
                        continue
                if fit.chunk_event is None:
                    running += 1
                grown = fit.grown_bytes
                done = fit.poll()
                used += fit.grown_bytes - grown
                if done:
                    beta, psnr = fit.finalize()
                    end = time.perf_counter() - t0
                    req = fit.req
                    self._results[req.id] = FitResult(beta, psnr, end - req.arrival_t, fit.status(), start, end)
                    self.regrowths[req.id] = fit.regrowths
                    used -= fit.prob.footprint + fit.table_bytes + fit.grown_bytes
                    free_streams.append(si)
                    self.log.append(("retire", req.id, end, used))
                    if self.progress:
                        self.progress(f"[serve] served fit {req.id} retired at {end:.1f} s "
                                      f"({len(self._results)} done)")
                    del fit
                else:
                    still.append((fit, si, start))
            if len(still) == len(active) and not (free_streams and self._pick(pending, now, used) is not None):
                time.sleep(2e-4)   # nothing to admit or retire yet
            active = still
        return self._results


def run_sequential(problems: list[Problem], device: str = "cuda:0",
                   hbm_budget_bytes: int = 200 << 30, progress=None) -> dict[int, FitResult]:
    """Plain baseline: one request at a time in arrival order, eager
    lmrs_lm_step calls on the current stream, no graphs, no overlap."""
    out: dict[int, FitResult] = {}
    order = sorted(problems, key=lambda p: p.req.arrival_t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stream = torch.cuda.current_stream()
    for prob in order:
        req = prob.req
        now = time.perf_counter() - t0
        if req.arrival_t > now:
            time.sleep(req.arrival_t - now)
        start = time.perf_counter() - t0
        fit = _Fit(prob, stream, False, device, ws_op=L.OP_LM, table_bytes_max=hbm_budget_bytes - prob.footprint)
        for it in range(req.lm_iters):
            L.lmrs_lm_step(fit.fr, fit.targets, L.lm_params(it, req.cg_iters, req.lam), report=fit.rep, grow_blend=False,
                           ws=fit.ws, stream=stream)
            fit.fail.bitwise_or_(fit.rep[L.REP["status"]:L.REP["status"] + 1].to(torch.int32))
        beta, psnr = fit.finalize()
        end = time.perf_counter() - t0
        out[req.id] = FitResult(beta, psnr, end - req.arrival_t, fit.status(), start, end)
        if progress:
            progress(f"[serve] sequential fit {req.id} done at {end:.1f} s ({len(out)} done)")
        del fit
    return out


def summarize(results: dict[int, FitResult], problems: list[Problem]) -> dict:
    arr = {p.req.id: p.req.arrival_t for p in problems}
    lat = np.array([r.latency_s for r in results.values()])
    first = min(arr.values())
    last = max(r.end_s for r in results.values())
    return {"fits": len(results), "fits_per_s": len(results) / (last - first),
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "makespan_s": last - first}
