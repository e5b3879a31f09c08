#!/usr/bin/env python3
"""Benchmark: Gauss-Newton products per second inside LM steps on one MI355X.

Workload (object-scale fit, FP32): 100k Gaussians in the unit ball, SH degree 3,
64 cameras of 800x800 on a radius-4 sphere. Each LM step samples 8 views and
10 % of the pixels of every 16x16 tile (26 per tile, uniform, Philox keys),
runs 8 CG iterations (8 GN products) and updates the parameters. A timed
"step" is one full LM step through the C ABI: projection, binning, sampling,
render, residuals, b = J^T W r, diagonal, PCG with 8 GN products, learning
rate and update. `value` = GN products completed per second of LM stepping
(8 per step), with all inputs resident in HBM.

Also measured: the GN product on its own (HIP events on the library's stream,
per launch), the roofline position of its dominant kernel (the fused splat
kernel), the unfused J p -> J^T u comparator, and the FP64 CPU oracle timed on
the same GN product (its result also gives the parity of the timed product).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GN products (J^T J p)/sec at 100k Gaussians vs plain; served fits/sec + p99"
# Published MI355X peaks: HBM3E 8 TB/s; FP32 vector 157.3 TFLOP/s.
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
# For reference only: the FP32 vector rate without packed FP32 instructions
# (256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz); the library is built
# with packed FP32 arithmetic switched off.
FP32_UNPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
SPLAT_SOURCE = os.path.join(ROOT, "paper_2504_12905_amd", "csrc", "kernels_splat.hip")
# the GN product's splat kernels: over the blend table (when built) and the
# fused list walk; name match in profiler output, summary files
SPLAT_KERNELS = {
    # the float-atomic instantiation (the deterministic one, blend_gn_kernel<true>, is timed on the side)
    "table": ("blend_gn_kernel<false>", "blend_gn_kernel<false> (GN product over the blend table)",
              os.path.join(ROOT, "profiles", "gn_blend_traffic_cfg1.txt"),
              os.path.join(ROOT, "profiles", "gn_blend_counters_cfg1.txt")),
    "walk": ("deriv_kernel<3", "deriv_kernel<3> (fused list walk of the GN product)",
             os.path.join(ROOT, "profiles", "gn_splat_traffic_cfg1.txt"),
             os.path.join(ROOT, "profiles", "gn_splat_counters_cfg1.txt")),
}

# Algorithmic work of one GN product, per unit the method must touch:
#   per traversed list entry (the prefix L*_t of each tile's list up to the
#   deepest last blended entry of its sampled pixels): id 4 B + screen record
#   36 B + its tangent 36 B read = 76 B;
#   per contributing entry (blended by at least one sampled pixel of the
#   tile): 36 B of screen-gradient partials written;
#   per sampled pixel: pixel index, weight, final transmittance, last = 16 B;
#   per blending (pixel, entry) pair: 100 FP32 operations (primal recompute,
#   tangent, reverse), per walked pair that does not blend: 10 (the opacity
#   test);
#   around the splat: p, the parameters and the output once each (4 P x 3 B),
#   and per visible (view, Gaussian) the tangent record and the screen
#   gradient written and read (4 x 36 B) and ~600 FP32 operations of the
#   tangent and reverse projection.
B_ENTRY, B_CONTRIB, B_PIXEL = 76, 36, 16
F_ACT, F_SKIP = 100, 10
B_VIS, F_VIS = 4 * 36, 600


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def render_targets(L, torch, w, beta_gt, cams, dev):
    """Render every camera of the workload at full resolution (setup, untimed)."""
    V_all = cams.shape[0]
    H, W = w.height, w.width
    targets = torch.empty((V_all, H, W, 3), dtype=torch.float32, device=dev)
    TX = W // 16
    for a in range(0, V_all, 8):
        ids = torch.arange(a, min(a + 8, V_all), dtype=torch.int32, device=dev)
        fr = L.Frame(w.n, w.sh_degree, beta_gt, cams, W, H, ids.numel(), view_ids=ids, k=256)
        L.lmrs_project(fr)
        L.lmrs_bin_tiles(fr)
        L.lmrs_render(fr)
        T = fr.T
        col = fr.color.view(ids.numel(), T, 256, 3)
        t = torch.arange(T, device=dev)
        p = torch.arange(256, device=dev)
        y = ((t // TX) * 16)[:, None] + (p // 16)[None, :]
        x = ((t % TX) * 16)[:, None] + (p % 16)[None, :]
        for v in range(ids.numel()):
            targets[a + v, y, x] = col[v]
    torch.cuda.synchronize()
    return targets


def traffic_from_profile(kernel_hash: str, default_workload: bool, which: str = "table"):
    """HBM bytes per launch of a splat kernel ("table" or "walk") from the
    committed rocprofv3 counter summary, if it was taken on the current kernel
    source and on the workload being timed (the summary covers the default
    100k one)."""
    path = SPLAT_KERNELS[which][2]
    if not default_workload or not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_hash:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _one_core_seconds(w, beta, cams_np, views, pix, wts, lam, pd, threads_after):
    """Median of 3 oracle GN products on one thread over `views` (after a first call)."""
    from oracle import Oracle, set_num_threads
    set_num_threads(1)
    try:
        nv = len(views)
        o1 = Oracle(w.n, w.sh_degree, beta, cams_np[views], w.width, w.height)
        o1.set_samples(pix.shape[-1], pix[:nv], wts[:nv])
        o1.gn(pd, lam)
        times = []
        for _ in range(3):
            t0 = time.perf_counter()
            o1.gn(pd, lam)
            times.append(time.perf_counter() - t0)
        return times
    finally:
        set_num_threads(threads_after)


def cpu_baseline(w, beta, cams_np, view_ids, pix, wts, lam, p, budget_s=20.0, n_views=None, one_core_views=1):
    """FP64 oracle GN products/s on the same product the GPU timed: the batch
    views (or the first n_views of them, the time then scaled to the whole
    batch), the same samples, parameters and direction p. The first call also
    builds the record Jacobians the later calls reuse (reported apart); then
    products are repeated until about `budget_s` seconds of CPU work. Then the
    same on one thread, restricted to the first `one_core_views` views (time
    scaled to the batch), median of 3 after the first call."""
    from oracle import Oracle, num_threads
    V = len(view_ids)
    nv = V if n_views is None else n_views
    orc = Oracle(w.n, w.sh_degree, beta, cams_np[view_ids[:nv]], w.width, w.height)
    orc.set_samples(pix.shape[-1], pix[:nv], wts[:nv])
    pd = p.astype(np.float64)
    threads = num_threads()
    t0 = time.perf_counter()
    ref = orc.gn(pd, lam)
    first = time.perf_counter() - t0
    times = []
    while (not times or sum(times) + first < budget_s) and len(times) < 500:
        t0 = time.perf_counter()
        orc.gn(pd, lam)
        times.append(time.perf_counter() - t0)
    t1 = float(np.median(times)) * V / nv
    del orc
    t_one = _one_core_seconds(w, beta, cams_np, view_ids[:one_core_views], pix, wts, lam, pd, threads) \
        if one_core_views else None
    part = (f"the full GN product of one LM step ({V} views" if nv == V else
            f"the GN product restricted to {nv} of the {V} batch views, time scaled by {V}/{nv} ({nv} views")
    return {"value": round(1.0 / t1, 4), "unit": "GN products/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{part}, {pix.shape[-1]} samples/tile, same parameters and p as the GPU's timed "
                      f"product); median of {len(times)} products after a first call of {first:.1f} s that "
                      f"also builds the record Jacobians",
            "seconds_per_product": round(t1, 4),
            "one_core": None if t_one is None else {
                "value": round(1.0 / (float(np.median(t_one)) * V / one_core_views), 5), "unit": "GN products/s",
                "cores": 1,
                "sample": f"the product restricted to {one_core_views} of the {V} batch views on one thread, "
                          f"median of 3 after a first call, time scaled by {V}/{one_core_views}",
                "seconds_per_product": round(float(np.median(t_one)) * V / one_core_views, 3)}}, \
        (ref if nv == V else None)


def copy_calibration(torch, dev, mib=1024, reps=3):
    """Plain device copies of a known size (the HBM-counter calibration
    kernel of the traffic pass): reads and writes mib MiB each."""
    n = mib * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def _working(rows):
    """Counter values of the dispatches that did the splat's work: each splat
    kernel is launched for every GN product and returns at once when the other
    path is selected, so dispatches shorter than a quarter of the longest one
    are left out. rows: (value, duration) pairs."""
    if not rows:
        return []
    longest = max(d for _, d in rows)
    return [v for v, d in rows if d >= 0.25 * longest]


def _counter_rows(d: str):
    """{(kernel name, counter): [(value, duration ns)]} from a --pmc output folder."""
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    out: dict = {}
    for f in files:
        for row in csv.DictReader(open(f)):
            dur = float(row.get("End_Timestamp") or 0) - float(row.get("Start_Timestamp") or 0)
            out.setdefault((row["Kernel_Name"], row["Counter_Name"]), []).append((float(row["Counter_Value"]), dur))
    return out


def summarize_traffic(fetch_dir: str, write_dir: str, copy_mib: int, command: str, copy_reps: int = 3) -> str:
    """Per-launch HBM bytes of the GN product's splat kernels (over the blend
    table and the fused list walk, each where the run launched it) from two
    rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch), each
    scaled by the ratio of the known copy size to what the same counter reads
    for the plain copy kernel of the same run. Writes one summary file per
    kernel found and returns their text."""
    runs = {c: _counter_rows(d) for c, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir))}
    copy = {}
    for counter, rows in runs.items():
        # the calibration copies are the largest dispatches of the runtime's
        # device-to-device copy kernel in the run (reps of the same size)
        c = sorted(v for (k, cn), xs in rows.items() if cn == counter and "copyBuffer" in k
                   for v, _ in xs)[-copy_reps:]
        if not c:
            raise SystemExit(f"{counter}: no copy kernel; kernels found: {sorted({k for k, _ in rows})[:20]}")
        copy[counter] = float(np.median(c))
    kernel_hash = hashlib.sha256(open(SPLAT_SOURCE, "rb").read()).hexdigest()
    texts = []
    for which, (match, title, path, _) in SPLAT_KERNELS.items():
        out, used = {}, 0
        for counter, rows in runs.items():
            xs = _working([r for (k, cn), v in rows.items() if cn == counter and match in k for r in v])
            if xs:
                out[counter] = (float(np.median(xs)), copy[counter], copy_mib * 1024.0 / copy[counter])
                used = len(xs)
        if len(out) < 2:
            continue
        fetch = out["FETCH_SIZE"][0] * out["FETCH_SIZE"][2] * 1024
        write = out["WRITE_SIZE"][0] * out["WRITE_SIZE"][2] * 1024
        text = (f"# HBM traffic of {title}, one launch per GN product,\n"
                f"# 100k-Gaussian object-scale workload (8 views 800x800, 26 samples/tile).\n"
                f"# Commands (one counter per run, from the repository root):\n"
                f"#   {command}\n"
                f"# Counter values are KiB per dispatch (median over the {used} launches of the run that did\n"
                f"# the work; launches that found the other splat path selected return at once);\n"
                f"# each is scaled by (known copy size / the same counter for a {copy_mib} MiB device copy).\n"
                f"fetch_kib_splat: {out['FETCH_SIZE'][0]:.1f}\n"
                f"fetch_kib_copy_{copy_mib}MiB: {out['FETCH_SIZE'][1]:.1f}\n"
                f"fetch_scale: {out['FETCH_SIZE'][2]:.4f}\n"
                f"write_kib_splat: {out['WRITE_SIZE'][0]:.1f}\n"
                f"write_kib_copy_{copy_mib}MiB: {out['WRITE_SIZE'][1]:.1f}\n"
                f"write_scale: {out['WRITE_SIZE'][2]:.4f}\n"
                f"hbm_bytes_per_launch: {fetch + write:.0f}\n"
                f"kernel_source_sha256: {kernel_hash}\n")
        with open(path, "w") as f:
            f.write(text)
        texts.append(text)
    if not texts:
        raise SystemExit("no splat kernel dispatches in both counter runs")
    return "\n".join(texts)


def lm_breakdown(L, torch, fr, targets, w, sampler, it, gn_ms):
    """Wall milliseconds of each stage of one LM step, each run on its own
    through the C ABI at the current parameters (synchronised before and
    after, so launch overheads are included); the PCG vector work is the PCG
    call minus its diagonal and GN products."""
    dev = fr.beta.device

    def wall(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3

    out = {"project": wall(lambda: L.lmrs_project(fr)), "bin": wall(lambda: L.lmrs_bin_tiles(fr))}
    if sampler == L.SAMPLER_RESIDUAL:
        scores = torch.empty((fr.n_views, fr.T, 256), dtype=torch.float32, device=dev)
        out["full render (residual scores)"] = wall(lambda: L.lmrs_residual_scores(fr, targets, out=scores))
        out["sample"] = wall(lambda: L.lmrs_sample(fr, sampler, w.seed, it, scores))
    else:
        out["sample"] = wall(lambda: L.lmrs_sample(fr, sampler, w.seed, it))
    out["render"] = wall(lambda: L.lmrs_render(fr))
    u = torch.randn((fr.S, 3), generator=torch.Generator(device="cpu").manual_seed(1)).to(dev)
    b = torch.empty(fr.P, dtype=torch.float32, device=dev)
    L.lmrs_vjp(fr, u, out=b)
    out["b = J^T W r"] = wall(lambda: L.lmrs_vjp(fr, u, out=b))
    dg = torch.empty_like(b)
    L.lmrs_gn_diag(fr, out=dg)
    out["diag (+ blend table)"] = wall(lambda: L.lmrs_gn_diag(fr, out=dg))
    out[f"{w.cg_iters} GN products"] = w.cg_iters * gn_ms
    x = torch.empty_like(b)
    L.lmrs_pcg(fr, b, w.lam, w.cg_iters, x=x)
    pcg = wall(lambda: L.lmrs_pcg(fr, b, w.lam, w.cg_iters, x=x))
    out["PCG vector work"] = max(0.0, pcg - out["diag (+ blend table)"] - w.cg_iters * gn_ms)
    return out


def serving_leg(args, n_requests: int | None = None, deterministic: bool | None = None) -> dict:
    """Served fits/s and p50/p99 latency on the first requests of the seeded
    Poisson stream of fit requests (256 requests at 20 req/s), against the
    plain sequential solver on the same requests and GPU."""
    import torch

    from paper_2504_12905_amd import serving, synth

    count = n_requests or args.requests
    stream = synth.request_stream(256, args.rate, seed=0)[:count]
    reqs = [serving.FitRequest.from_stream(d) for d in stream]
    det = bool(args.deterministic) if deterministic is None else deterministic
    for r in reqs:
        r.deterministic = det
        if args.lm_iters:
            r.lm_iters = args.lm_iters
    log(f"[serve] preparing {len(reqs)} requests on the host")
    probs = [serving.make_problem(r) for r in reqs]
    budget = int(args.hbm_budget_gb * 2 ** 30)
    # warm the library's kernels once (code-object loading) outside both runs
    serving.run_sequential([serving.make_problem(serving.FitRequest(seed=999, n=2000, sh_degree=3, n_views=4,
                                                                    res=256, lm_iters=2))])
    log("[serve] sequential plain solves")
    seq = serving.run_sequential(probs, hbm_budget_bytes=budget, progress=log)
    s_seq = serving.summarize(seq, probs)
    log(f"[serve] sequential: {s_seq}")
    log(f"[serve] continuous batching, {args.slots} slots, budget {args.hbm_budget_gb} GiB")
    srv = serving.Server(budget, max_slots=args.slots, use_graphs=not args.no_graphs, policy=args.policy,
                         progress=log)
    for p in probs:
        srv.submit(p.req, p)
    got = srv.run_until_idle()
    s_srv = serving.summarize(got, probs)
    log(f"[serve] served: {s_srv}")
    dpsnr = max(abs(got[i].final_psnr - seq[i].final_psnr) for i in got)
    dbeta = max(float(np.linalg.norm(got[i].beta - seq[i].beta) / np.linalg.norm(seq[i].beta)) for i in got)
    torch.cuda.synchronize()
    return {
        "workload": f"fit-request stream: the first {len(reqs)} of 256 requests (Poisson {args.rate} req/s; "
                    f"Gaussians log-uniform 2k-200k, SH 0-3, 4-32 views of 256/512/800 px, every pixel)",
        "requests": len(reqs), "lm_iters": reqs[0].lm_iters, "cg_iters": reqs[0].cg_iters, "lambda": reqs[0].lam,
        "slots": args.slots, "hbm_budget_gib": args.hbm_budget_gb, "graphs": not args.no_graphs,
        "policy": args.policy, "deterministic": det,
        "fits_per_s": round(s_srv["fits_per_s"], 4), "p50_latency_s": round(s_srv["p50_latency_s"], 3),
        "p99_latency_s": round(s_srv["p99_latency_s"], 3),
        "sequential": {k: round(v, 4) if isinstance(v, float) else v for k, v in s_seq.items()},
        "served": {k: round(v, 4) if isinstance(v, float) else v for k, v in s_srv.items()},
        "speedup_fits_per_s": round(s_srv["fits_per_s"] / s_seq["fits_per_s"], 3),
        "max_final_psnr_diff_db": round(dpsnr, 5), "max_beta_rel_diff": dbeta,
        "statuses": sorted({r.status for r in got.values()}),
        "per_request": [{"id": r.id, "n": r.n, "sh": r.sh_degree, "views": r.n_views, "res": r.res,
                         "arrival_s": round(r.arrival_t, 3),
                         "seq_s": round(seq[r.id].end_s - seq[r.id].start_s, 3),
                         "srv_start_s": round(got[r.id].start_s, 3), "srv_end_s": round(got[r.id].end_s, 3),
                         "psnr_seq": round(seq[r.id].final_psnr, 3), "psnr_srv": round(got[r.id].final_psnr, 3)}
                        for r in reqs],
    }


def serving_main(args):
    """--serving: the serving leg alone, as its own JSON line."""
    leg = serving_leg(args)
    res = {"metric": "served fits/s (continuous batching) vs sequential plain solves", "value": leg["fits_per_s"],
           "unit": "fits/s", "n_gpus": 1, "steps": leg["requests"], "warmup": 0,
           "ms_per_step": round(1e3 / leg["fits_per_s"], 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": leg["workload"]}, "serving": leg}
    print(json.dumps(res), flush=True)


def summarize_counters(dirs: list[str], command: str) -> str:
    """Median per dispatch of every counter found in rocprofv3 --pmc output
    folders, for each of the GN product's splat kernels the run launched;
    writes one summary file per kernel."""
    rows_all = [_counter_rows(d) for d in dirs if os.path.isdir(d)]
    texts = []
    for which, (match, title, _, path) in SPLAT_KERNELS.items():
        vals: dict[str, list[float]] = {}
        for rows in rows_all:
            for (k, cn), v in rows.items():
                if match in k:
                    vals.setdefault(cn, []).extend(v)
        vals = {cn: _working(v) for cn, v in vals.items()}
        if not vals:
            continue
        lines = [f"# rocprofv3 counters of {title},",
                 "# 100k-Gaussian object-scale workload (8 views 800x800, 26 samples/tile); median per dispatch",
                 "# over the launches that did the work (those that found the other splat path selected",
                 "# return at once and are left out).",
                 "# Commands (one --pmc pass per counter group, from the repository root):",
                 f"#   {command}"]
        for k in sorted(vals):
            lines.append(f"{k}: {float(np.median(vals[k])):.6g}  (dispatches: {len(vals[k])})")
        text = "\n".join(lines) + "\n"
        with open(path, "w") as f:
            f.write(text)
        texts.append(text)
    if not texts:
        raise SystemExit("no splat kernel dispatches in " + " ".join(dirs))
    return "\n".join(texts)


def run_workload(args, workload: str, steps: int, warmup: int, with_cpu: bool, n: int | None = None) -> dict:
    """LM steps of one workload through the C ABI, timed; then the GN product
    alone, its roofline position, the LM-step stage breakdown and (with_cpu)
    the oracle baseline. Returns the JSON record."""
    import torch

    from paper_2504_12905_amd import lmrs as L
    from paper_2504_12905_amd import synth

    dev = "cuda:0"
    if workload == "cfg1":
        w = synth.config1(**({} if n is None else {"n": n}))
        sampler = L.SAMPLER_UNIFORM
    else:
        w = synth.config2(**({} if n is None else {"n": n}))
        sampler = L.SAMPLER_RESIDUAL
    cams = torch.tensor(w.cams, device=dev)
    beta_gt = torch.tensor(w.beta_gt, device=dev)
    log(f"[bench] {w.name}: rendering {w.cams.shape[0]} targets")
    targets = render_targets(L, torch, w, beta_gt, cams, dev)
    del beta_gt
    V, k = w.views_per_step, w.samples_per_tile
    beta = torch.tensor(w.beta_init, device=dev)
    view_ids = torch.zeros(V, dtype=torch.int32, device=dev)
    fr = L.Frame(w.n, w.sh_degree, beta, cams, w.width, w.height, V, view_ids=view_ids, k=k, sampled=True,
                 deterministic=args.deterministic)
    rep = torch.zeros(L.REPORT_FLOATS, device=dev)
    rng = np.random.default_rng(w.seed)
    ws = None
    # the views of every LM step, drawn up front and kept on the device
    all_vids = torch.tensor(np.stack([rng.choice(w.cams.shape[0], V, replace=False)
                                      for _ in range(warmup + steps)]).astype(np.int32), device=dev)

    def step(it, grow=False):
        view_ids.copy_(all_vids[it])
        # the binding allocates a larger workspace itself if the tile lists outgrow ws
        L.lmrs_lm_step(fr, targets, L.lm_params(it, w.cg_iters, w.lam, seed=w.seed, sampler=sampler), report=rep,
                       ws=ws, grow_blend=grow)

    log(f"[bench] warmup {warmup} LM steps")
    it = 0
    max_pairs = 0
    for _ in range(warmup):
        step(it, grow=True)
        max_pairs = max(max_pairs, fr.blend_pairs())
        it += 1
    # blend table for the largest pair count seen, with room for other view batches
    fr.ensure_blend(int(max_pairs * 1.3))
    torch.cuda.synchronize()
    # grow the workspace once for the largest instance count seen, outside the timed region
    ws = torch.empty(int(L._lib.lmrs_workspace_bytes(L.OP_LM, L.C.byref(fr.struct())) * 1.1) + 4096,
                     dtype=torch.uint8, device=dev)
    log(f"[bench] timing {steps} LM steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(it)
        it += 1
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    products = w.cg_iters * steps
    value = products / el
    r = rep.cpu().numpy()
    log(f"[bench] {el / steps * 1e3:.2f} ms/LM step, {value:.1f} GN products/s; last step: loss "
        f"{r[0]:.4e} eta {r[1]:.3f} instances {r[7]:.0f} blend pairs {r[9]:.0f} (table for {fr.blend_capacity})")

    # --- the GN product on its own, at the current parameters and the last step's samples
    L.lmrs_project(fr)
    L.lmrs_bin_tiles(fr)
    L.lmrs_render(fr)
    torch.cuda.synchronize()
    p = torch.randn(fr.P, generator=torch.Generator(device="cpu").manual_seed(0)).to(dev)
    out = torch.empty_like(p)
    gws = L.workspace(L.OP_GN, fr)
    if args.calibrate_copy:
        copy_calibration(torch, dev, args.calibrate_copy)
    stream = torch.cuda.current_stream()

    def median_gn_ms():
        for _ in range(5):
            L.lmrs_gn_product(fr, p, w.lam, out=out, ws=gws)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.gn_reps)]
        for e0, e1 in ev:
            e0.record(stream)
            L.lmrs_gn_product(fr, p, w.lam, out=out, ws=gws)
            e1.record(stream)
        torch.cuda.synchronize()
        return float(np.median(np.array([e0.elapsed_time(e1) for e0, e1 in ev])))

    # the plain matrix-free product: every product walks the tile lists (the
    # render left the blend table stale)
    assert not fr.blend_built()
    walk_ms = median_gn_ms()
    walk_phases = np.median(np.array([L.lmrs_gn_product_timed(fr, p, w.lam, out=out, ws=gws)[1]
                                      for _ in range(args.gn_reps)]), axis=0)
    # the blend table (built once per LM step by the right-hand-side pass; here on its own)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    L.lmrs_linearize(fr)
    e1.record(stream)
    torch.cuda.synchronize()
    linearize_ms = e0.elapsed_time(e1)
    table = fr.blend_built()
    gn_ms = median_gn_ms()
    phases = np.array([L.lmrs_gn_product_timed(fr, p, w.lam, out=out, ws=gws)[1] for _ in range(args.gn_reps)])
    phase_ms = np.median(phases, axis=0)
    splat_phase = 2 if table else 3
    log(f"[bench] GN product median {gn_ms:.3f} ms over {args.gn_reps} calls (tangent {phase_ms[0]:.3f}, "
        f"fill {phase_ms[1]:.3f}, table splat {phase_ms[2]:.3f}, fused walk {phase_ms[3]:.3f}, "
        f"chain {phase_ms[4]:.3f}); blend table built: {table} ({linearize_ms:.3f} ms on its own); "
        f"walking the lists instead: {walk_ms:.3f} ms (fused walk {walk_phases[3]:.3f})")
    # the unfused comparator: J p to HBM, weights, then J^T u (same state)
    wts = fr.w.view(-1, 1)
    jp = torch.empty((fr.S, 3), dtype=torch.float32, device=dev)
    jtu = torch.empty_like(p)
    for _ in range(3):
        L.lmrs_vjp(fr, L.lmrs_jvp(fr, p, out=jp).mul_(wts), out=jtu)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.gn_reps):
        L.lmrs_vjp(fr, L.lmrs_jvp(fr, p, out=jp).mul_(wts), out=jtu)
    e1.record(stream)
    e1.synchronize()
    unfused_ms = e0.elapsed_time(e1) / args.gn_reps
    out_gpu = out.double().cpu().numpy()
    # the same product in the other accumulation mode (fixed-point sums when
    # the run uses float atomics, and the reverse), phases median of gn_reps
    fr.deterministic = not args.deterministic
    other_ws = L.workspace(L.OP_GN, fr)
    other_phases = np.median(np.array([L.lmrs_gn_product_timed(fr, p, w.lam, out=out, ws=other_ws)[1]
                                       for _ in range(args.gn_reps)]), axis=0)
    fr.deterministic = args.deterministic
    del other_ws
    log(f"[bench] GN product with {'float-atomic' if args.deterministic else 'deterministic'} accumulation: "
        f"{other_phases.sum():.3f} ms (phases {', '.join(f'{x:.4f}' for x in other_phases)})")
    # the state of the timed product, for the oracle (the stage breakdown below re-samples)
    beta_h, pix_h, w_h, vids_h = (fr.beta.cpu().numpy(), fr.pix.cpu().numpy(), fr.w.cpu().numpy(),
                                  view_ids.cpu().numpy())
    cnt = L.lmrs_walk_counts(fr).cpu().numpy().astype(np.int64)
    entries, contrib, n_act, n_walk = (int(x) for x in cnt)
    n_vis = int((fr.rect[..., 0] < fr.rect[..., 2]).sum().item())

    breakdown = lm_breakdown(L, torch, fr, targets, w, sampler, it, gn_ms)
    log("[bench] LM-step stages (ms, each run alone): " + ", ".join(f"{k} {v:.2f}" for k, v in breakdown.items()))

    # --- algorithmic work of the fused splat kernel in the timed launches
    S = fr.S
    b_alg = entries * B_ENTRY + contrib * B_CONTRIB + S * B_PIXEL
    f_alg = n_act * F_ACT + (n_walk - n_act) * F_SKIP
    t_splat = phase_ms[splat_phase] * 1e-3
    gbs = b_alg / t_splat / 1e9
    tflops = f_alg / t_splat / 1e12
    t_hbm, t_alu = b_alg / (HBM_PEAK_GBS * 1e9), f_alg / (FP32_PEAK_TFLOPS * 1e12)
    bound_alu = t_alu > t_hbm
    kernel_hash = hashlib.sha256(open(SPLAT_SOURCE, "rb").read()).hexdigest()
    # the committed counter summaries cover the float-atomic kernels
    traffic = None if args.deterministic else traffic_from_profile(kernel_hash, workload == "cfg1" and n is None,
                                                                   "table" if table else "walk")
    # the whole GN product (tangent projection, splat, reverse chain)
    b_gn = 4 * fr.P * 3 + n_vis * B_VIS + b_alg
    f_gn = f_alg + n_vis * F_VIS
    t_gn = gn_ms * 1e-3
    roofline = {
        "kernel": (f"blend_gn_kernel<{'true' if args.deterministic else 'false'}> (J p / weight / J^T u over the "
                   "blend table, in lmrs_gn_product)" if table
                   else "deriv_kernel<3> (fused J p / weight / J^T u walk of lmrs_gn_product)"),
        "bound": "alu" if bound_alu else "hbm",
        "achieved": round(tflops if bound_alu else gbs, 4),
        "peak": FP32_PEAK_TFLOPS if bound_alu else HBM_PEAK_GBS,
        "unit": "TFLOP/s" if bound_alu else "GB/s",
        "frac": round((t_alu if bound_alu else t_hbm) / t_splat, 6),
        "traffic": traffic,
        "hbm_gbs": round(gbs, 3), "hbm_frac": round(gbs / HBM_PEAK_GBS, 6),
        "alu_tflops": round(tflops, 4), "alu_frac": round(tflops / FP32_PEAK_TFLOPS, 6),
        "alu_frac_of_unpacked_fp32_rate_note": round(tflops / FP32_UNPACKED_TFLOPS, 6),
        "t_hbm_bound_ms": round(t_hbm * 1e3, 5), "t_alu_bound_ms": round(t_alu * 1e3, 5),
        "algorithmic_bytes": b_alg, "algorithmic_flops": f_alg,
        "traversed_entries": entries, "contributing_entries": contrib, "blending_pairs": n_act,
        "walked_pairs": n_walk, "sampled_pixels": S, "visible_view_gaussians": n_vis,
        "ms_per_launch": round(float(phase_ms[splat_phase]), 4),
        "gn_product": {"algorithmic_bytes": b_gn, "algorithmic_flops": f_gn, "ms": round(gn_ms, 4),
                       "hbm_gbs": round(b_gn / t_gn / 1e9, 3), "hbm_frac": round(b_gn / t_gn / 1e9 / HBM_PEAK_GBS, 6),
                       "alu_frac": round(f_gn / t_gn / 1e12 / FP32_PEAK_TFLOPS, 6)},
    }

    cpu, parity = None, None
    if with_cpu:
        log("[bench] CPU oracle baseline (the same GN product in FP64)")
        cpu, ref = cpu_baseline(w, beta_h, w.cams, vids_h, pix_h, w_h, w.lam, p.cpu().numpy(), args.cpu_budget,
                                n_views=None if workload == "cfg1" else 2,
                                one_core_views=1 if workload == "cfg1" else None)
        if ref is not None:
            parity = float(np.linalg.norm(out_gpu - ref) / np.linalg.norm(ref))
        log(f"[bench] oracle {cpu['value']:.4f} GN products/s on {cpu['cores']} threads; "
            f"GPU vs oracle rel {parity}")

    res = {
        "metric": METRIC, "value": round(value, 3), "unit": "GN products/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": round(el / steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "gaussians": w.n, "sh_degree": w.sh_degree,
                   "views_per_step": V, "views_total": int(w.cams.shape[0]), "resolution": [w.width, w.height],
                   "samples_per_tile": k, "cg_iters": w.cg_iters, "lambda": w.lam,
                   "deterministic": bool(args.deterministic),
                   "gn_product_ms_median": round(gn_ms, 4),
                   "gn_products_per_s_isolated": round(1e3 / gn_ms, 2),
                   "gn_phase_ms_median": [round(float(x), 4) for x in phase_ms],
                   "gn_phases": ["tangent", "fill", "blend-table splat", "fused walk", "chain"],
                   "gn_walk_ms_median": round(walk_ms, 4),
                   "gn_walk_phase_ms_median": [round(float(x), 4) for x in walk_phases],
                   ("gn_float_atomic_phase_ms_median" if args.deterministic else
                    "gn_deterministic_phase_ms_median"): [round(float(x), 4) for x in other_phases],
                   "linearize_ms": round(linearize_ms, 4),
                   "blend_table": {"built": table, "pairs": fr.blend_pairs(), "bytes_per_pair": 44},
                   "gn_unfused_jvp_vjp_ms": round(unfused_ms, 4),
                   "gn_parity_rel_vs_oracle": parity,
                   "sampler": "residual" if sampler == L.SAMPLER_RESIDUAL else "uniform",
                   "lm_step_stage_ms": {k: round(v, 3) for k, v in breakdown.items()}},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    del fr, targets, ws
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--gn-reps", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--n", type=int, default=None, help="Gaussians (default: the workload's)")
    ap.add_argument("--workload", choices=["cfg1", "cfg2"], default="cfg1",
                    help="cfg1: 100k-Gaussian object-scale fit (default); cfg2: 1.5M-Gaussian "
                         "unbounded-scene fit with residual-weighted sampling")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="run MIB-MiB device copies before the GN timing (HBM-counter calibration)")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the splat traffic summary from two rocprofv3 --pmc output folders and exit")
    ap.add_argument("--traffic-command", default="", help="command line recorded in the traffic summary")
    ap.add_argument("--summarize-counters", nargs="+", metavar="PMC_DIR",
                    help="write the splat counter summary from rocprofv3 --pmc output folders and exit")
    ap.add_argument("--serving", action="store_true", help="serving benchmark (fit-request stream)")
    ap.add_argument("--requests", type=int, default=32, help="requests of the serving leg (first of the 256)")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the 100k workload (no 1.5M-Gaussian and serving sub-records)")
    ap.add_argument("--cfg2-steps", type=int, default=5, help="timed LM steps of the 1.5M-Gaussian sub-record")
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--hbm-budget-gb", type=float, default=200.0)
    ap.add_argument("--lm-iters", type=int, default=0, help="override the requests' LM iterations")
    ap.add_argument("--no-graphs", action="store_true")
    ap.add_argument("--policy", choices=["fifo", "sjf"], default="fifo", help="serving admission order")
    ap.add_argument("--deterministic", action="store_true",
                    help="fixed-point accumulation (the same bits on every run) for the workload and the fits")
    args = ap.parse_args()
    if args.serving:
        return serving_main(args)
    if args.summarize_counters:
        print(summarize_counters(args.summarize_counters, args.traffic_command))
        return
    if args.summarize_traffic:
        print(summarize_traffic(*args.summarize_traffic, args.calibrate_copy or 1024, args.traffic_command))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU layout "
              "(view sharding, one all-reduce per GN product) is described in DESIGN.md", file=sys.stderr)
        sys.exit(2)

    primary = run_workload(args, args.workload, args.steps, args.warmup, not args.no_cpu, args.n)
    if args.workload == "cfg1" and args.n is None and not args.no_extra:
        # the 1.5M-Gaussian unbounded-scene workload: LM-step time and GN-product bandwidth
        sub = run_workload(args, "cfg2", args.cfg2_steps, 2, False)
        primary["cfg2"] = {k: sub[k] for k in ("value", "unit", "ms_per_step", "steps", "warmup", "config",
                                                "roofline")}
        # served fits/s and latency against the sequential plain solver
        primary["serving"] = serving_leg(args)
        if not args.deterministic:
            # the same stream with deterministic accumulation: served and
            # sequential fits then end with the same bits
            try:
                leg = serving_leg(args, deterministic=True)
                primary["serving_deterministic"] = {k: v for k, v in leg.items() if k != "per_request"}
            except Exception as e:  # reported, not fatal to the headline line
                primary["serving_deterministic"] = {"error": f"{type(e).__name__}: {e}"}
    print(json.dumps(primary), flush=True)


if __name__ == "__main__":
    main()
