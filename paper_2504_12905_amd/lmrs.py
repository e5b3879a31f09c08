"""Python binding of liblmrs (argument marshalling only).

Every call forwards device pointers of torch tensors and the current HIP stream
to the C ABI declared in include/lmrs.h; all arithmetic runs in the library's
HIP kernels. Importing this module raises if the library has not been built:
there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblmrs.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"liblmrs.so not built at {LIB_PATH}: run __graft_entry__.build() first")

_lib = C.CDLL(LIB_PATH)

LMRS_OK, LMRS_EINVAL, LMRS_ECAPACITY, LMRS_EWORKSPACE, LMRS_EHIP = 0, -1, -2, -3, -4
LMRS_ENUMERIC, LMRS_EUNSUPPORTED = -5, -6
LMRS_REC = 12
OP_BIN, OP_JVP, OP_VJP, OP_GN, OP_DIAG, OP_PCG, OP_LM, OP_SOLVE = 1, 2, 3, 4, 5, 6, 7, 8
REPORT_FLOATS = 12
SAMPLER_UNIFORM, SAMPLER_RESIDUAL, SAMPLER_GAUSSIAN = 0, 1, 2
REP = dict(loss=0, eta=1, xdc_max=2, cg_done=3, r0=4, rn=5, bx=6, instances=7, status=8, pairs=9)
FAIL_NONFINITE, FAIL_BREAKDOWN, FAIL_CAPACITY = 1, 2, 4


class LmrsError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.lmrs_last_error().decode()
        super().__init__(f"{where}: {_lib.lmrs_status_str(status).decode()} ({msg})")
        self.status = status


class RenderOpts(C.Structure):
    _fields_ = [("alpha_min", C.c_float), ("alpha_max", C.c_float), ("t_min", C.c_float),
                ("lowpass", C.c_float), ("znear", C.c_float), ("cutoff", C.c_float),
                ("bg", C.c_float * 3)]


def default_opts(**kw) -> RenderOpts:
    o = RenderOpts(1.0 / 255.0, 0.99, 1e-4, 0.3, 0.2, 3.0, (C.c_float * 3)(0.0, 0.0, 0.0))
    for k, v in kw.items():
        if k == "bg":
            o.bg = (C.c_float * 3)(*v)
        else:
            setattr(o, k, v)
    return o


class _Frame(C.Structure):
    _fields_ = [("n", C.c_int32), ("sh_degree", C.c_int32), ("n_views", C.c_int32),
                ("width", C.c_int32), ("height", C.c_int32), ("k", C.c_int32),
                ("beta", C.c_void_p), ("cams", C.c_void_p), ("view_ids", C.c_void_p),
                ("rec", C.c_void_p), ("rect", C.c_void_p), ("tile_start", C.c_void_p),
                ("ids", C.c_void_p), ("capacity", C.c_int64), ("n_instances", C.c_void_p),
                ("pix", C.c_void_p), ("w", C.c_void_p), ("color", C.c_void_p),
                ("trans", C.c_void_p), ("last", C.c_void_p), ("sched", C.c_void_p),
                ("blend_k", C.c_void_p), ("blend_m", C.c_void_p), ("blend_run", C.c_void_p),
                ("blend_runs", C.c_void_p), ("blend_start", C.c_void_p), ("blend_capacity", C.c_int64),
                ("wc", C.c_void_p), ("image", C.c_void_p), ("deterministic", C.c_int32)]


BLEND_BYTES_PER_PAIR = 44   # blend_k (2 x 16) + blend_m (2 x 4) + blend_run (4)


def sched_ints(tiles: int) -> int:
    """int32 length of lmrs_frame.sched for `tiles` = V*T (LMRS_SCHED_INTS)."""
    return 2 * int(tiles) + 4


class LmParams(C.Structure):
    _fields_ = [("iter", C.c_int32), ("cg_iters", C.c_int32), ("lam", C.c_float),
                ("eta_cap", C.c_float), ("eta_warm", C.c_float), ("warm_iters", C.c_int32),
                ("seed", C.c_uint64), ("sampler", C.c_int32), ("cg_iters_late", C.c_int32),
                ("late_iter", C.c_int32), ("ssim_weight", C.c_float)]


_vp, _i32, _f32, _sz = C.c_void_p, C.c_int32, C.c_float, C.c_size_t
_FP = C.POINTER(_Frame)
_lib.lmrs_status_str.restype = C.c_char_p
_lib.lmrs_status_str.argtypes = [_i32]
_lib.lmrs_last_error.restype = C.c_char_p
_lib.lmrs_report_status.restype = _i32
_lib.lmrs_report_status.argtypes = [_vp]
_lib.lmrs_workspace_bytes.restype = _sz
_lib.lmrs_workspace_bytes.argtypes = [_i32, _FP]
_lib.lmrs_project.argtypes = [_FP, _vp, _vp]
_lib.lmrs_bin_tiles.argtypes = [_FP, _vp, _sz, _vp]
_lib.lmrs_render.argtypes = [_FP, _vp, _vp]
_lib.lmrs_jvp.argtypes = [_FP, _vp, _vp, _vp, _vp, _sz, _vp]
_lib.lmrs_vjp.argtypes = [_FP, _vp, _vp, _vp, _vp, _sz, _vp]
_lib.lmrs_gn_product.argtypes = [_FP, _vp, _vp, _f32, _vp, _vp, _vp, _sz, _vp]
_lib.lmrs_gn_product_timed.argtypes = [_FP, _vp, _vp, _f32, _vp, _vp, _vp, _sz, _vp, _vp]
_lib.lmrs_gn_product_noalloc.argtypes = [_FP, _vp, _vp, _f32, _vp, _vp, _vp]
_lib.lmrs_walk_counts.argtypes = [_FP, _vp, _vp, _vp]
_lib.lmrs_linearize.argtypes = [_FP, _vp, _vp]
_lib.lmrs_gn_diag.argtypes = [_FP, _vp, _vp, _vp, _sz, _vp]
_lib.lmrs_pcg.argtypes = [_FP, _vp, _vp, _f32, _vp, _i32, _vp, _vp, _vp, _sz, _vp]
_lib.lmrs_lm_step.argtypes = [_FP, _vp, _vp, _vp, C.POINTER(LmParams), _vp, _vp, _vp, _sz, _vp]
_lib.lmrs_lm_solve.argtypes = [_FP, _vp, _vp, _vp, C.POINTER(LmParams), _vp, _vp, _vp, _sz, _vp]
_lib.lmrs_lm_iterate.argtypes = [_FP, _vp, _vp, _vp, C.POINTER(LmParams), _vp, _vp, _vp, _sz, _vp]
_lib.lmrs_bin_tiles_async.argtypes = [_FP, _vp, _sz, _vp]
_lib.lmrs_residual_scores.argtypes = [_FP, _vp, _vp, _vp, _vp]
_lib.lmrs_sample.argtypes = [_FP, _i32, C.c_uint64, _i32, _vp, _vp]
_lib.lmrs_contributor_counts.argtypes = [_FP, _vp, _vp, _vp]
_lib.lmrs_ssim_residual.argtypes = [_FP, _vp, _vp, _f32, _vp, _vp, _vp]
_lib.lmrs_view_clusters.argtypes = [_vp, _i32, _i32, C.c_uint64, _vp]
_lib.lmrs_view_batch.argtypes = [_vp, _i32, _i32, C.c_uint64, _i32, _vp]
for _name in ("lmrs_project", "lmrs_bin_tiles", "lmrs_render", "lmrs_jvp", "lmrs_vjp",
              "lmrs_gn_product", "lmrs_gn_product_timed", "lmrs_gn_product_noalloc", "lmrs_walk_counts", "lmrs_linearize",
              "lmrs_gn_diag", "lmrs_pcg", "lmrs_lm_step", "lmrs_residual_scores", "lmrs_sample", "lmrs_lm_solve",
              "lmrs_contributor_counts", "lmrs_view_clusters", "lmrs_view_batch", "lmrs_lm_iterate",
              "lmrs_bin_tiles_async", "lmrs_ssim_residual"):
    getattr(_lib, _name).restype = _i32


def _ptr(t: torch.Tensor | None):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _check(status: int, where: str):
    if status != LMRS_OK:
        raise LmrsError(status, where)


@dataclass
class Frame:
    """Device buffers of one view batch (see lmrs_frame in include/lmrs.h).

    beta: float32 [P]; cams: float32 [V_total, 16]; view_ids: int32 [V] or None
    (batch view v is camera v); k: samples per tile (256 = all pixels).
    """
    n: int
    sh_degree: int
    beta: torch.Tensor
    cams: torch.Tensor
    width: int
    height: int
    n_views: int
    view_ids: torch.Tensor | None = None
    k: int = 256
    sampled: bool = False          # allocate pix / w (needed when k < 256)
    capacity: int = 0
    blend: bool = True             # keep the blend table (the render's linearization; see lmrs_frame)
    blend_capacity: int = 0        # pairs it can hold (grown by ensure_blend)
    ssim: bool = False             # allocate wc / image (the SSIM residual's buffers)
    deterministic: bool = False    # fixed-point sums over tiles: the same bits on every run
    tensors: dict = field(default_factory=dict)

    def __post_init__(self):
        dev = self.beta.device
        V, n = self.n_views, self.n
        self.TX, self.TY = self.width // 16, self.height // 16
        self.T = self.TX * self.TY
        self.P = n * (11 + 3 * (self.sh_degree + 1) ** 2)
        assert self.beta.dtype == torch.float32 and self.beta.numel() == self.P and self.beta.is_contiguous()
        assert self.cams.dtype == torch.float32 and self.cams.shape[-1] == 16
        if self.view_ids is not None:
            assert self.view_ids.dtype == torch.int32 and self.view_ids.numel() == V
        t = self.tensors
        t["rec"] = torch.empty((V, n, LMRS_REC), dtype=torch.float32, device=dev)
        t["rect"] = torch.empty((V, n, 4), dtype=torch.int32, device=dev)
        t["tile_start"] = torch.zeros(V * self.T + 1, dtype=torch.int64, device=dev)
        t["n_instances"] = torch.zeros(1, dtype=torch.int64, device=dev)
        t["sched"] = torch.zeros(sched_ints(V * self.T), dtype=torch.int32, device=dev)
        t["ids"] = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=dev)
        if self.blend:
            t["blend_start"] = torch.zeros(V * self.T + 2, dtype=torch.int64, device=dev)
            t["blend_runs"] = torch.zeros(V * self.T, dtype=torch.int32, device=dev)
            self._alloc_blend(self.blend_capacity)
        self.set_k(self.k, self.sampled or self.k < 256)

    def _alloc_blend(self, cap: int):
        dev = self.beta.device
        t = self.tensors
        for key in ("blend_k", "blend_m", "blend_run"):   # the old table goes before the new one comes
            t.pop(key, None)
        self.blend_capacity = max(int(cap), 0)
        m = max(self.blend_capacity, 1)
        t["blend_k"] = torch.empty((2, m, 4), dtype=torch.float32, device=dev)   # two orders of the pairs
        t["blend_m"] = torch.empty((2, m), dtype=torch.int32, device=dev)
        t["blend_run"] = torch.empty(m, dtype=torch.int32, device=dev)
        if "blend_start" in t:
            t["blend_start"][self.n_views * self.T + 1] = 0   # new buffers hold no table

    def blend_pairs(self) -> int:
        """Blending (pixel, Gaussian) pairs of the last render (waits for the device)."""
        return int(self.tensors["blend_start"][self.n_views * self.T].item()) if self.blend else 0

    def blend_built(self) -> bool:
        return bool(self.blend and int(self.tensors["blend_start"][self.n_views * self.T + 1].item()) == 1)

    def set_blend_capacity(self, pairs: int):
        """Reallocates the blend table for exactly `pairs` pairs (the table is then unbuilt)."""
        if self.blend:
            self._alloc_blend(pairs)

    def ensure_blend(self, needed: int | None = None, margin: float = 1.15) -> bool:
        """Grows the blend table to hold `needed` pairs (default: the last
        render's count); returns True when it grew."""
        if not self.blend:
            return False
        needed = self.blend_pairs() if needed is None else int(needed)
        if needed <= self.blend_capacity:
            return False
        self._alloc_blend(int(needed * margin) + 4096)
        return True

    def set_k(self, k: int, sampled: bool):
        dev = self.beta.device
        self.k, self.sampled = int(k), bool(sampled)
        S = self.n_views * self.T * self.k
        t = self.tensors
        if self.sampled:
            t["pix"] = torch.empty((self.n_views, self.T, self.k), dtype=torch.uint8, device=dev)
            t["w"] = torch.empty((self.n_views, self.T, self.k), dtype=torch.float32, device=dev)
        else:
            t["pix"], t["w"] = None, None
        t["color"] = torch.empty((S, 3), dtype=torch.float32, device=dev)
        if self.ssim:
            t["wc"] = torch.empty((S, 3), dtype=torch.float32, device=dev)
            t["image"] = torch.empty((self.n_views, self.height, self.width, 3), dtype=torch.float32, device=dev)
        else:
            t["wc"], t["image"] = None, None
        t["trans"] = torch.empty(S, dtype=torch.float32, device=dev)
        t["last"] = torch.empty(S, dtype=torch.int32, device=dev)

    @property
    def S(self) -> int:
        return self.n_views * self.T * self.k

    def __getattr__(self, name):
        t = self.__dict__.get("tensors", {})
        if name in t:
            return t[name]
        raise AttributeError(name)

    def struct(self) -> _Frame:
        t = self.tensors
        return _Frame(self.n, self.sh_degree, self.n_views, self.width, self.height, self.k,
                      self.beta.data_ptr(), self.cams.data_ptr(),
                      None if self.view_ids is None else self.view_ids.data_ptr(),
                      t["rec"].data_ptr(), t["rect"].data_ptr(), t["tile_start"].data_ptr(),
                      t["ids"].data_ptr(), self.capacity, t["n_instances"].data_ptr(),
                      None if t["pix"] is None else t["pix"].data_ptr(),
                      None if t["w"] is None else t["w"].data_ptr(),
                      t["color"].data_ptr(), t["trans"].data_ptr(), t["last"].data_ptr(),
                      t["sched"].data_ptr(), *self._blend_fields(),
                      None if t["wc"] is None else t["wc"].data_ptr(),
                      None if t["image"] is None else t["image"].data_ptr(),
                      1 if self.deterministic else 0)

    def _blend_fields(self):
        if not self.blend:
            return (None, None, None, None, None, 0)
        t = self.tensors
        return (t["blend_k"].data_ptr(), t["blend_m"].data_ptr(), t["blend_run"].data_ptr(),
                t["blend_runs"].data_ptr(), t["blend_start"].data_ptr(), self.blend_capacity)

    def grow_ids(self, needed: int):
        self.capacity = int(needed * 1.25) + 1024
        self.tensors["ids"] = torch.empty(self.capacity, dtype=torch.int32, device=self.beta.device)


def workspace_bytes(op: int, frame: Frame) -> int:
    fs = frame.struct()
    return int(_lib.lmrs_workspace_bytes(op, C.byref(fs)))


def workspace(op: int, frame: Frame) -> torch.Tensor:
    return torch.empty(max(workspace_bytes(op, frame), 256), dtype=torch.uint8, device=frame.beta.device)


def lmrs_project(frame: Frame, opts: RenderOpts | None = None, stream=None):
    opts = opts or default_opts()
    fs = frame.struct()
    _check(_lib.lmrs_project(C.byref(fs), C.byref(opts), _stream(stream)), "lmrs_project")


def lmrs_bin_tiles(frame: Frame, stream=None, ws: torch.Tensor | None = None) -> int:
    """Bins; grows the id buffer and retries when the capacity is exceeded.
    ws: optional caller workspace, used when it holds lmrs_workspace_bytes(OP_BIN)."""
    for _ in range(2):
        fs = frame.struct()
        need = _lib.lmrs_workspace_bytes(OP_BIN, C.byref(fs))
        w = ws if (ws is not None and ws.numel() >= need) else workspace(OP_BIN, frame)
        st = _lib.lmrs_bin_tiles(C.byref(fs), _ptr(w), w.numel(), _stream(stream))
        if st == LMRS_ECAPACITY:
            frame.grow_ids(int(frame.n_instances.item()))
            continue
        _check(st, "lmrs_bin_tiles")
        return int(frame.n_instances.item())
    raise LmrsError(LMRS_ECAPACITY, "lmrs_bin_tiles")


def lmrs_render(frame: Frame, opts: RenderOpts | None = None, stream=None, grow_blend: bool = True):
    """grow_blend: afterwards wait for the render's pair count and grow the
    frame's blend table to hold it (so that lmrs_linearize can build it)."""
    opts = opts or default_opts()
    fs = frame.struct()
    _check(_lib.lmrs_render(C.byref(fs), C.byref(opts), _stream(stream)), "lmrs_render")
    if grow_blend and frame.blend:
        frame.ensure_blend()


def lmrs_linearize(frame: Frame, opts: RenderOpts | None = None, stream=None):
    """Builds the frame's blend table for its current render (see lmrs_linearize in lmrs.h)."""
    opts = opts or default_opts()
    fs = frame.struct()
    _check(_lib.lmrs_linearize(C.byref(fs), C.byref(opts), _stream(stream)), "lmrs_linearize")


def lmrs_jvp(frame: Frame, p: torch.Tensor, out: torch.Tensor | None = None, opts=None, stream=None):
    opts = opts or default_opts()
    out = out if out is not None else torch.empty((frame.S, 3), dtype=torch.float32, device=p.device)
    ws = workspace(OP_JVP, frame)
    fs = frame.struct()
    _check(_lib.lmrs_jvp(C.byref(fs), C.byref(opts), _ptr(p), _ptr(out), _ptr(ws), ws.numel(),
                         _stream(stream)), "lmrs_jvp")
    return out


def lmrs_vjp(frame: Frame, u: torch.Tensor, out: torch.Tensor | None = None, opts=None, stream=None):
    opts = opts or default_opts()
    out = out if out is not None else torch.empty(frame.P, dtype=torch.float32, device=u.device)
    ws = workspace(OP_VJP, frame)
    fs = frame.struct()
    _check(_lib.lmrs_vjp(C.byref(fs), C.byref(opts), _ptr(u), _ptr(out), _ptr(ws), ws.numel(),
                         _stream(stream)), "lmrs_vjp")
    return out


def lmrs_gn_product(frame: Frame, p: torch.Tensor, lam: float, d: torch.Tensor | None = None,
                    out: torch.Tensor | None = None, opts=None, stream=None, ws: torch.Tensor | None = None):
    opts = opts or default_opts()
    out = out if out is not None else torch.empty(frame.P, dtype=torch.float32, device=p.device)
    ws = ws if ws is not None else workspace(OP_GN, frame)
    fs = frame.struct()
    _check(_lib.lmrs_gn_product(C.byref(fs), C.byref(opts), _ptr(p), float(lam), _ptr(d), _ptr(out),
                                _ptr(ws), ws.numel(), _stream(stream)), "lmrs_gn_product")
    return out


def lmrs_gn_product_noalloc(frame: Frame, p: torch.Tensor, lam: float, out: torch.Tensor,
                            d: torch.Tensor | None = None, opts=None, stream=None):
    """lmrs_gn_product with the library's static scratch array (no workspace;
    the C call allocates nothing). out: caller-allocated [P]."""
    opts = opts or default_opts()
    fs = frame.struct()
    _check(_lib.lmrs_gn_product_noalloc(C.byref(fs), C.byref(opts), _ptr(p), float(lam), _ptr(d), _ptr(out),
                                        _stream(stream)), "lmrs_gn_product_noalloc")
    return out


def lmrs_gn_product_timed(frame: Frame, p: torch.Tensor, lam: float, d: torch.Tensor | None = None,
                          out: torch.Tensor | None = None, opts=None, stream=None,
                          ws: torch.Tensor | None = None):
    """Returns (out, [ms tangent, ms fill, ms blend-table splat, ms fused walk, ms chain]);
    of the two splats one exits at once (the table when it is not built)."""
    opts = opts or default_opts()
    out = out if out is not None else torch.empty(frame.P, dtype=torch.float32, device=p.device)
    ws = ws if ws is not None else workspace(OP_GN, frame)
    ms = (C.c_float * 5)()
    fs = frame.struct()
    _check(_lib.lmrs_gn_product_timed(C.byref(fs), C.byref(opts), _ptr(p), float(lam), _ptr(d), _ptr(out),
                                      _ptr(ws), ws.numel(), _stream(stream), ms), "lmrs_gn_product_timed")
    return out, [float(x) for x in ms]


def lmrs_walk_counts(frame: Frame, opts=None, stream=None) -> torch.Tensor:
    """int64 [4] on the device: traversed entries (sum L*_t), contributing
    entries (sum C_t), blending pairs, pairs up to each pixel's last blend."""
    opts = opts or default_opts()
    out = torch.empty(4, dtype=torch.int64, device=frame.beta.device)
    fs = frame.struct()
    _check(_lib.lmrs_walk_counts(C.byref(fs), C.byref(opts), _ptr(out), _stream(stream)), "lmrs_walk_counts")
    return out


def lmrs_gn_diag(frame: Frame, out: torch.Tensor | None = None, opts=None, stream=None):
    opts = opts or default_opts()
    out = out if out is not None else torch.empty(frame.P, dtype=torch.float32, device=frame.beta.device)
    ws = workspace(OP_DIAG, frame)
    fs = frame.struct()
    _check(_lib.lmrs_gn_diag(C.byref(fs), C.byref(opts), _ptr(out), _ptr(ws), ws.numel(),
                             _stream(stream)), "lmrs_gn_diag")
    return out


def lmrs_pcg(frame: Frame, b: torch.Tensor, lam: float, iters: int, d: torch.Tensor | None = None,
             x: torch.Tensor | None = None, report: torch.Tensor | None = None, opts=None, stream=None):
    opts = opts or default_opts()
    x = x if x is not None else torch.empty(frame.P, dtype=torch.float32, device=b.device)
    ws = workspace(OP_PCG, frame)
    fs = frame.struct()
    _check(_lib.lmrs_pcg(C.byref(fs), C.byref(opts), _ptr(b), float(lam), _ptr(d), int(iters), _ptr(x),
                         _ptr(report), _ptr(ws), ws.numel(), _stream(stream)), "lmrs_pcg")
    return x


def lmrs_residual_scores(frame: Frame, targets: torch.Tensor, out: torch.Tensor | None = None, opts=None,
                         stream=None) -> torch.Tensor:
    """[V, T, 256] residual magnitudes of every pixel (needs project + bin)."""
    opts = opts or default_opts()
    assert targets.dtype == torch.float32 and targets.is_contiguous()
    out = out if out is not None else torch.empty((frame.n_views, frame.T, 256), dtype=torch.float32,
                                                  device=frame.beta.device)
    fs = frame.struct()
    _check(_lib.lmrs_residual_scores(C.byref(fs), C.byref(opts), _ptr(targets), _ptr(out), _stream(stream)),
           "lmrs_residual_scores")
    return out


def lmrs_contributor_counts(frame: Frame, out: torch.Tensor | None = None, opts=None, stream=None) -> torch.Tensor:
    """[V, T, 256] number of Gaussians blended into every pixel (needs project + bin)."""
    opts = opts or default_opts()
    out = out if out is not None else torch.empty((frame.n_views, frame.T, 256), dtype=torch.float32,
                                                  device=frame.beta.device)
    fs = frame.struct()
    _check(_lib.lmrs_contributor_counts(C.byref(fs), C.byref(opts), _ptr(out), _stream(stream)),
           "lmrs_contributor_counts")
    return out


def lmrs_ssim_residual(frame: Frame, targets: torch.Tensor, s: float = 0.2, u: torch.Tensor | None = None,
                       tile_loss: torch.Tensor | None = None, opts=None, stream=None) -> torch.Tensor:
    """SSIM residual with the diagonal approximation at the frame's samples
    (needs project + bin + samples; frame built with ssim=True): renders every
    pixel into frame.image, writes frame.wc and returns u [S, 3] =
    w (r + s delta rho). tile_loss: float64 [V*T] or None."""
    opts = opts or default_opts()
    assert frame.ssim, "Frame(ssim=True) holds the SSIM buffers"
    assert targets.dtype == torch.float32 and targets.is_contiguous()
    assert targets.shape[1:] == (frame.height, frame.width, 3)
    u = u if u is not None else torch.empty((frame.S, 3), dtype=torch.float32, device=frame.beta.device)
    assert u.dtype == torch.float32 and u.is_contiguous() and u.numel() == 3 * frame.S
    if tile_loss is not None:
        assert tile_loss.dtype == torch.float64 and tile_loss.numel() == frame.n_views * frame.T
    fs = frame.struct()
    _check(_lib.lmrs_ssim_residual(C.byref(fs), C.byref(opts), _ptr(targets), float(s), _ptr(u), _ptr(tile_loss),
                                   _stream(stream)), "lmrs_ssim_residual")
    return u


def lmrs_sample(frame: Frame, sampler: int, seed: int, iter: int, scores: torch.Tensor | None = None,
                stream=None):
    """Fills frame.pix / frame.w (frame must be sampled)."""
    if scores is not None:
        assert scores.dtype == torch.float32 and scores.is_contiguous()
        assert scores.numel() == frame.n_views * frame.T * 256
    fs = frame.struct()
    _check(_lib.lmrs_sample(C.byref(fs), int(sampler), int(seed), int(iter), _ptr(scores), _stream(stream)),
           "lmrs_sample")


def lmrs_lm_step(frame: Frame, targets: torch.Tensor, params: LmParams, d: torch.Tensor | None = None,
                 report: torch.Tensor | None = None, opts=None, stream=None, ws: torch.Tensor | None = None,
                 grow_blend: bool = True):
    """One LM iteration in place on frame.beta; grows the id buffer and retries on overflow.
    grow_blend: afterwards wait for the step's pair count and grow the frame's
    blend table for the next step (a step whose pairs do not fit walks the
    lists instead)."""
    opts = opts or default_opts()
    for _ in range(3):
        fs = frame.struct()
        w = ws if (ws is not None and ws.numel() >= _lib.lmrs_workspace_bytes(OP_LM, C.byref(fs))) \
            else workspace(OP_LM, frame)
        st = _lib.lmrs_lm_step(C.byref(fs), _ptr(frame.beta), _ptr(targets), _ptr(d), C.byref(params),
                               C.byref(opts), _ptr(report), _ptr(w), w.numel(), _stream(stream))
        if st == LMRS_ECAPACITY:
            frame.grow_ids(int(frame.n_instances.item()))
            continue
        _check(st, "lmrs_lm_step")
        if grow_blend and frame.blend:
            frame.ensure_blend()
        return
    raise LmrsError(LMRS_ECAPACITY, "lmrs_lm_step")


def lmrs_bin_tiles_async(frame: Frame, ws: torch.Tensor, stream=None):
    """Binning without the host wait (lists empty if frame.capacity is too small)."""
    fs = frame.struct()
    _check(_lib.lmrs_bin_tiles_async(C.byref(fs), _ptr(ws), ws.numel(), _stream(stream)), "lmrs_bin_tiles_async")


def lmrs_lm_iterate(frame: Frame, targets: torch.Tensor, params: LmParams, ws: torch.Tensor,
                    d: torch.Tensor | None = None, report: torch.Tensor | None = None, opts=None, stream=None):
    """One LM iteration that never waits on the host (graph-capturable).
    ws: at least lmrs_workspace_bytes(OP_LM) bytes. A tile-list count above
    frame.capacity shows as FAIL_CAPACITY in the report."""
    opts = opts or default_opts()
    fs = frame.struct()
    _check(_lib.lmrs_lm_iterate(C.byref(fs), _ptr(frame.beta), _ptr(targets), _ptr(d), C.byref(params),
                                C.byref(opts), _ptr(report), _ptr(ws), ws.numel(), _stream(stream)),
           "lmrs_lm_iterate")


def lmrs_lm_solve(frame: Frame, targets: torch.Tensor, params: LmParams, ws: torch.Tensor,
                  d: torch.Tensor | None = None, report: torch.Tensor | None = None, opts=None, stream=None):
    """The LM iteration after project + bin (no host wait; graph-capturable).
    ws: at least lmrs_workspace_bytes(OP_SOLVE) bytes (see workspace())."""
    opts = opts or default_opts()
    fs = frame.struct()
    _check(_lib.lmrs_lm_solve(C.byref(fs), _ptr(frame.beta), _ptr(targets), _ptr(d), C.byref(params),
                              C.byref(opts), _ptr(report), _ptr(ws), ws.numel(), _stream(stream)),
           "lmrs_lm_solve")


def check_report(report: torch.Tensor, where: str = "report"):
    """Raises LmrsError(LMRS_ENUMERIC) when a report (device or host tensor of
    REPORT_FLOATS floats) carries numeric-failure bits (waits for the device)."""
    host = report.detach().to("cpu", torch.float32).contiguous()
    _check(_lib.lmrs_report_status(C.c_void_p(host.data_ptr())), where)


def view_clusters(cams: "np.ndarray", batch: int, seed: int) -> "np.ndarray":
    """Cluster label of every camera (host float32 [N, 16] rows), Sec. 4.3."""
    import numpy as np
    cams = np.ascontiguousarray(cams, dtype=np.float32)
    labels = np.zeros(cams.shape[0], np.int32)
    _check(_lib.lmrs_view_clusters(C.c_void_p(cams.ctypes.data), cams.shape[0], int(batch), int(seed),
                                   C.c_void_p(labels.ctypes.data)), "lmrs_view_clusters")
    return labels


def view_batch(labels: "np.ndarray", batch: int, seed: int, iter: int) -> "np.ndarray":
    """One camera per cluster for LM iteration `iter` (int32 [batch])."""
    import numpy as np
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    ids = np.zeros(int(batch), np.int32)
    _check(_lib.lmrs_view_batch(C.c_void_p(labels.ctypes.data), labels.size, int(batch), int(seed), int(iter),
                                C.c_void_p(ids.ctypes.data)), "lmrs_view_batch")
    return ids


def lm_params(iter: int, cg_iters: int, lam: float, seed: int = 0, eta_cap: float = 0.2,
              eta_warm: float = 0.05, warm_iters: int = 10, sampler: int = SAMPLER_UNIFORM,
              cg_iters_late: int = 0, late_iter: int = 0, ssim_weight: float = 0.0) -> LmParams:
    return LmParams(int(iter), int(cg_iters), float(lam), float(eta_cap), float(eta_warm), int(warm_iters),
                    int(seed), int(sampler), int(cg_iters_late), int(late_iter), float(ssim_weight))


EXPORTS = ("lmrs_status_str", "lmrs_last_error", "lmrs_report_status", "lmrs_workspace_bytes", "lmrs_project",
           "lmrs_bin_tiles", "lmrs_render", "lmrs_jvp", "lmrs_vjp", "lmrs_gn_product",
           "lmrs_gn_product_timed", "lmrs_gn_product_noalloc", "lmrs_walk_counts", "lmrs_linearize",
           "lmrs_gn_diag", "lmrs_pcg", "lmrs_lm_step",
           "lmrs_residual_scores", "lmrs_contributor_counts", "lmrs_sample", "lmrs_lm_solve",
           "lmrs_view_clusters", "lmrs_view_batch", "lmrs_lm_iterate", "lmrs_bin_tiles_async",
           "lmrs_ssim_residual")
