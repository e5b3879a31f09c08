"""FP64 CPU oracle for the LM-RS hot path: test infrastructure only.

Plain, slow and obviously correct. Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path (the HIP
library and its binding) never does, and the two share no code.

C++ part (``lmrs_oracle.cpp``): projection, tile lists, render, J p by dual
numbers, J^T u by reverse accumulation, the Gauss-Newton product and the exact
diagonal. Python part: the Philox counter RNG and the uniform stratified
sampler (``sampling.py``), and the PCG / LM step in the order of Alg. 1
(``solver.py``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, build

_lib = None

# Rasteriser options: alpha floor and cap, transmittance stop, EWA low-pass
# (px^2), near plane, footprint extent in sigmas, background RGB. The options
# block of the problem statement holds FP32 numbers, so each value is the
# FP32 number nearest the decimal one (0.3 is 0.30000001192092896), on the
# FP64 side as well: both sides then decide with the same thresholds.
def _f32(x: float) -> float:
    return float(np.float32(x))


DEFAULT_OPTS = dict(alpha_min=_f32(1.0 / 255.0), alpha_max=_f32(0.99), t_min=_f32(1e-4), lowpass=_f32(0.3),
                    znear=_f32(0.2), cutoff=3.0, bg=(0.0, 0.0, 0.0))

# Bound on how far two FP64 evaluations of a list decision (footprint radius
# extent, rectangle edge, near-plane depth) may disagree, in pixels / depth
# units: the extents are below 1e4 px and FP64 carries 16 digits.
TAU_LIST = 1e-9


def opts_array(opts: dict | None = None) -> np.ndarray:
    o = dict(DEFAULT_OPTS)
    if opts:
        o.update(opts)
    vals = [o["alpha_min"], o["alpha_max"], o["t_min"], o["lowpass"], o["znear"], o["cutoff"], *o["bg"]]
    return np.array([_f32(x) for x in vals], dtype=np.float64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        vp, i32, i64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_double
        L.or_create.restype = vp
        L.or_create.argtypes = [i32, i32, vp, i32, vp, i32, i32, vp, vp]
        L.or_destroy.argtypes = [vp]
        L.or_num_instances.restype = i64
        L.or_num_instances.argtypes = [vp]
        L.or_get_projection.argtypes = [vp] * 8
        L.or_get_lists.argtypes = [vp, vp, vp]
        L.or_undecided_tiles.argtypes = [vp, dbl, vp]
        L.or_set_samples.argtypes = [vp, i32, vp, vp]
        L.or_set_tile_mask.argtypes = [vp, vp]
        L.or_set_channel_weights.argtypes = [vp, vp]
        L.or_render.argtypes = [vp] * 7
        L.or_jvp.argtypes = [vp, vp, vp]
        L.or_vjp.argtypes = [vp, vp, vp]
        L.or_vjp_screen.argtypes = [vp, vp, vp]
        L.or_vjp_abs.argtypes = [vp, vp, vp]
        L.or_gn.argtypes = [vp, vp, dbl, vp, vp]
        L.or_diag.argtypes = [vp, vp]
        L.or_proj_jacobian.argtypes = [vp, i32, i32, vp]
        L.or_sh_basis.argtypes = [i32, dbl, dbl, dbl, vp]
        L.or_num_threads.restype = i32
        L.or_set_num_threads.argtypes = [i32]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


class Oracle:
    """FP64 evaluation of one view batch at one parameter vector.

    beta: [P] (kept in FP64; FP32 inputs convert exactly); cams: float32 [V, 16];
    width/height multiples of 16.
    The tile lists are built on construction.
    """

    def __init__(self, n: int, sh_degree: int, beta: np.ndarray, cams: np.ndarray, width: int,
                 height: int, opts: dict | None = None, only_tiles: np.ndarray | None = None):
        self.n, self.deg = int(n), int(sh_degree)
        self.K = (self.deg + 1) ** 2
        self.Pg = 11 + 3 * self.K
        self.P = self.n * self.Pg
        self.V = int(cams.shape[0])
        self.W, self.H = int(width), int(height)
        self.TX, self.TY = self.W // 16, self.H // 16
        self.T = self.TX * self.TY
        self._beta = np.ascontiguousarray(beta, dtype=np.float64)
        assert self._beta.size == self.P
        self._cams = np.ascontiguousarray(cams, dtype=np.float32)
        self._opts = opts_array(opts)
        # only_tiles (uint8 [V*T]): build the lists of these tiles only (the
        # others stay empty); renders and derivatives are then valid there only
        self._only = None if only_tiles is None else np.ascontiguousarray(only_tiles, dtype=np.uint8).reshape(-1)
        if self._only is not None:
            assert self._only.size == self.V * (self.W // 16) * (self.H // 16)
        self.h = lib().or_create(self.n, self.deg, _p(self._beta), self.V, _p(self._cams), self.W,
                                 self.H, _p(self._opts), _p(self._only))
        if not self.h:
            raise ValueError("oracle: bad problem description")
        self.k = 256
        self.pix = None
        self.w = None

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_destroy(self.h)
            self.h = None

    # ------------------------------------------------------------ geometry
    def projection(self):
        VN = self.V * self.n
        rec = np.zeros((self.V, self.n, 9))
        depth = np.zeros((self.V, self.n))
        rect = np.zeros((self.V, self.n, 4), np.int32)
        radius = np.zeros((self.V, self.n), np.int32)
        margin = np.zeros((self.V, self.n))
        margin_rad = np.zeros((self.V, self.n))
        vis = np.zeros((self.V, self.n), np.uint8)
        lib().or_get_projection(self.h, _p(rec), _p(depth), _p(rect), _p(radius), _p(margin), _p(vis),
                                _p(margin_rad))
        assert rec.size == VN * 9
        # depth: FP64 camera z (the sort key); margin: distance of the closest list
        # decision to its threshold (radius extent to an integer, rectangle edge
        # to a tile edge, depth to the near plane), margin_rad: the radius part
        return dict(rec=rec, depth=depth, rect=rect, radius=radius, margin=margin, margin_rad=margin_rad,
                    visible=vis)

    def lists(self):
        ni = lib().or_num_instances(self.h)
        ts = np.zeros(self.V * self.T + 1, np.int64)
        ids = np.zeros(max(ni, 1), np.int32)
        lib().or_get_lists(self.h, _p(ts), _p(ids))
        return ts, ids[:ni]

    # ------------------------------------------------------------- samples
    def set_samples(self, k: int = 256, pix: np.ndarray | None = None, w: np.ndarray | None = None):
        self.k = int(k)
        self.pix = None if pix is None else np.ascontiguousarray(pix, dtype=np.uint8).reshape(-1)
        self.w = None if w is None else np.ascontiguousarray(w, dtype=np.float32).reshape(-1)
        if self.pix is not None:
            assert self.pix.size == self.V * self.T * self.k
        if self.w is not None:
            assert self.w.size == self.V * self.T * self.k
        lib().or_set_samples(self.h, self.k, _p(self.pix), _p(self.w))
        self._wc = None

    def set_channel_weights(self, wc: np.ndarray | None):
        """Per-channel weights [S, 3] of the GN operator (None: the sample weights)."""
        self._wc = None if wc is None else np.ascontiguousarray(wc, dtype=np.float64).reshape(-1)
        if self._wc is not None:
            assert self._wc.size == 3 * self.S
        lib().or_set_channel_weights(self.h, _p(self._wc))

    def set_tile_mask(self, mask: np.ndarray | None):
        self._mask = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
        lib().or_set_tile_mask(self.h, _p(self._mask))

    @property
    def S(self) -> int:
        return self.V * self.T * self.k

    def weights(self) -> np.ndarray:
        return np.ones(self.S) if self.w is None else self.w.astype(np.float64)

    def pixel_coords(self) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
        """(view, x, y) of every sampled pixel in sample order."""
        V, T, k = self.V, self.T, self.k
        v = np.repeat(np.arange(V), T * k)
        t = np.tile(np.repeat(np.arange(T), k), V)
        p = np.tile(np.arange(256), V * T) if self.pix is None else self.pix.astype(np.int64)
        x = (t % self.TX) * 16 + p % 16
        y = (t // self.TX) * 16 + p // 16
        return v, x, y

    # ------------------------------------------------------------- render
    def render(self):
        S = self.S
        Cc = np.zeros((S, 3))
        T = np.zeros(S)
        last = np.zeros(S, np.int32)
        nc = np.zeros(S, np.int32)
        tr = np.zeros(S, np.uint64)
        mg = np.zeros(S)
        lib().or_render(self.h, _p(Cc), _p(T), _p(last), _p(nc), _p(tr), _p(mg))
        return dict(C=Cc, T=T, last=last, n_contrib=nc, trace=tr, margin=mg)

    def undecided_tiles(self, tau: float = TAU_LIST) -> np.ndarray:
        """uint8 [V*T]: tiles whose list could hold one Gaussian more or less
        under a less exact evaluation of a footprint radius (its extent within
        tau px of an integer: the tiles held with only one of the two radii;
        see or_undecided_tiles)."""
        flags = np.zeros(self.V * self.T, np.uint8)
        lib().or_undecided_tiles(self.h, float(tau), _p(flags))
        return flags

    def decided(self, tau: float = 1e-4, tau_list: float = TAU_LIST) -> np.ndarray:
        """Sampled pixels whose blend decisions (exponent sign, alpha floor and
        cap, transmittance stop) all lie farther than tau (relative) from their
        thresholds, in tiles whose lists no radius within tau_list px of an
        integer could change. The blend decisions are taken in FP32 on the GPU
        and in FP64 here, so below tau they may differ, and the pixel's colour
        and derivative are then not unique at FP32 precision. List decisions
        are FP64 on both sides (tau_list bounds the disagreement of two FP64
        evaluations)."""
        ok = self.render()["margin"] >= tau
        tile = np.arange(self.S) // self.k
        return ok & (self.undecided_tiles(tau_list)[tile] == 0)

    def render_image(self) -> np.ndarray:
        """Full images [V, H, W, 3] (uses all pixels; resets the sample set)."""
        self.set_samples(256)
        out = self.render()["C"]
        v, x, y = self.pixel_coords()
        img = np.zeros((self.V, self.H, self.W, 3))
        img[v, y, x] = out
        return img

    # --------------------------------------------------------- derivatives
    def jvp(self, p: np.ndarray) -> np.ndarray:
        p = np.ascontiguousarray(p, dtype=np.float64)
        assert p.size == self.P
        out = np.zeros((self.S, 3))
        lib().or_jvp(self.h, _p(p), _p(out))
        return out

    def vjp(self, u: np.ndarray) -> np.ndarray:
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.S, 3)
        out = np.zeros(self.P)
        lib().or_vjp(self.h, _p(u), _p(out))
        return out

    def vjp_abs(self, u: np.ndarray) -> np.ndarray:
        """Entry-wise magnitude of the terms J^T u is summed from: the
        reverse pass with every quantity replaced by the sum of the magnitudes
        of its terms (the colour behind, d/d alpha = T u.rgb - behind/(1-alpha)
        as T|u.rgb| + |behind|/(1-alpha), ...), then the chain with
        |d rec / d beta|. It bounds |J^T u| and |J|^T |u| from above and equals
        them where no term can cancel; tests divide entry-wise differences by
        it (a scale for rounding, not part of the method)."""
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.S, 3)
        out = np.zeros(self.P)
        lib().or_vjp_abs(self.h, _p(u), _p(out))
        return out

    def vjp_screen(self, u: np.ndarray) -> np.ndarray:
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.S, 3)
        out = np.zeros((self.V, self.n, 9))
        lib().or_vjp_screen(self.h, _p(u), _p(out))
        return out

    def gn(self, p: np.ndarray, lam: float, d: np.ndarray | None = None) -> np.ndarray:
        p = np.ascontiguousarray(p, dtype=np.float64)
        d = None if d is None else np.ascontiguousarray(d, dtype=np.float64)
        out = np.zeros(self.P)
        lib().or_gn(self.h, _p(p), float(lam), _p(d), _p(out))
        return out

    def diag(self) -> np.ndarray:
        out = np.zeros(self.P)
        lib().or_diag(self.h, _p(out))
        return out

    def proj_jacobian(self, v: int, g: int) -> np.ndarray:
        J = np.zeros((9, self.Pg))
        lib().or_proj_jacobian(self.h, int(v), int(g), _p(J))
        return J

    def dense_jacobian(self) -> np.ndarray:
        """Dense J [3S, P] column by column with dual numbers (tiny problems only)."""
        assert self.P <= 4000 and self.S <= 20000
        J = np.zeros((3 * self.S, self.P))
        e = np.zeros(self.P)
        for j in range(self.P):
            e[j] = 1.0
            J[:, j] = self.jvp(e).reshape(-1)
            e[j] = 0.0
        return J


def sh_basis(deg: int, d: np.ndarray) -> np.ndarray:
    d = np.asarray(d, dtype=np.float64)
    Y = np.zeros(16)
    lib().or_sh_basis(int(deg), float(d[0]), float(d[1]), float(d[2]), _p(Y))
    return Y[: (deg + 1) ** 2]


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_num_threads(t: int) -> None:
    """Threads of the oracle's OpenMP regions from now on (this thread)."""
    lib().or_set_num_threads(int(t))
