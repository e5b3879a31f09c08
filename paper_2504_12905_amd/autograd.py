"""PyTorch autograd adapter over the HIP render (argument marshalling only).

`LmrsRender.apply(beta, views)` renders every pixel of the views with
lmrs_project / lmrs_bin_tiles / lmrs_render and returns images [V, H, W, 3].
Its backward is the library's hand-written reverse pass (lmrs_vjp) and its
forward-mode rule is the dual-number tangent pass (lmrs_jvp), so both
`torch.autograd.grad` and `torch.autograd.forward_ad` run the HIP kernels.
The discrete decisions of the forward render (tile lists, skips, last
blended entry) are kept and reused by both derivative passes: the
derivative is that of the render with those decisions held fixed.

`render(means, log_scales, quats, opacity_logits, sh, views)` packs per-group
parameter tensors ([n,3], [n,3], [n,4] as w,x,y,z, [n], [n,K,3]) into the
component-major parameter vector of the library and renders them.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import lmrs as L


@dataclass
class Views:
    """Cameras to render: float32 [V_total, 16] rows (R, t, fx, fy, cx, cy),
    the selected camera indices and the common image size."""
    cams: torch.Tensor
    width: int
    height: int
    view_ids: torch.Tensor | None = None   # int32 [V]; None = all cameras
    opts: object = None

    @property
    def n_views(self) -> int:
        return int(self.cams.shape[0] if self.view_ids is None else self.view_ids.numel())


def _image_index(frame: L.Frame, device) -> torch.Tensor:
    """Flat image index (v*H*W + y*W + x) of every sample in the library's
    tile-major order (all 256 pixels per tile)."""
    T, TX = frame.T, frame.TX
    t = torch.arange(T, device=device)
    p = torch.arange(256, device=device)
    y = ((t // TX) * 16)[:, None] + (p // 16)[None, :]
    x = ((t % TX) * 16)[:, None] + (p % 16)[None, :]
    pix = (y * frame.width + x).reshape(-1)
    v = torch.arange(frame.n_views, device=device)[:, None] * (frame.width * frame.height)
    return (v + pix[None, :]).reshape(-1)


class LmrsRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, beta: torch.Tensor, n: int, sh_degree: int, views: Views):
        b = beta.detach().contiguous()
        fr = L.Frame(n, sh_degree, b, views.cams, views.width, views.height, views.n_views,
                     view_ids=views.view_ids, k=256, blend=False)
        opts = views.opts or L.default_opts()
        L.lmrs_project(fr, opts)
        L.lmrs_bin_tiles(fr)
        L.lmrs_render(fr, opts)
        idx = _image_index(fr, b.device)
        img = torch.empty((views.n_views * views.height * views.width, 3), dtype=torch.float32, device=b.device)
        img[idx] = fr.color
        ctx.frame, ctx.idx, ctx.opts = fr, idx, opts
        return img.view(views.n_views, views.height, views.width, 3)

    @staticmethod
    def backward(ctx, grad_img: torch.Tensor):
        fr, idx = ctx.frame, ctx.idx
        u = grad_img.contiguous().view(-1, 3)[idx].contiguous()
        g = L.lmrs_vjp(fr, u, opts=ctx.opts)
        return g, None, None, None

    @staticmethod
    def jvp(ctx, beta_t: torch.Tensor, *_):
        fr, idx = ctx.frame, ctx.idx
        jp = L.lmrs_jvp(fr, beta_t.contiguous(), opts=ctx.opts)
        out = torch.empty((fr.n_views * fr.height * fr.width, 3), dtype=torch.float32, device=jp.device)
        out[idx] = jp
        return out.view(fr.n_views, fr.height, fr.width, 3)


def pack(means, log_scales, quats, opacity_logits, sh) -> torch.Tensor:
    """Component-major parameter vector from per-group tensors (differentiable)."""
    n = means.shape[0]
    K = sh.shape[1]
    parts = [means.t().reshape(-1), log_scales.t().reshape(-1), quats.t().reshape(-1),
             opacity_logits.reshape(-1), sh.reshape(n, K * 3).t().reshape(-1)]
    return torch.cat(parts).contiguous()


def render(means, log_scales, quats, opacity_logits, sh, views: Views) -> torch.Tensor:
    n, K = means.shape[0], sh.shape[1]
    deg = {1: 0, 4: 1, 9: 2, 16: 3}[K]
    return LmrsRender.apply(pack(means, log_scales, quats, opacity_logits, sh), n, deg, views)
