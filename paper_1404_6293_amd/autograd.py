"""Differentiable rendering on top of the binned rasterizer.

``RasterizeFn`` wraps one frame (forward: pk_setup, pk_assign_bin,
pk_raster_shade with the barycentric buffer saved; backward: pk_backward)
in a ``torch.autograd.Function``.  Gradients flow to the per-vertex colours
and, for textured shading, to the texels.  Coverage is not differentiated:
positions, UVs and matrices receive no gradient.
"""
from __future__ import annotations

from types import SimpleNamespace
from typing import Optional

import torch

from . import pk


class RasterizeFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vcolor, texture, pos, idx, uv, mvp, width, height, num_views, bin_size,
                schedule):
        shading = "textured" if texture is not None else "gouraud"
        sc = SimpleNamespace(width=width, height=height, pos=pos, color=vcolor, idx=idx,
                             num_tris=int(idx.shape[0]) if idx is not None else pos.shape[1] // 3,
                             mvp=mvp, num_scenes=num_views, scene_tri_off=None,
                             scene_vtx_off=None, instanced=num_views > 1, uv=uv,
                             normal=None, texture=texture, lights=None, shading=shading)
        r = pk.Renderer(pk.DeviceScene(sc, device=str(vcolor.device)),
                        pk.RenderConfig(bin_size=bin_size, schedule=schedule, want_bary=True))
        out = r.render()
        ctx.renderer = r
        ctx.textured = texture is not None
        ctx.mark_non_differentiable(out["primid"], out["depth"])
        return out["color"], out["depth"], out["primid"]

    @staticmethod
    def backward(ctx, grad_color, grad_depth, grad_primid):
        r = ctx.renderer
        d = r.dev
        gv = torch.zeros((3, d.num_vertices), dtype=torch.float32, device=d.device)
        gt = torch.zeros_like(d.texture) if ctx.textured else None
        r.backward(grad_color.contiguous().to(torch.float32), gv, gt)
        ctx.renderer = None
        return (gv, gt) + (None,) * 9


def rasterize(vcolor: torch.Tensor, pos: torch.Tensor, idx: Optional[torch.Tensor], *,
              width: int, height: int, mvp: Optional[torch.Tensor] = None,
              uv: Optional[torch.Tensor] = None, texture: Optional[torch.Tensor] = None,
              num_views: int = 1, bin_size: int = 16, schedule: str = "direct_map"):
    """Render ``num_views`` views (one MVP each) of a mesh.

    vcolor [3][V], pos [3][V] float32 SoA planes; idx [T][3] int32 or None;
    mvp [num_views][16]; uv [2][V] and texture [th][tw][3] for textured
    shading.  Returns (color [S][H][W][4], depth [S][H][W], primid [S][H][W]);
    color is differentiable with respect to vcolor and texture.
    """
    return RasterizeFn.apply(vcolor, texture, pos, idx, uv, mvp, width, height, num_views,
                             bin_size, schedule)
