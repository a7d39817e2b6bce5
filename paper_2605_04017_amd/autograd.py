"""torch.autograd.Function over the map's hand-written forward/backward.

Forward: lt_map_forward_train (BF16 MFMA, activations kept in a workspace);
backward: lt_map_backward.  The parameter tensor is the differentiable input;
its values are loaded into the map before the forward pass.
"""
from __future__ import annotations

import torch

from . import (Map, RAY_FIELDS, lt_map_backward, lt_map_forward_train, lt_map_set_params,
               workspace)


class MapFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, x, y, dx, dy, dz, lambda_nm, m: Map):
        n = int(x.numel())
        rays = dict(zip(RAY_FIELDS, (x, y, dx, dy, dz, lambda_nm)))
        lt_map_set_params(m, params.detach().contiguous())
        ws = workspace(m, n, x.device)
        o, ws = lt_map_forward_train(m, rays, ws=ws, n=n)
        ctx.m, ctx.ws, ctx.n = m, ws, n
        return o

    @staticmethod
    def backward(ctx, grad_o):
        g = lt_map_backward(ctx.m, grad_o.contiguous(), ctx.ws, n=ctx.n)
        return (g,) + (None,) * 7


def map_forward(params: torch.Tensor, rays: dict, m: Map) -> torch.Tensor:
    """Raw map outputs (6 * n_heads, n) as a differentiable function of params."""
    return MapFunction.apply(params, *(rays[k] for k in RAY_FIELDS), m)
