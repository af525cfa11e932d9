"""Differentiable right Jacobian transformation of the MLCC3 triples terms.

`RightTransform` is a torch.autograd.Function: its forward is the library's right transform
rho = J(omega) R of the symmetrised trial vector; its backward is the library's left
(transpose) transform, mapped between elementwise gradients and the pairing of left and right
vectors by `mlcc3_vec_map`:

    grad_R = LEFT_TO_GRAD( sigma ),  sigma = left transform of GRAD_TO_LEFT( grad_rho ).

This is exact: the left transform is the adjoint of the right one under the pairing
G(L, R) = sum L1 R1 + sum_{(AI)>=(BJ)} L~ R (Implementation section: contravariant doubles),
GRAD_TO_LEFT turns an elementwise gradient into the vector that represents it under G, and
LEFT_TO_GRAD turns sigma back into an elementwise gradient over the two stored doubles blocks.
The forward symmetrises R first (mean over the stored positions of each amplitude), so the
elementwise gradient is well defined for any block pair, consistent or not.  omega and the
ground state are parameters (no gradient).  Every step runs in the library's kernels.
"""
from __future__ import annotations

import torch

from . import mlcc3


class RightTransform(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x1, x2_vVoo, x2_vvoO, ws, ground, omega, precision):
        R = {"x1": x1.detach().contiguous(), "x2_vVoo": x2_vVoo.detach().contiguous(),
             "x2_vvoO": x2_vvoO.detach().contiguous()}
        Rs = mlcc3.vec_map(ws, ground, mlcc3.MAP_SYMMETRIZE, [R])[0]
        rho = mlcc3.right_transform(ws, ground, [omega], [Rs], reuse_ground=True, precision=precision)[0]
        ctx.ws, ctx.ground, ctx.omega, ctx.precision = ws, ground, omega, precision
        return rho["x1"], rho["x2_vVoo"], rho["x2_vvoO"]

    @staticmethod
    def backward(ctx, g1, g2a, g2b):
        d = ctx.ground.dims
        dev = ctx.ws.device
        zero = mlcc3.empty_out(d, dev)
        g = {"x1": g1.contiguous() if g1 is not None else zero["x1"].zero_(),
             "x2_vVoo": g2a.contiguous() if g2a is not None else zero["x2_vVoo"].zero_(),
             "x2_vvoO": g2b.contiguous() if g2b is not None else zero["x2_vvoO"].zero_()}
        L = mlcc3.vec_map(ctx.ws, ctx.ground, mlcc3.MAP_GRAD_TO_LEFT, [g])[0]
        sig = mlcc3.left_transform(ctx.ws, ctx.ground, [ctx.omega], [L], reuse_ground=True,
                                   precision=ctx.precision)[0]
        h = mlcc3.vec_map(ctx.ws, ctx.ground, mlcc3.MAP_LEFT_TO_GRAD, [sig])[0]
        return h["x1"], h["x2_vVoo"], h["x2_vvoO"], None, None, None, None


def right_transform(ws, ground, omega, x1, x2_vVoo, x2_vvoO, precision="fp64"):
    """rho = J(omega) R as three differentiable device tensors (singles and the two doubles blocks)."""
    return RightTransform.apply(x1, x2_vVoo, x2_vvoO, ws, ground, float(omega), precision)
