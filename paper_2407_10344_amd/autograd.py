"""``torch.autograd.Function`` over the device VGICP error with a hand-written backward.

Forward: e_f = e(T0_f Exp(xi_f); points) for every factor f of a batch, with
correspondences and W = (C~ + R C R^T)^-1 recomputed at the evaluated pose
(GLIM Sec. III-C, Eq. (em), Eq. (d2d)).  Backward (a device kernel): the exact
gradient of that error with the correspondences held fixed,
    de/dxi' = 2 sum [w x (mu + C w); -w],  de/dmu_k = -2 sum_l w,  w = R^T W d,
chained through the SE(3) right Jacobian, de/dxi = J_r(xi)^T de/dxi'.
"""

from __future__ import annotations

import torch

from .vgicp import FactorBatch


def _set_points(batch: FactorBatch, points: torch.Tensor):
    seen = set()
    for s in batch.sources:
        if id(s) in seen:
            continue
        seen.add(id(s))
        row0, n = batch.source_rows[id(s)]
        s.set_points(points[row0:row0 + n])


class VGICPCost(torch.autograd.Function):
    """e = VGICPCost.apply(xi, points, batch, T0).

    xi:     (F, 6) float64 device tensor, tangent [omega; v] applied on the right of T0.
    points: (R, 3) float32/float64 device tensor, the positions of the batch's distinct
            sources concatenated in order of first use (R = batch.grad_rows).
    batch:  a FactorBatch.
    T0:     (F, 12) float64 device tensor of base poses (not differentiated).
    """

    @staticmethod
    def forward(ctx, xi, points, batch: FactorBatch, T0):
        points = points.contiguous()
        _set_points(batch, points)
        T, jr = batch.ctx.se3_retract(T0, xi, jacobian=True)
        e = batch.evaluate_async(T)
        ctx.batch = batch
        ctx.save_for_backward(T, jr, points)
        return e

    @staticmethod
    def backward(ctx, grad_e):
        T, jr, points = ctx.saved_tensors
        batch = ctx.batch
        _set_points(batch, points)
        want_pts = ctx.needs_input_grad[1]
        gxi, gp = batch.backward_async(T, grad_e, jr=jr, points_dtype=points.dtype if want_pts else None)
        return (gxi if ctx.needs_input_grad[0] else None), gp, None, None
