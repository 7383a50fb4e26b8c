"""Q/Tw maps as a differentiable torch operation.

QTwMap.apply(B, grid, target, params, segment) returns the q2d map of a seed plane,
or the q3d map of a voxel grid (Q, Tw, backward and forward end points, status), of
the all-FP64 form (or of the F32X form, if params ask for it), traced once with the
checkpoints of its derivative kept (fastqsl_q2d_record, fastqsl_q3d_record); its
backward runs the hand-written adjoint of the tracer and the Q stencil on them
(fastqsl_backward_recorded, fastqsl_q3d_backward_recorded) and returns dL/dB. Composed with a field model written in torch (for instance point
charges -> node values), autograd then yields the gradient with respect to the
model's parameters, so the model can be fitted to target maps.
"""

from __future__ import annotations

import torch

from . import (FQ_PREC_F64, ST_NOTAPE, Params, _is_voxels, backward_recorded, q2d_record,
               q3d_backward_recorded, q3d_record)


class QTwMap(torch.autograd.Function):
    @staticmethod
    def forward(ctx, B, grid, plane, params=None, segment: int = 32):
        params = params or Params(precision=FQ_PREC_F64)
        vox = _is_voxels(plane)
        rec = q3d_record if vox else q2d_record
        r = rec(B.detach(), grid, plane, params, segment, want_lines=True)
        shape = tuple(int(n) for n in reversed(plane.n)) if vox else (plane.nv, plane.nu)
        ctx.reverse = q3d_backward_recorded if vox else backward_recorded
        eb = r["lines"]["end_b"].view(*shape, 3)
        ef = r["lines"]["end_f"].view(*shape, 3)
        ctx.save_for_backward(B)
        ctx.grid, ctx.plane, ctx.params, ctx.segment = grid, plane, params, segment
        ctx.rec = r  # the workspace with the checkpoints, read by the backward pass
        st = r["status"]
        if bool(((st.to(torch.int32) & ST_NOTAPE) != 0).any()):
            raise RuntimeError("the adjoint's checkpoint pool ran out: raise params.tape_steps "
                               "(accepted steps per half line the pool holds on average)")
        ctx.mark_non_differentiable(st)
        return r["q"], r["tw"], eb, ef, st

    @staticmethod
    def backward(ctx, gq, gtw, geb, gef, _gst):
        (B,) = ctx.saved_tensors
        gb = ctx.reverse(B.detach(), ctx.grid, ctx.plane, ctx.rec, ctx.params, ctx.segment,
                               dq=None if gq is None else gq.reshape(-1),
                               dtw=None if gtw is None else gtw.reshape(-1),
                               dend_b=None if geb is None else geb.reshape(-1, 3),
                               dend_f=None if gef is None else gef.reshape(-1, 3))
        return gb.to(B.dtype), None, None, None, None


def qtw_map(B, grid, plane, params=None, segment: int = 32):
    """(Q, Tw, end_b, end_f, status) of the q2d map of a plane, or the q3d map of a
    voxel grid, differentiable in B."""
    return QTwMap.apply(B, grid, plane, params, segment)
