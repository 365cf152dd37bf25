"""torch.autograd binding of the sweep and its hand-written adjoint.

`emergent_stokes(...)` returns the Stokes vectors of the upward rays on the top
plane, [nray_up][nfreq][ny][nx][4], as a differentiable function of the
line-centre transfer coefficients (kappa, propmat, emis).  Its backward pass is
porta_fs_adjoint: the reverse sweep with plane checkpointing, not torch's
autograd of a traced program.
"""
from __future__ import annotations

import torch

from . import porta


class PortaSweep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, kappa, propmat, emis, hg, i_bottom, w2, prec, checkpoint_stride, opts,
                keep_checkpoints, interp):
        ck = None
        if keep_checkpoints:
            n = porta.checkpoint_size(hg, prec, checkpoint_stride, opts)
            ck = torch.empty(max(n, 256), dtype=torch.uint8, device=kappa.device)
        _, itop = porta.fs_sweep(hg, kappa, propmat, emis, i_bottom, w2, prec=prec,
                                 interp=interp, want_jkq=False, opts=opts, checkpoints=ck,
                                 checkpoint_stride=checkpoint_stride if ck is not None else 0)
        ctx.save_for_backward(kappa, propmat, emis)
        ctx.cfg = (hg, i_bottom, w2, prec, checkpoint_stride, opts, ck, interp)
        return itop

    @staticmethod
    def backward(ctx, grad_itop):
        kappa, propmat, emis = ctx.saved_tensors
        hg, i_bottom, w2, prec, stride, opts, ck, interp = ctx.cfg
        seed = grad_itop.to(porta.dtype_of(prec)).contiguous()
        gk, gp, ge = porta.fs_adjoint(hg, kappa.detach(), propmat.detach(), emis.detach(),
                                      i_bottom, seed, w2, prec=prec, interp=interp,
                                      checkpoint_stride=stride, opts=opts, checkpoints=ck)
        ctx.cfg = None
        return gk, gp, ge, None, None, None, None, None, None, None, None


def emergent_stokes(hg, kappa, propmat, emis, i_bottom, w2=1.0, prec=porta.F32,
                    checkpoint_stride=8, opts=None, keep_checkpoints=False,
                    interp=porta.BILINEAR):
    """Differentiable I_top; kappa [N], propmat [6][N], emis [6][N] on the GPU in the sweep
    precision (float32 for F32, float64 for F64), M and P interpolated as `interp` says.
    keep_checkpoints=True makes the forward sweep keep the plane checkpoints for the
    backward pass (more memory between the two passes, one sweep of the upward rays less
    in backward)."""
    return PortaSweep.apply(kappa, propmat, emis, hg, float(i_bottom), float(w2), int(prec),
                            int(checkpoint_stride), opts, bool(keep_checkpoints), int(interp))
