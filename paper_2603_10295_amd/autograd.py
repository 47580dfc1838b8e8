"""torch.autograd binding of the weighted-|g|^2 loss and its hand-written adjoint.

    L = eph_loss(system, g, k, q, kq_index, seed)

computes L = sum w_{mn nu}(k,q) |g_{mn nu}(k,q)|^2 over every (k, q) pair with
the library's forward kernels; L.backward() runs ephw_loss_backward, which
recomputes the forward in (q batch, k tile) units and returns dL/dg(Re,Rp),
dL/dk and dL/dq.  k+q must lie on the k grid (kq_index); dL/dk is the
derivative at the given points with V(k+q) taken at the indexed grid point.
Complex gradients follow torch's convention (dL/dRe + i dL/dIm).
"""
from __future__ import annotations

import torch

from . import ephw


class EphLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, g, k, q, system, kq_index, seed, prec):
        system.set_g(g.detach().contiguous())
        ks = ephw.KSet(system, k.detach().contiguous(), prec)
        loss = torch.zeros(1, dtype=torch.float64, device=g.device)
        ephw.interpolate(ks, q.detach().contiguous(), kq_index=kq_index, flags=ephw.OUT_LOSS, loss=loss,
                         loss_seed=seed)
        ks.close()
        ctx.system, ctx.kq_index, ctx.seed, ctx.prec = system, kq_index, seed, prec
        ctx.save_for_backward(g, k, q)
        return loss[0]

    @staticmethod
    def backward(ctx, grad_out):
        g, k, q = ctx.saved_tensors
        system = ctx.system
        system.set_g(g.detach().contiguous())
        ks = ephw.KSet(system, k.detach().contiguous(), ctx.prec)
        dg = torch.zeros_like(g) if ctx.needs_input_grad[0] else None
        dk = torch.zeros(k.shape, dtype=torch.float64, device=k.device) if ctx.needs_input_grad[1] else None
        dq = torch.zeros(q.shape, dtype=torch.float64, device=q.device) if ctx.needs_input_grad[2] else None
        ephw.loss_backward(ks, q.detach().contiguous(), ctx.kq_index, loss_seed=ctx.seed, dL_dg=dg, dL_dk=dk,
                           dL_dq=dq)
        ks.close()
        scale = grad_out.to(torch.float64)
        out_g = None if dg is None else dg * scale.to(dg.real.dtype)
        out_k = None if dk is None else dk * scale
        out_q = None if dq is None else dq * scale
        return out_g, out_k, out_q, None, None, None, None


def eph_loss(system: "ephw.System", g: torch.Tensor, k: torch.Tensor, q: torch.Tensor, kq_index: torch.Tensor,
             seed: int = 0) -> torch.Tensor:
    prec = ephw.FP64 if g.dtype == torch.complex128 else ephw.FP32
    return EphLoss.apply(g, k, q, system, kq_index, int(seed), prec)
