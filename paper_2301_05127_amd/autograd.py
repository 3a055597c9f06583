"""torch.autograd view of the solver: traces = F(m) for a model m, whose backward is the
hand-written discrete adjoint.  Acoustic: m = wave speed c or bulk modulus
K = rho c^2.  Elastic: m = (vp, vs) or the Lame parameters (lambda, mu).

The forward runs the checkpointed acoustic stepper (`loss_forward_ckpt`); the backward
injects the incoming trace gradient at the receivers and runs the adjoint sweep
(`loss_adjoint`), which returns the vector-Jacobian product sum_r g_r dtraces_r/dm.
Paper Sec. 2 (acoustic and elastic systems) and Sec. 3.3 (the Strang step that is
transposed).
"""
from __future__ import annotations

import torch

from . import loss


class _Seismograms(torch.autograd.Function):
    @staticmethod
    def forward(ctx, m, sim, rho, nsteps, ckpt_every, param):
        if not m.is_cuda:
            raise ValueError("the model must be a CUDA tensor")
        r = rho.to(device=m.device, dtype=torch.float32).contiguous()
        mf = m.detach().to(torch.float32)
        vp = mf if param == loss.GRAD_VP else torch.sqrt(mf / r)
        torch.cuda.current_stream(m.device).synchronize()
        sim.set_media(vp.contiguous(), r)
        sim.forward_ckpt(nsteps, ckpt_every)
        ctx.sim, ctx.param, ctx.dtype = sim, param, m.dtype
        return sim.traces_tensor(m.device)

    @staticmethod
    def backward(ctx, g):
        grad = ctx.sim.adjoint(g.detach().to(torch.float64).contiguous(), ctx.param)
        return grad.to(ctx.dtype), None, None, None, None, None


def seismograms(sim, m, rho, nsteps, ckpt_every=100, param=loss.GRAD_VP):
    """Traces [S][nrec][trace_len] (FP64, CUDA) of every shot of `sim` for the model `m`
    (a CUDA tensor of the field shape: c when param is GRAD_VP, K when GRAD_K); rho is
    held fixed.  Differentiable with respect to m through the discrete adjoint."""
    return _Seismograms.apply(m, sim, rho, int(nsteps), int(ckpt_every), int(param))


class _ElasticSeismograms(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a, b, sim, rho, nsteps, ckpt_every, param):
        if not (a.is_cuda and b.is_cuda):
            raise ValueError("the model must be CUDA tensors")
        r = rho.to(device=a.device, dtype=torch.float32).contiguous()
        af, bf = a.detach().to(torch.float32), b.detach().to(torch.float32)
        if param == loss.GRAD_VPVS:
            vp, vs = af, bf
        else:   # (lambda, mu)
            vp, vs = torch.sqrt((af + 2.0 * bf) / r), torch.sqrt(bf / r)
        torch.cuda.current_stream(a.device).synchronize()
        sim.set_media(vp.contiguous(), r, vs.contiguous())
        sim.forward_ckpt(nsteps, ckpt_every)
        # the density's gradient comes with the _RHO form of the parameterisation
        with_rho = ctx.needs_input_grad[3]
        ctx.sim, ctx.dtypes, ctx.with_rho = sim, (a.dtype, b.dtype, rho.dtype), with_rho
        ctx.param = param + 2 if with_rho else param
        return sim.traces_tensor(a.device)

    @staticmethod
    def backward(ctx, g):
        grad = ctx.sim.adjoint(g.detach().to(torch.float64).contiguous(), ctx.param)
        grho = grad[2].to(ctx.dtypes[2]) if ctx.with_rho else None
        return grad[0].to(ctx.dtypes[0]), grad[1].to(ctx.dtypes[1]), None, grho, None, None, None


def elastic_seismograms(sim, a, b, rho, nsteps, ckpt_every=20, param=loss.GRAD_VPVS):
    """Traces [S][nrec][trace_len] (FP64, CUDA) of every shot of the elastic `sim` for the
    model (a, b): (vp, vs) when param is GRAD_VPVS, (lambda, mu) when GRAD_LAME, CUDA
    tensors of the field shape, and the density rho.  Differentiable with respect to a
    and b, and to rho when it requires a gradient (with (a, b) held fixed), through the
    discrete adjoint."""
    if param not in (loss.GRAD_VPVS, loss.GRAD_LAME):
        raise ValueError("param must be GRAD_VPVS or GRAD_LAME")
    return _ElasticSeismograms.apply(a, b, sim, rho, int(nsteps), int(ckpt_every), int(param))
