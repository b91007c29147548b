"""Receiver traces as a differentiable function of the medium and the source
amplitudes: the forward runs the fused step with checkpoints, the backward
runs the library's discrete adjoint (lbm_adjoint_step) on the incoming trace
gradient. Only argument marshalling happens here."""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from .solver import Solver


class ShotTraces(torch.autograd.Function):
    """traces[g] of shot g (all shots through one medium of shape (ny, nx)),
    differentiable with respect to lambda, mu (per cell) and amp[g], the
    amplitude of shot g's first source."""

    @staticmethod
    def forward(ctx, lam, mu, amp, problems, nsteps, seg_steps, dtype, launch):
        shots = []
        amps = amp.detach().double().cpu().tolist()
        for p, a in zip(problems, amps):
            src = list(p.sources)
            if not src:
                raise ValueError("every shot needs a source")
            q = src[0]
            src[0] = type(q)(q.x, q.y, q.sigma, q.dir_x, q.dir_y, float(a), q.period, q.t0)
            shots.append(p.replace(sources=src))
        _, _, rho = problems[0].medium.full(problems[0].ny, problems[0].nx)
        s = Solver(shots, dtype=dtype, device=lam.device, trace_steps=nsteps, launch=launch,
                   fields=(lam.detach(), mu.detach(), torch.as_tensor(rho)))
        s.adjoint_begin(nsteps, seg_steps)
        s.step(nsteps)
        ctx.solver = s
        ctx.nsteps = nsteps
        ctx.dtypes = (lam.dtype, mu.dtype, amp.dtype)
        return torch.stack([t for t in s.traces])

    @staticmethod
    def backward(ctx, grad_traces):
        s = ctx.solver
        n = len(s.problems)
        p0 = s.problems[0]
        dev = s.device
        gk = torch.zeros((n, p0.ny, p0.nx), dtype=torch.float64, device=dev)
        nsrc = max(len(p.sources) for p in s.problems)
        ga = torch.zeros((n, max(nsrc, 1)), dtype=torch.float64, device=dev)
        res = grad_traces.to(dtype=s.tdtype).contiguous()
        for g in range(n):
            s.adjoint_set_io(g, res[g], gk[g], ga[g])
        s.adjoint_step(ctx.nsteps)
        gl = torch.zeros((p0.ny, p0.nx), dtype=torch.float64, device=dev)
        gm = torch.zeros_like(gl)
        for g in range(n):
            s.lame_gradient(g, gk[g], gl, gm)
        torch.cuda.synchronize(dev)
        s.close()
        ctx.solver = None
        lt, mt, at = ctx.dtypes
        return gl.to(lt), gm.to(mt), ga[:, 0].to(at), None, None, None, None, None


def shot_traces(lam: torch.Tensor, mu: torch.Tensor, amp: torch.Tensor, problems: Sequence,
                nsteps: int, seg_steps: int = 100, dtype: str = "f32",
                launch: Optional[dict] = None) -> torch.Tensor:
    """Traces (nshots, nsteps, nrec, ncomp) of shots sharing the medium
    (lam, mu) with per-shot source amplitudes amp; differentiable."""
    return ShotTraces.apply(lam, mu, amp, list(problems), int(nsteps), int(seg_steps), dtype,
                            launch)
