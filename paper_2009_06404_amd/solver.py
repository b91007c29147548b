"""Solver: owns the torch tensors (workspace, Lame fields, traces) that the C
ABI borrows, and forwards every call to liblbm.so. No arithmetic of the scheme
happens here; every step of the path runs in the library's HIP kernels."""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L

_DT = {"f32": (L.LBM_F32, torch.float32), "f64": (L.LBM_F64, torch.float64)}


def _field_tensor(medium, ny: int, nx: int, tdtype, device) -> List[torch.Tensor]:
    rows = medium.rows(ny)
    out = []
    if rows is not None:
        for r in rows:
            t = torch.as_tensor(np.asarray(r, dtype=np.float64), dtype=tdtype, device=device)
            out.append(t[:, None].expand(ny, nx).contiguous())
    else:
        for a in medium.full(ny, nx):
            out.append(torch.as_tensor(a, dtype=tdtype, device=device))
    return out


class Solver:
    """One context for one problem or a batch of problems advanced together.

    ``problems`` are objects with the attributes of ``workloads.Problem``
    (nx, ny, bc, rigid_row, tau, medium, sponge_thick, profile(e), sources,
    receivers, comp_mask). All problems of a batch share dtype and tau.
    """

    def __init__(self, problems, dtype: Optional[str] = None, device: str = "cuda",
                 trace_steps: Optional[int] = None, launch: Optional[dict] = None,
                 autotune: bool = False, fields=None):
        if not isinstance(problems, (list, tuple)):
            problems = [problems]
        self.problems = list(problems)
        p0 = self.problems[0]
        self.dtype = dtype or p0.dtype
        self.code, self.tdtype = _DT[self.dtype]
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        taus = {float(p.tau) for p in self.problems}
        if len(taus) != 1:
            raise ValueError("all problems of a batch must share tau")
        self.tau = taus.pop()
        grids = [(p.nx, p.ny) for p in self.problems]
        lam, mu, rho = [], [], []
        for p in self.problems:
            if fields is not None:
                # (lam, mu, rho) tensors of shape (ny, nx), shared by every grid
                l, m, r = (torch.as_tensor(f).to(device=self.device, dtype=self.tdtype)
                           for f in fields)
                if tuple(l.shape) != (p.ny, p.nx):
                    raise ValueError("fields must have each grid's shape (ny, nx)")
            else:
                l, m, r = _field_tensor(p.medium, p.ny, p.nx, self.tdtype, self.device)
            lam.append(l.reshape(-1))
            mu.append(m.reshape(-1))
            rho.append(r.reshape(-1))
        self.lam = torch.cat(lam)
        self.mu = torch.cat(mu)
        self.rho = torch.cat(rho)
        self.cell_off = np.cumsum([0] + [p.nx * p.ny for p in self.problems])
        self.ws_bytes = L.lbm_workspace_bytes(grids, self.code)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        bcs = [(p.bc[0], p.bc[1], p.bc[2], p.bc[3], p.rigid_row) for p in self.problems]
        sponges = [(tuple(p.sponge_thick), tuple(p.profile(e) for e in range(4)))
                   for p in self.problems]
        self.ctx = L.lbm_init(grids, self.code, self.lam.data_ptr(), self.mu.data_ptr(),
                              self.rho.data_ptr(), self.tau, bcs, sponges,
                              self.workspace.data_ptr(), self.ws_bytes, self.stream.cuda_stream)
        self.traces: List[Optional[torch.Tensor]] = [None] * len(self.problems)
        for g, p in enumerate(self.problems):
            if p.sources:
                L.lbm_set_sources(self.ctx, g, [s.as_tuple() for s in p.sources])
            if p.nrec > 0:
                steps = trace_steps if trace_steps is not None else max(int(p.nsteps), 1)
                self.attach_receivers(g, p.receivers, p.comp_mask, steps)
        if launch is not None:
            self.set_launch(**launch)
        if autotune:
            self.autotune()

    # -- entry points -----------------------------------------------------
    def attach_receivers(self, g: int, xy, comp_mask: int, steps: int) -> torch.Tensor:
        xy = np.asarray(xy, dtype=np.int32).reshape(-1, 2)
        ncomp = (comp_mask & 1) + ((comp_mask >> 1) & 1)
        tr = torch.zeros((steps, xy.shape[0], ncomp), dtype=self.tdtype, device=self.device)
        L.lbm_set_receivers(self.ctx, g, xy, comp_mask, tr.data_ptr(), steps)
        self.traces[g] = tr
        return tr

    def step(self, n: int) -> None:
        L.lbm_step(self.ctx, n)

    def filter(self, sigma: float) -> None:
        """High-wavenumber filter of the current state (lbm_filter)."""
        L.lbm_filter(self.ctx, sigma)

    def step_timed(self, n: int) -> dict:
        """Advance n steps with per-kernel event timing (synchronous)."""
        return L.lbm_step_timed(self.ctx, n)

    def moments(self, g: int = 0) -> torch.Tensor:
        p = self.problems[g]
        out = torch.empty((6, p.ny, p.nx), dtype=self.tdtype, device=self.device)
        L.lbm_moments(self.ctx, g, out.data_ptr())
        return out

    def state(self, g: int = 0) -> torch.Tensor:
        p = self.problems[g]
        out = torch.empty((9, p.ny, p.nx), dtype=self.tdtype, device=self.device)
        L.lbm_get_state(self.ctx, g, out.data_ptr())
        return out

    def set_state(self, g: int, src: torch.Tensor, t: int) -> None:
        p = self.problems[g]
        src = src.to(device=self.device, dtype=self.tdtype).contiguous()
        if tuple(src.shape) != (9, p.ny, p.nx):
            raise ValueError("state must have shape (9, ny, nx)")
        self._keep = src
        L.lbm_set_state(self.ctx, g, src.data_ptr(), t)

    @property
    def time(self) -> int:
        return L.lbm_get_time(self.ctx)

    def check_finite(self) -> bool:
        return L.lbm_check_finite(self.ctx)

    def launch(self) -> dict:
        return L.lbm_get_launch(self.ctx)

    def set_launch(self, waves: int, rows: int, graph_chunk: int = 0, prefetch: int = 1,
                   split: int = 1, pair: int = 0, overlap: int = 1, fuse_rows: int = 0,
                   fuse_steps: int = 2, tri_waves: int = 0) -> None:
        L.lbm_set_launch(self.ctx, waves, rows, graph_chunk, prefetch, split, pair, overlap,
                         fuse_rows, fuse_steps, tri_waves)

    def autotune(self, steps: int = 5) -> dict:
        return L.lbm_autotune(self.ctx, steps)

    # -- adjoint ---------------------------------------------------------
    def adjoint_reserve(self, nsteps: int, seg_steps: int = 100, resident_steps: int = 0) -> int:
        """Allocate (or keep, when large enough) the adjoint workspace for a
        recording of nsteps steps; returns its byte count. A workspace kept
        across recordings spares each one a device allocation."""
        nbytes = L.lbm_adjoint_workspace_bytes_resident(self.ctx, seg_steps, nsteps,
                                                        resident_steps)
        ws = getattr(self, "adj_ws", None)
        if ws is None or ws.numel() < nbytes:
            self.adj_ws = None       # the previous workspace goes first
            self.adj_ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return nbytes

    def adjoint_begin(self, nsteps: int, seg_steps: int = 100, resident_steps: int = 0) -> None:
        """Record the next nsteps forward steps (checkpoints every seg_steps),
        keeping the densities of the last resident_steps steps (whole trailing
        segments) in HBM: those segments need no recompute."""
        nbytes = self.adjoint_reserve(nsteps, seg_steps, resident_steps)
        L.lbm_adjoint_begin(self.ctx, seg_steps, nsteps, self.adj_ws.data_ptr(), nbytes)
        self._adj_keep = {}

    def adjoint_set_io(self, g: int, residual: Optional[torch.Tensor] = None,
                       grad_kappa: Optional[torch.Tensor] = None,
                       grad_amp: Optional[torch.Tensor] = None) -> None:
        """Residual dL/dv (traces' layout and dtype) and the FP64 gradient
        buffers of grid g (accumulated into)."""
        ptrs = []
        for t, dt in ((residual, self.tdtype), (grad_kappa, torch.float64),
                      (grad_amp, torch.float64)):
            if t is None:
                ptrs.append(None)
                continue
            if t.dtype != dt or not t.is_contiguous() or t.device != self.device:
                raise ValueError("adjoint buffers must be contiguous device tensors of the "
                                 "expected dtype")
            ptrs.append(t.data_ptr())
        self._adj_keep[g] = (residual, grad_kappa, grad_amp)
        L.lbm_adjoint_set_io(self.ctx, g, *ptrs)

    def adjoint_step(self, n: int) -> None:
        L.lbm_adjoint_step(self.ctx, n)

    def adjoint_step_timed(self, n: int) -> dict:
        """n adjoint steps with per-kernel event timing (synchronous)."""
        return L.lbm_adjoint_step_timed(self.ctx, n)

    @property
    def adjoint_time(self) -> int:
        return L.lbm_adjoint_time(self.ctx)

    def adjoint_state(self, g: int = 0) -> torch.Tensor:
        p = self.problems[g]
        out = torch.empty((9, p.ny, p.nx), dtype=self.tdtype, device=self.device)
        L.lbm_adjoint_get_state(self.ctx, g, out.data_ptr())
        return out

    def set_adjoint_state(self, g: int, src: torch.Tensor) -> None:
        p = self.problems[g]
        src = src.to(device=self.device, dtype=self.tdtype).contiguous()
        if tuple(src.shape) != (9, p.ny, p.nx):
            raise ValueError("adjoint state must have shape (9, ny, nx)")
        self._keep = src
        L.lbm_adjoint_set_state(self.ctx, g, src.data_ptr())

    def misfit(self, g: int, d_obs: torch.Tensor, nrows: Optional[int] = None):
        """(misfit, residual) of grid g's first nrows trace rows against d_obs:
        residual = traces - d_obs, misfit = 1/2 sum residual^2 (FP64)."""
        tr = self.traces[g]
        n = tr.shape[0] if nrows is None else int(nrows)
        d = d_obs.to(device=self.device, dtype=self.tdtype).contiguous()
        if d.shape[1:] != tr.shape[1:] or d.shape[0] < n:
            raise ValueError("d_obs must have the traces' layout")
        res = torch.zeros_like(tr)
        mis = torch.zeros(1, dtype=torch.float64, device=self.device)
        L.lbm_misfit(self.ctx, g, d.data_ptr(), res.data_ptr(), n, mis.data_ptr())
        return mis, res

    def lame_gradient(self, g: int, grad_kappa: torch.Tensor, grad_lam: torch.Tensor,
                      grad_mu: torch.Tensor) -> None:
        """Add grid g's dL/dlambda, dL/dmu (from dL/dkappa) into the buffers."""
        o0, o1 = int(self.cell_off[g]), int(self.cell_off[g + 1])
        for t in (grad_kappa, grad_lam, grad_mu):
            if t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != o1 - o0:
                raise ValueError("gradient buffers must be contiguous FP64 (ny, nx) tensors")
        L.lbm_lame_gradient(self.ctx, g, self.lam[o0:o1].data_ptr(), self.mu[o0:o1].data_ptr(),
                            grad_kappa.data_ptr(), grad_lam.data_ptr(), grad_mu.data_ptr())

    def close(self) -> None:
        if getattr(self, "ctx", None):
            torch.cuda.synchronize(self.device)
            L.lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
