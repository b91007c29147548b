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
                 autotune: bool = False):
        if not isinstance(problems, (list, tuple)):
            problems = [problems]
        self.problems = list(problems)
        p0 = self.problems[0]
        self.dtype = dtype or p0.dtype
        self.code, self.tdtype = _DT[self.dtype]
        self.device = torch.device(device)
        taus = {float(p.tau) for p in self.problems}
        if len(taus) != 1:
            raise ValueError("all problems of a batch must share tau")
        self.tau = taus.pop()
        grids = [(p.nx, p.ny) for p in self.problems]
        lam, mu, rho = [], [], []
        for p in self.problems:
            l, m, r = _field_tensor(p.medium, p.ny, p.nx, self.tdtype, self.device)
            lam.append(l.reshape(-1))
            mu.append(m.reshape(-1))
            rho.append(r.reshape(-1))
        self.lam = torch.cat(lam)
        self.mu = torch.cat(mu)
        self.rho = torch.cat(rho)
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
                   split: int = 1, pair: int = 0) -> None:
        L.lbm_set_launch(self.ctx, waves, rows, graph_chunk, prefetch, split, pair)

    def autotune(self, steps: int = 5) -> dict:
        return L.lbm_autotune(self.ctx, steps)

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
