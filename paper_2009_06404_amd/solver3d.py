"""Solver3: owns the torch tensors (workspace, Lame fields, traces) that the
three-dimensional entry points of liblbm.so borrow, and forwards every call to
the library. No arithmetic of the scheme happens here; every step runs in the
library's HIP kernels."""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from . import _lib as L
from . import _lib3d as L3

_DT = {"f32": (L.LBM_F32, torch.float32), "f64": (L.LBM_F64, torch.float64)}


class Solver3:
    """One context for one volume. ``problem`` has the attributes of
    ``workloads.problem3.Problem3`` (nx, ny, nz, q, faces, full(), tau,
    sponge_thick, profile(f), sources, receivers, comp_mask)."""

    def __init__(self, problem, dtype: str = "f32", device: str = "cuda",
                 trace_steps: Optional[int] = None, tile: Optional[tuple] = None):
        p = self.problem = problem
        self.dtype = dtype
        self.code, self.tdtype = _DT[dtype]
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        lam, mu, rho = p.full()
        self.lam = torch.as_tensor(lam, dtype=self.tdtype, device=self.device).contiguous()
        self.mu = torch.as_tensor(mu, dtype=self.tdtype, device=self.device).contiguous()
        self.rho = torch.as_tensor(rho, dtype=self.tdtype, device=self.device).contiguous()
        self.q = int(getattr(p, "q", 19))
        self.ws_bytes = L3.lbm3_workspace_bytes(p.nx, p.ny, p.nz, self.q, self.code)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        bc, keep = L3.make_bc(p.faces, p.sponge_thick, [p.profile(f) for f in range(6)])
        self.ctx = L3.lbm3_init(p.nx, p.ny, p.nz, self.q, self.code, self.lam.data_ptr(),
                                self.mu.data_ptr(), self.rho.data_ptr(), p.tau, bc,
                                self.workspace.data_ptr(), self.ws_bytes, self.stream.cuda_stream)
        del keep
        if p.sources:
            L3.lbm3_set_sources(self.ctx, [s.as_tuple() for s in p.sources])
        if tile is not None:
            L3.lbm3_set_tile(self.ctx, *tile)
        self.trace = None
        if trace_steps and p.nrec > 0:
            self.attach_receivers(p.receivers, p.comp_mask, trace_steps)

    def attach_receivers(self, xyz, comp_mask: int, steps: int) -> torch.Tensor:
        xyz = np.asarray(xyz, np.int32).reshape(-1, 3)
        ncomp = bin(comp_mask).count("1")
        self.trace = torch.zeros((steps, xyz.shape[0], ncomp), dtype=self.tdtype, device=self.device)
        L3.lbm3_set_receivers(self.ctx, xyz, comp_mask, self.trace.data_ptr(), steps)
        return self.trace

    def step(self, n: int) -> None:
        L3.lbm3_step(self.ctx, n)

    def step_timed(self, n: int) -> dict:
        """Mean durations and cells of the lean and general launches of a step."""
        return L3.lbm3_step_timed(self.ctx, n)

    def moments(self) -> torch.Tensor:
        p = self.problem
        out = torch.empty((10, p.nz, p.ny, p.nx), dtype=self.tdtype, device=self.device)
        L3.lbm3_moments(self.ctx, out.data_ptr())
        return out

    def state(self) -> torch.Tensor:
        p = self.problem
        out = torch.empty((self.q, p.nz, p.ny, p.nx), dtype=self.tdtype, device=self.device)
        L3.lbm3_get_state(self.ctx, out.data_ptr())
        return out

    def set_state(self, src: torch.Tensor, t: int) -> None:
        p = self.problem
        src = src.to(device=self.device, dtype=self.tdtype).contiguous()
        if tuple(src.shape) != (self.q, p.nz, p.ny, p.nx):
            raise ValueError("state must have shape (q, nz, ny, nx)")
        self._state_in = src       # kept until the asynchronous copy has run
        L3.lbm3_set_state(self.ctx, src.data_ptr(), t)

    @property
    def time(self) -> int:
        return L3.lbm3_get_time(self.ctx)

    def tile(self):
        return L3.lbm3_get_tile(self.ctx)

    def set_tile(self, rows_y: int, planes_z: int = 0) -> None:
        L3.lbm3_set_tile(self.ctx, rows_y, planes_z)

    @property
    def lean_width(self) -> int:
        """Columns of the lean tiles (64, or 128 for FP32)."""
        return L3.lbm3_get_lean_width(self.ctx)

    def set_lean_width(self, columns: int) -> None:
        L3.lbm3_set_lean_width(self.ctx, columns)

    def close(self) -> None:
        if getattr(self, "ctx", None) is not None:
            L3.lbm3_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
