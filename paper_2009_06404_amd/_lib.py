"""ctypes binding of liblbm.so: the C ABI of include/lbm.h, one Python function
per entry point, argument marshalling only.

torch is imported first so that the HIP runtime it carries is the one the
library binds to (both export the same soname); torch is used for device memory
and streams only. Importing this module without the built library raises.
"""
from __future__ import annotations

import ctypes as C
import os
import warnings

import torch  # noqa: F401  (loads the HIP runtime before liblbm.so)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_WARN_UNSTABLE = 1
LBM_OK = 0
LBM_E_INVALID = -1
LBM_E_NOMEM = -2
LBM_E_DEVICE = -3
LBM_E_NONFINITE = -4
LBM_E_STATE = -5
LBM_F32 = 0
LBM_F64 = 1
LBM_PERIODIC = 0
LBM_FREE = 1
LBM_RIGID = 2
LBM_FREE0 = 3

ENTRY_POINTS = (
    "lbm_abi_version", "lbm_last_error", "lbm_workspace_bytes", "lbm_init",
    "lbm_set_sources", "lbm_set_receivers", "lbm_step", "lbm_step_timed", "lbm_moments",
    "lbm_get_time", "lbm_get_state", "lbm_set_state", "lbm_check_finite",
    "lbm_get_launch", "lbm_set_launch", "lbm_autotune", "lbm_destroy",
    "lbm_adjoint_workspace_bytes", "lbm_adjoint_workspace_bytes_resident", "lbm_adjoint_begin",
    "lbm_adjoint_set_io",
    "lbm_adjoint_step", "lbm_adjoint_step_timed", "lbm_adjoint_time", "lbm_adjoint_get_state",
    "lbm_adjoint_set_state",
    "lbm_misfit", "lbm_lame_gradient", "lbm_vn_growth", "lbm_stability",
    "lbm_vn_growth_filtered", "lbm_filter", "lbm_check_finite_noalloc",
    "lbm_set_finite_check", "lbm_finite_status",
)


class lbm_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32)]


class lbm_bc(C.Structure):
    _fields_ = [("edge", C.c_int32 * 4), ("rigid_row", C.c_int32)]


class lbm_sponge(C.Structure):
    _fields_ = [("thick", C.c_int32 * 4), ("profile", C.POINTER(C.c_double) * 4)]


class lbm_source(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("x", "y", "sigma", "dir_x", "dir_y", "amp", "period", "t0")]


class lbm_launch(C.Structure):
    _fields_ = [("waves", C.c_int32), ("rows", C.c_int32), ("graph_chunk", C.c_int32),
                ("prefetch", C.c_int32), ("split", C.c_int32), ("pair", C.c_int32),
                ("overlap", C.c_int32), ("fuse_rows", C.c_int32), ("fuse_steps", C.c_int32),
                ("tri_waves", C.c_int32)]


class lbm_kernel_times(C.Structure):
    _fields_ = [("steps", C.c_int64), ("interior_ms", C.c_double), ("general_ms", C.c_double),
                ("interior_cells", C.c_int64), ("general_cells", C.c_int64),
                ("fused_ms", C.c_double), ("fused_cells", C.c_int64), ("fused_steps", C.c_int32)]


class LBMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"liblbm error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                "(hipcc --offload-arch=gfx950); there is no fallback path")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        i32, i64 = C.c_int32, C.c_int64
        sig = {
            "lbm_abi_version": ([], C.c_int),
            "lbm_last_error": ([], C.c_char_p),
            "lbm_workspace_bytes": ([C.POINTER(lbm_grid), i32, i32, C.POINTER(C.c_size_t)], C.c_int),
            "lbm_init": ([C.POINTER(vp), C.POINTER(lbm_grid), i32, i32, vp, vp, vp, C.c_double,
                          C.POINTER(lbm_bc), C.POINTER(lbm_sponge), vp, C.c_size_t, vp], C.c_int),
            "lbm_set_sources": ([vp, i32, C.POINTER(lbm_source), i32], C.c_int),
            "lbm_set_receivers": ([vp, i32, C.POINTER(C.c_int32), i32, i32, vp, i64], C.c_int),
            "lbm_step": ([vp, i64], C.c_int),
            "lbm_step_timed": ([vp, i64, C.POINTER(lbm_kernel_times)], C.c_int),
            "lbm_moments": ([vp, i32, vp], C.c_int),
            "lbm_get_time": ([vp, C.POINTER(i64)], C.c_int),
            "lbm_get_state": ([vp, i32, vp], C.c_int),
            "lbm_set_state": ([vp, i32, vp, i64], C.c_int),
            "lbm_check_finite": ([vp], C.c_int),
            "lbm_check_finite_noalloc": ([vp], C.c_int),
            "lbm_set_finite_check": ([vp, i64], C.c_int),
            "lbm_finite_status": ([vp, C.POINTER(i64)], C.c_int),
            "lbm_get_launch": ([vp, C.POINTER(lbm_launch)], C.c_int),
            "lbm_set_launch": ([vp, C.POINTER(lbm_launch)], C.c_int),
            "lbm_autotune": ([vp, i32, C.POINTER(lbm_launch)], C.c_int),
            "lbm_destroy": ([vp], C.c_int),
            "lbm_adjoint_workspace_bytes": ([vp, i32, i64, C.POINTER(C.c_size_t)], C.c_int),
            "lbm_adjoint_workspace_bytes_resident": ([vp, i32, i64, i64, C.POINTER(C.c_size_t)],
                                                     C.c_int),
            "lbm_adjoint_begin": ([vp, i32, i64, vp, C.c_size_t], C.c_int),
            "lbm_adjoint_set_io": ([vp, i32, vp, vp, vp], C.c_int),
            "lbm_adjoint_step": ([vp, i64], C.c_int),
            "lbm_adjoint_step_timed": ([vp, i64, C.POINTER(lbm_kernel_times)], C.c_int),
            "lbm_adjoint_time": ([vp, C.POINTER(i64)], C.c_int),
            "lbm_adjoint_get_state": ([vp, i32, vp], C.c_int),
            "lbm_adjoint_set_state": ([vp, i32, vp], C.c_int),
            "lbm_misfit": ([vp, i32, vp, vp, i64, vp], C.c_int),
            "lbm_lame_gradient": ([vp, i32, vp, vp, vp, vp, vp], C.c_int),
            "lbm_vn_growth": ([C.c_double, C.c_double, i32, C.POINTER(C.c_double)], C.c_int),
            "lbm_stability": ([vp, C.POINTER(C.c_double)], C.c_int),
            "lbm_vn_growth_filtered": ([C.c_double, C.c_double, C.c_double, i32, i32,
                                        C.POINTER(C.c_double)], C.c_int),
            "lbm_filter": ([vp, C.c_double], C.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def last_error() -> str:
    return lib().lbm_last_error().decode()


def check(rc: int) -> int:
    if rc < 0:
        raise LBMError(rc, last_error())
    return rc


# ---- one wrapper per entry point (same names as the C ABI) -----------------

def lbm_abi_version() -> int:
    return lib().lbm_abi_version()


def lbm_workspace_bytes(grids, dtype: int) -> int:
    arr = (lbm_grid * len(grids))(*[lbm_grid(nx, ny) for nx, ny in grids])
    out = C.c_size_t(0)
    check(lib().lbm_workspace_bytes(arr, len(grids), dtype, C.byref(out)))
    return out.value


def lbm_init(grids, dtype, lam_ptr, mu_ptr, rho_ptr, tau, bcs, sponges, ws_ptr, ws_bytes,
             stream_ptr):
    """grids: [(nx, ny)]; bcs: [(top, bottom, left, right, rigid_row)];
    sponges: [((t0, t1, t2, t3), (prof0, ..., prof3))] with float64 numpy
    profiles (copied by the library). Returns the opaque context handle."""
    n = len(grids)
    g = (lbm_grid * n)(*[lbm_grid(nx, ny) for nx, ny in grids])
    b = (lbm_bc * n)()
    for i, (t, bo, l, r, rr) in enumerate(bcs):
        b[i].edge[0], b[i].edge[1], b[i].edge[2], b[i].edge[3] = t, bo, l, r
        b[i].rigid_row = rr
    s = (lbm_sponge * n)()
    keep = []
    for i, (thick, profs) in enumerate(sponges):
        for e in range(4):
            s[i].thick[e] = int(thick[e])
            if thick[e] > 0:
                import numpy as np
                arr = np.ascontiguousarray(profs[e], dtype=np.float64)
                keep.append(arr)
                s[i].profile[e] = arr.ctypes.data_as(C.POINTER(C.c_double))
    ctx = C.c_void_p()
    rc = check(lib().lbm_init(C.byref(ctx), g, n, dtype, lam_ptr, mu_ptr, rho_ptr, float(tau), b, s,
                              ws_ptr, ws_bytes, stream_ptr))
    del keep
    if rc == LBM_WARN_UNSTABLE:
        warnings.warn("liblbm: " + last_error(), RuntimeWarning, stacklevel=3)
    return ctx


def lbm_vn_growth(nu: float, tau: float, nk: int = 17) -> float:
    out = C.c_double()
    check(lib().lbm_vn_growth(float(nu), float(tau), int(nk), C.byref(out)))
    return out.value


def lbm_vn_growth_filtered(nu: float, tau: float, sigma: float, every: int = 1, nk: int = 17) -> float:
    out = C.c_double()
    check(lib().lbm_vn_growth_filtered(float(nu), float(tau), float(sigma), int(every), int(nk),
                                       C.byref(out)))
    return out.value


def lbm_filter(ctx, sigma: float) -> None:
    check(lib().lbm_filter(ctx, float(sigma)))


def lbm_stability(ctx):
    """(largest von Neumann factor, stable?) of the context."""
    out = C.c_double()
    rc = check(lib().lbm_stability(ctx, C.byref(out)))
    return out.value, rc == LBM_OK


def lbm_set_sources(ctx, g: int, sources) -> None:
    """sources: sequence of 8-tuples (x, y, sigma, dir_x, dir_y, amp, period, t0)."""
    arr = (lbm_source * max(len(sources), 1))()
    for i, s in enumerate(sources):
        arr[i] = lbm_source(*[float(v) for v in s])
    check(lib().lbm_set_sources(ctx, g, arr, len(sources)))


def lbm_set_receivers(ctx, g: int, xy, comp_mask: int, trace_ptr, max_steps: int) -> None:
    import numpy as np
    a = np.ascontiguousarray(np.asarray(xy, dtype=np.int32).reshape(-1, 2))
    n = int(a.shape[0])
    check(lib().lbm_set_receivers(ctx, g, a.ctypes.data_as(C.POINTER(C.c_int32)), n, comp_mask,
                                  trace_ptr, int(max_steps)))


def lbm_step(ctx, n: int) -> None:
    check(lib().lbm_step(ctx, int(n)))


def lbm_step_timed(ctx, n: int) -> dict:
    out = lbm_kernel_times()
    check(lib().lbm_step_timed(ctx, int(n), C.byref(out)))
    return {k: getattr(out, k) for k, _ in lbm_kernel_times._fields_}


def lbm_moments(ctx, g: int, out_ptr) -> None:
    check(lib().lbm_moments(ctx, g, out_ptr))


def lbm_get_time(ctx) -> int:
    t = C.c_int64()
    check(lib().lbm_get_time(ctx, C.byref(t)))
    return t.value


def lbm_get_state(ctx, g: int, dst_ptr) -> None:
    check(lib().lbm_get_state(ctx, g, dst_ptr))


def lbm_set_state(ctx, g: int, src_ptr, t: int) -> None:
    check(lib().lbm_set_state(ctx, g, src_ptr, int(t)))


def lbm_check_finite(ctx) -> bool:
    rc = lib().lbm_check_finite(ctx)
    if rc == LBM_E_NONFINITE:
        return False
    check(rc)
    return True


def lbm_set_finite_check(ctx, every: int) -> None:
    check(lib().lbm_set_finite_check(ctx, int(every)))


def lbm_finite_status(ctx):
    """(ok, t_bad): t_bad is the first checked time whose state held NaN or
    Inf, -1 when none."""
    t = C.c_int64(-1)
    rc = lib().lbm_finite_status(ctx, C.byref(t))
    if rc == LBM_E_NONFINITE:
        return False, t.value
    check(rc)
    return True, t.value


def lbm_check_finite_noalloc(ctx) -> bool:
    rc = lib().lbm_check_finite_noalloc(ctx)
    if rc == LBM_E_NONFINITE:
        return False
    check(rc)
    return True


def lbm_get_launch(ctx):
    o = lbm_launch()
    check(lib().lbm_get_launch(ctx, C.byref(o)))
    return {k: getattr(o, k) for k, _ in lbm_launch._fields_}


def lbm_set_launch(ctx, waves: int, rows: int, graph_chunk: int = 0, prefetch: int = 1,
                   split: int = 1, pair: int = 0, overlap: int = 1, fuse_rows: int = 0,
                   fuse_steps: int = 2, tri_waves: int = 0) -> None:
    o = lbm_launch(waves, rows, graph_chunk, prefetch, split, pair, overlap, fuse_rows, fuse_steps,
                   tri_waves)
    check(lib().lbm_set_launch(ctx, C.byref(o)))


def lbm_autotune(ctx, steps: int = 5):
    o = lbm_launch()
    check(lib().lbm_autotune(ctx, int(steps), C.byref(o)))
    return {k: getattr(o, k) for k, _ in lbm_launch._fields_}


def lbm_destroy(ctx) -> None:
    if ctx:
        check(lib().lbm_destroy(ctx))


def lbm_adjoint_workspace_bytes(ctx, seg_steps: int, nsteps: int) -> int:
    out = C.c_size_t(0)
    check(lib().lbm_adjoint_workspace_bytes(ctx, int(seg_steps), int(nsteps), C.byref(out)))
    return int(out.value)


def lbm_adjoint_workspace_bytes_resident(ctx, seg_steps: int, nsteps: int,
                                         resident_steps: int) -> int:
    out = C.c_size_t()
    check(lib().lbm_adjoint_workspace_bytes_resident(ctx, int(seg_steps), int(nsteps),
                                                     int(resident_steps), C.byref(out)))
    return out.value


def lbm_adjoint_begin(ctx, seg_steps: int, nsteps: int, ws_ptr, ws_bytes: int) -> None:
    check(lib().lbm_adjoint_begin(ctx, int(seg_steps), int(nsteps), ws_ptr, int(ws_bytes)))


def lbm_adjoint_set_io(ctx, g: int, residual_ptr, grad_kappa_ptr, grad_amp_ptr) -> None:
    check(lib().lbm_adjoint_set_io(ctx, int(g), residual_ptr, grad_kappa_ptr, grad_amp_ptr))


def lbm_adjoint_step(ctx, n: int) -> None:
    check(lib().lbm_adjoint_step(ctx, int(n)))


def lbm_adjoint_step_timed(ctx, n: int) -> dict:
    out = lbm_kernel_times()
    check(lib().lbm_adjoint_step_timed(ctx, int(n), C.byref(out)))
    return {k: getattr(out, k) for k, _ in lbm_kernel_times._fields_}


def lbm_adjoint_time(ctx) -> int:
    t = C.c_int64(0)
    check(lib().lbm_adjoint_time(ctx, C.byref(t)))
    return int(t.value)


def lbm_adjoint_get_state(ctx, g: int, dst_ptr) -> None:
    check(lib().lbm_adjoint_get_state(ctx, int(g), dst_ptr))


def lbm_adjoint_set_state(ctx, g: int, src_ptr) -> None:
    check(lib().lbm_adjoint_set_state(ctx, int(g), src_ptr))


def lbm_misfit(ctx, g: int, d_obs_ptr, residual_ptr, nrows: int, misfit_ptr) -> None:
    check(lib().lbm_misfit(ctx, int(g), d_obs_ptr, residual_ptr, int(nrows), misfit_ptr))


def lbm_lame_gradient(ctx, g: int, lam_ptr, mu_ptr, grad_kappa_ptr, grad_lam_ptr, grad_mu_ptr) -> None:
    check(lib().lbm_lame_gradient(ctx, int(g), lam_ptr, mu_ptr, grad_kappa_ptr, grad_lam_ptr,
                                  grad_mu_ptr))
