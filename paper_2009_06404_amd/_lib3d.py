"""ctypes binding of the three-dimensional (D3Q19 / D3Q27) entry points of liblbm.so
(include/lbm3d.h): argument marshalling only, one wrapper per entry point with
the C name. Errors raise :class:`LBMError` with the library's message."""
from __future__ import annotations

import ctypes as C
import warnings

from ._lib import LBM_WARN_UNSTABLE, LBMError, check, last_error, lib as _lib2d  # noqa: F401

ENTRY_POINTS = (
    "lbm3_workspace_bytes", "lbm3_init", "lbm3_set_sources", "lbm3_set_receivers",
    "lbm3_step", "lbm3_step_timed", "lbm3_moments", "lbm3_get_time", "lbm3_get_state",
    "lbm3_set_state", "lbm3_set_tile", "lbm3_get_tile", "lbm3_set_lean_width",
    "lbm3_get_lean_width", "lbm3_destroy", "lbm3_vn_growth", "lbm3_stability",
)

FACE_TOP, FACE_BOTTOM, FACE_LEFT, FACE_RIGHT, FACE_FRONT, FACE_BACK = range(6)
D3Q19, D3Q27 = 19, 27

_dp = C.POINTER(C.c_double)


class lbm3_bc(C.Structure):
    _fields_ = [("face", C.c_int32 * 6), ("thick", C.c_int32 * 6), ("profile", _dp * 6)]


class lbm3_kernel_times(C.Structure):
    _fields_ = [("steps", C.c_int64), ("lean_ms", C.c_double), ("general_ms", C.c_double),
                ("lean_cells", C.c_int64), ("general_cells", C.c_int64), ("step_ms", C.c_double)]


class lbm3_source(C.Structure):
    _fields_ = [(n, C.c_double) for n in
                ("x", "y", "z", "sigma", "dir_x", "dir_y", "dir_z", "amp", "period", "t0")]


_bound = None


def lib():
    global _bound
    L = _lib2d()
    if _bound is not L:
        vp = C.c_void_p
        i32, i64 = C.c_int32, C.c_int64
        sig = {
            "lbm3_workspace_bytes": ([i32, i32, i32, i32, i32, C.POINTER(C.c_size_t)], C.c_int),
            "lbm3_init": ([C.POINTER(vp), i32, i32, i32, i32, i32, vp, vp, vp, C.c_double,
                           C.POINTER(lbm3_bc), vp, C.c_size_t, vp], C.c_int),
            "lbm3_set_sources": ([vp, C.POINTER(lbm3_source), i32], C.c_int),
            "lbm3_set_receivers": ([vp, C.POINTER(C.c_int32), i32, i32, vp, i64], C.c_int),
            "lbm3_step": ([vp, i64], C.c_int),
            "lbm3_step_timed": ([vp, i64, C.POINTER(lbm3_kernel_times)], C.c_int),
            "lbm3_moments": ([vp, vp], C.c_int),
            "lbm3_get_time": ([vp, C.POINTER(i64)], C.c_int),
            "lbm3_get_state": ([vp, vp], C.c_int),
            "lbm3_set_state": ([vp, vp, i64], C.c_int),
            "lbm3_set_tile": ([vp, i32, i32], C.c_int),
            "lbm3_get_tile": ([vp, C.POINTER(i32), C.POINTER(i32)], C.c_int),
            "lbm3_set_lean_width": ([vp, i32], C.c_int),
            "lbm3_get_lean_width": ([vp, C.POINTER(i32)], C.c_int),
            "lbm3_destroy": ([vp], C.c_int),
            "lbm3_vn_growth": ([i32, C.c_double, C.c_double, i32, C.POINTER(C.c_double)], C.c_int),
            "lbm3_stability": ([vp, C.POINTER(C.c_double)], C.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _bound = L
    return L


def lbm3_workspace_bytes(nx: int, ny: int, nz: int, q: int, dtype: int) -> int:
    out = C.c_size_t(0)
    check(lib().lbm3_workspace_bytes(nx, ny, nz, q, dtype, C.byref(out)))
    return out.value


def make_bc(faces, thick=(0,) * 6, profiles=(None,) * 6):
    """An lbm3_bc and the arrays it points to (keep both alive until init)."""
    bc = lbm3_bc()
    keep = []
    for f in range(6):
        bc.face[f] = int(faces[f])
        bc.thick[f] = int(thick[f])
        if thick[f] > 0:
            arr = (C.c_double * int(thick[f]))(*[float(v) for v in profiles[f][:thick[f]]])
            keep.append(arr)
            bc.profile[f] = C.cast(arr, _dp)
    return bc, keep


def lbm3_init(nx, ny, nz, q, dtype, lam_ptr, mu_ptr, rho_ptr, tau, bc, ws_ptr, ws_bytes, stream_ptr):
    """The context; a RuntimeWarning when the library reports LBM_WARN_UNSTABLE."""
    ctx = C.c_void_p()
    rc = check(lib().lbm3_init(C.byref(ctx), nx, ny, nz, q, dtype, lam_ptr, mu_ptr, rho_ptr, float(tau),
                               C.byref(bc), ws_ptr, ws_bytes, stream_ptr))
    if rc == LBM_WARN_UNSTABLE:
        warnings.warn(last_error(), RuntimeWarning, stacklevel=2)
    return ctx


def lbm3_vn_growth(q: int, nu: float, tau: float, nk: int = 13) -> float:
    g = C.c_double(0)
    check(lib().lbm3_vn_growth(q, nu, tau, nk, C.byref(g)))
    return g.value


def lbm3_stability(ctx):
    """(largest von Neumann factor, stable) of the context."""
    g = C.c_double(0)
    rc = check(lib().lbm3_stability(ctx, C.byref(g)))
    return g.value, rc == 0


def lbm3_set_sources(ctx, sources) -> None:
    """sources: sequence of 10-tuples (x, y, z, sigma, dir_x, dir_y, dir_z, amp, period, t0)."""
    n = len(sources)
    arr = (lbm3_source * max(n, 1))(*[lbm3_source(*map(float, s)) for s in sources])
    check(lib().lbm3_set_sources(ctx, arr, n))


def lbm3_set_receivers(ctx, xyz, comp_mask: int, trace_ptr, max_steps: int) -> None:
    import numpy as np
    a = np.ascontiguousarray(np.asarray(xyz, dtype=np.int32).reshape(-1, 3))
    ptr = a.ctypes.data_as(C.POINTER(C.c_int32)) if a.size else None
    check(lib().lbm3_set_receivers(ctx, ptr, int(a.shape[0]), comp_mask, trace_ptr, max_steps))


def lbm3_step(ctx, n: int) -> None:
    check(lib().lbm3_step(ctx, n))


def lbm3_step_timed(ctx, n: int) -> dict:
    kt = lbm3_kernel_times()
    check(lib().lbm3_step_timed(ctx, n, C.byref(kt)))
    return {name: getattr(kt, name) for name, _ in lbm3_kernel_times._fields_}


def lbm3_moments(ctx, out_ptr) -> None:
    check(lib().lbm3_moments(ctx, out_ptr))


def lbm3_get_time(ctx) -> int:
    t = C.c_int64(0)
    check(lib().lbm3_get_time(ctx, C.byref(t)))
    return t.value


def lbm3_get_state(ctx, dst_ptr) -> None:
    check(lib().lbm3_get_state(ctx, dst_ptr))


def lbm3_set_state(ctx, src_ptr, t: int) -> None:
    check(lib().lbm3_set_state(ctx, src_ptr, t))


def lbm3_set_tile(ctx, rows_y: int, planes_z: int = 0) -> None:
    check(lib().lbm3_set_tile(ctx, rows_y, planes_z))


def lbm3_get_tile(ctx):
    r = C.c_int32(0)
    p = C.c_int32(0)
    check(lib().lbm3_get_tile(ctx, C.byref(r), C.byref(p)))
    return r.value, p.value


def lbm3_set_lean_width(ctx, columns: int) -> None:
    check(lib().lbm3_set_lean_width(ctx, columns))


def lbm3_get_lean_width(ctx) -> int:
    c = C.c_int32(0)
    check(lib().lbm3_get_lean_width(ctx, C.byref(c)))
    return c.value


def lbm3_destroy(ctx) -> None:
    check(lib().lbm3_destroy(ctx))
