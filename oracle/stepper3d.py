"""ctypes front end of the D3Q19 oracle (test infrastructure, see ``oracle/__init__``).

``run(problem, ...)`` executes the three-dimensional form of the paper's
scheme (D3Q19 or D3Q27, ``problem.q``) in FP64 on the CPU and returns the
populations, the macroscopic fields and the receiver traces.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from .stepper import lib

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)

LATTICES = (19, 27)


class Oracle3Cfg(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("face", C.c_int32 * 6),
        ("sp_thick", C.c_int32 * 6),
        ("nsrc", C.c_int32),
        ("tau", C.c_double),
        ("sp_prof", _dp * 6),
        ("src", _dp),
        ("nrec", C.c_int32), ("comp_mask", C.c_int32),
        ("rec_xyz", _ip),
        ("q", C.c_int32), ("pad_", C.c_int32),
    ]


_bound = False


def _lib():
    global _bound
    L = lib()
    if not _bound:
        L.oracle3_run.restype = C.c_int
        L.oracle3_run.argtypes = [C.POINTER(Oracle3Cfg), _dp, _dp, _dp, _dp, C.c_int32,
                                  C.c_int64, C.c_int64, _dp, _dp, _dp, _dp]
        L.oracle3_collide_cell.restype = None
        L.oracle3_collide_cell.argtypes = [C.c_int32, _dp, _dp, C.c_double, C.c_double, _dp, _dp, _dp]
        L.oracle3_equilibrium.restype = None
        L.oracle3_equilibrium.argtypes = [C.c_int32, C.c_double, _dp, _dp, _dp]
        L.oracle3_lattice.restype = C.c_int
        L.oracle3_lattice.argtypes = [C.c_int32, _ip, _dp, _ip]
        _bound = True
    return L


def _ptr(a, ct=_dp):
    if a is None:
        return C.cast(None, ct)
    return a.ctypes.data_as(ct)


def lattice(q: int = 19):
    """(c (q, 3) int, w (q,), opp (q,)) of the oracle's D3Q19 / D3Q27 table."""
    c = np.zeros((q, 3), np.int32)
    w = np.zeros(q)
    opp = np.zeros(q, np.int32)
    if _lib().oracle3_lattice(q, _ptr(c, _ip), _ptr(w), _ptr(opp, _ip)) != q:
        raise ValueError("lattice must be 19 or 27")
    return c, w, opp


def equilibrium(rho: float, j, P, q: int = 19):
    """P = (P_xx, P_xy, P_xz, P_yy, P_yz, P_zz)."""
    j = np.ascontiguousarray(j, dtype=np.float64)
    P = np.ascontiguousarray(P, dtype=np.float64)
    out = np.zeros(q)
    _lib().oracle3_equilibrium(q, float(rho), _ptr(j), _ptr(P), _ptr(out))
    return out


def collide_cell(f, G, A: float, tau: float):
    f = np.ascontiguousarray(f, dtype=np.float64)
    q = f.size
    G = np.ascontiguousarray(G, dtype=np.float64)
    fs = np.zeros(q)
    j = np.zeros(3)
    S = np.zeros(3)
    _lib().oracle3_collide_cell(q, _ptr(f), _ptr(G), float(A), float(tau), _ptr(fs), _ptr(j), _ptr(S))
    return fs, j, S


def _cfg(p):
    cfg = Oracle3Cfg()
    cfg.nx, cfg.ny, cfg.nz = p.nx, p.ny, p.nz
    keep = []
    for e in range(6):
        cfg.face[e] = int(p.faces[e])
        cfg.sp_thick[e] = int(p.sponge_thick[e])
        prof = np.ascontiguousarray(p.profile(e), dtype=np.float64)
        if prof.size == 0:
            prof = np.zeros(1)
        keep.append(prof)
        cfg.sp_prof[e] = _ptr(prof)
    cfg.tau = float(p.tau)
    src = np.ascontiguousarray([s.as_tuple() for s in p.sources], dtype=np.float64).reshape(-1, 10)
    if src.size == 0:
        src = np.zeros((1, 10))
    rec = np.ascontiguousarray(p.receivers, dtype=np.int32).reshape(-1, 3)
    rec_buf = rec if rec.size else np.zeros((1, 3), np.int32)
    keep += [src, rec_buf]
    cfg.nsrc = len(p.sources)
    cfg.src = _ptr(src)
    cfg.nrec = int(rec.shape[0])
    cfg.comp_mask = int(p.comp_mask)
    cfg.rec_xyz = _ptr(rec_buf, _ip)
    cfg.q = int(getattr(p, "q", 19))
    return cfg, keep


def run(p, nsteps: Optional[int] = None, t0: int = 0,
        fstar_init: Optional[np.ndarray] = None, f_init: Optional[np.ndarray] = None,
        want_trace: bool = True):
    """Run the D3Q19 oracle on ``p`` for ``nsteps`` steps from time ``t0``.

    fstar_init: post-collision state at t0-1, shape (q, nz, ny, nx); or
    f_init: pre-collision state at t0; neither: the rest state. Returns a dict
    with ``fstar`` (t0+n-1), ``f`` (t0+n), ``mom`` (10, nz, ny, nx) = rho, j,
    P_xx, P_xy, P_xz, P_yy, P_yz, P_zz at t0+n, and ``trace`` (n, nrec, ncomp).
    """
    n = p.nsteps if nsteps is None else int(nsteps)
    lam, mu, rho0 = p.full()
    cfg, keep = _cfg(p)
    shape = (cfg.q,) + p.shape
    fs_out = np.zeros(shape)
    f_out = np.zeros(shape)
    mom = np.zeros((10,) + p.shape)
    trace = np.zeros((max(n, 1), max(p.nrec, 1), max(p.ncomp, 1)))
    init, kind = None, 0
    if fstar_init is not None:
        init = np.ascontiguousarray(fstar_init, dtype=np.float64).reshape(shape)
    elif f_init is not None:
        init, kind = np.ascontiguousarray(f_init, dtype=np.float64).reshape(shape), 1
    rc = _lib().oracle3_run(C.byref(cfg), _ptr(lam), _ptr(mu), _ptr(rho0), _ptr(init), kind,
                            int(t0), n, _ptr(fs_out), _ptr(f_out), _ptr(mom),
                            _ptr(trace) if (want_trace and p.nrec > 0) else _ptr(None))
    if rc != 0:
        raise MemoryError("oracle3_run failed with %d" % rc)
    del keep
    return {"fstar": fs_out, "f": f_out, "mom": mom,
            "trace": trace[:n, :p.nrec, :p.ncomp]}
