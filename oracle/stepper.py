"""ctypes front end of the C oracle (test infrastructure, see ``oracle/__init__``).

``run(problem, ...)`` executes the paper's scheme in FP64 on the CPU and returns
the populations, the macroscopic fields and the receiver traces.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_oracle.so")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class OracleCfg(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("bc", C.c_int32 * 4),
        ("rigid_row", C.c_int32),
        ("sp_thick", C.c_int32 * 4),
        ("tau", C.c_double),
        ("sp_prof", _dp * 4),
        ("nsrc", C.c_int32), ("nrec", C.c_int32),
        ("src", _dp),
        ("rec_xy", _ip),
        ("comp_mask", C.c_int32), ("pad_", C.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        L.oracle_run.restype = C.c_int
        L.oracle_run.argtypes = [C.POINTER(OracleCfg), _dp, _dp, _dp, _dp, C.c_int32,
                                 C.c_int64, C.c_int64, _dp, _dp, _dp, _dp]
        L.oracle_adjoint.restype = C.c_int
        L.oracle_adjoint.argtypes = [C.POINTER(OracleCfg), _dp, _dp, _dp, _dp, C.c_int32,
                                     C.c_int64, C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp]
        L.oracle_collide_cell.restype = None
        L.oracle_collide_cell.argtypes = [_dp, _dp, C.c_double, C.c_double, _dp, _dp, _dp]
        L.oracle_equilibrium.restype = None
        L.oracle_equilibrium.argtypes = [C.c_double, _dp, _dp, _dp]
        L.oracle_lattice.restype = None
        L.oracle_lattice.argtypes = [_ip, _ip, _dp, _ip]
        L.oracle_num_threads.restype = C.c_int
        L.oracle_set_num_threads.restype = None
        L.oracle_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray], ct=_dp):
    if a is None:
        return C.cast(None, ct)
    return a.ctypes.data_as(ct)


def lattice():
    cx = np.zeros(9, np.int32)
    cy = np.zeros(9, np.int32)
    w = np.zeros(9)
    opp = np.zeros(9, np.int32)
    lib().oracle_lattice(_ptr(cx, _ip), _ptr(cy, _ip), _ptr(w), _ptr(opp, _ip))
    return cx, cy, w, opp


def equilibrium(rho: float, j, P):
    j = np.ascontiguousarray(j, dtype=np.float64)
    P = np.ascontiguousarray(P, dtype=np.float64)
    out = np.zeros(9)
    lib().oracle_equilibrium(float(rho), _ptr(j), _ptr(P), _ptr(out))
    return out


def collide_cell(f, G, A: float, tau: float):
    f = np.ascontiguousarray(f, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.float64)
    fs = np.zeros(9)
    j = np.zeros(2)
    S = np.zeros(2)
    lib().oracle_collide_cell(_ptr(f), _ptr(G), float(A), float(tau), _ptr(fs), _ptr(j), _ptr(S))
    return fs, j, S


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's OpenMP regions from here on."""
    lib().oracle_set_num_threads(int(n))


def _cfg(p):
    cfg = OracleCfg()
    cfg.nx, cfg.ny = p.nx, p.ny
    for e in range(4):
        cfg.bc[e] = int(p.bc[e])
        cfg.sp_thick[e] = int(p.sponge_thick[e])
    cfg.rigid_row = int(p.rigid_row)
    cfg.tau = float(p.tau)
    keep = []
    for e in range(4):
        prof = np.ascontiguousarray(p.profile(e), dtype=np.float64)
        if prof.size == 0:
            prof = np.zeros(1)
        keep.append(prof)
        cfg.sp_prof[e] = _ptr(prof)
    src = np.ascontiguousarray([s.as_tuple() for s in p.sources], dtype=np.float64).reshape(-1, 8)
    if src.size == 0:
        src = np.zeros((1, 8))
    rec = np.ascontiguousarray(p.receivers, dtype=np.int32).reshape(-1, 2)
    if rec.size == 0:
        rec_buf = np.zeros((1, 2), np.int32)
    else:
        rec_buf = rec
    keep += [src, rec_buf]
    cfg.nsrc = len(p.sources)
    cfg.nrec = int(rec.shape[0])
    cfg.src = _ptr(src)
    cfg.rec_xy = _ptr(rec_buf, _ip)
    cfg.comp_mask = int(p.comp_mask)
    return cfg, keep


def run(p, nsteps: Optional[int] = None, t0: int = 0,
        fstar_init: Optional[np.ndarray] = None, medium=None,
        want_trace: bool = True, f_init: Optional[np.ndarray] = None):
    """Run the oracle on problem ``p`` for ``nsteps`` steps from time ``t0``.

    fstar_init: post-collision state at t0-1, shape (9, ny, nx); or f_init:
    pre-collision state at t0; neither: the rest state. Returns a dict with ``fstar`` (t0+n-1), ``f`` (t0+n),
    ``mom`` (6, ny, nx) = rho, j_x, j_y, P_xx, P_xy, P_yy at t0+n, and
    ``trace`` (n, nrec, ncomp).
    """
    n = p.nsteps if nsteps is None else int(nsteps)
    lam, mu, rho0 = (medium if medium is not None else p.medium.full(p.ny, p.nx))
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
    cfg, keep = _cfg(p)
    shape = (9, p.ny, p.nx)
    fs_out = np.zeros(shape)
    f_out = np.zeros(shape)
    mom = np.zeros((6, p.ny, p.nx))
    trace = np.zeros((max(n, 1), max(p.nrec, 1), max(p.ncomp, 1)))
    init, kind = None, 0
    if fstar_init is not None:
        init = np.ascontiguousarray(fstar_init, dtype=np.float64).reshape(shape)
    elif f_init is not None:
        init, kind = np.ascontiguousarray(f_init, dtype=np.float64).reshape(shape), 1
    rc = lib().oracle_run(C.byref(cfg), _ptr(lam), _ptr(mu), _ptr(rho0), _ptr(init),
                          kind, int(t0), n, _ptr(fs_out), _ptr(f_out), _ptr(mom),
                          _ptr(trace) if (want_trace and p.nrec > 0) else _ptr(None))
    if rc != 0:
        raise MemoryError("oracle_run failed with %d" % rc)
    del keep
    return {"fstar": fs_out, "f": f_out, "mom": mom,
            "trace": trace[:n, :p.nrec, :p.ncomp]}


def adjoint(p, nsteps: Optional[int] = None, residual: Optional[np.ndarray] = None,
            adj_init: Optional[np.ndarray] = None, t0: int = 0,
            fstar_init: Optional[np.ndarray] = None, f_init: Optional[np.ndarray] = None,
            medium=None):
    """Forward run of ``p`` from t0 for nsteps steps, then the discrete adjoint
    back to t0 (FP64, the transpose of every phase of the step).

    residual: e(t) = v(t) - d(t), shape (nsteps, nrec, ncomp), or None (zero);
    adj_init: fh(t0+nsteps) = dL/df(t0+nsteps), shape (9, ny, nx), or None.
    Returns ``adj`` = dL/df(t0) (pre-collision populations at t0), ``grad_kappa``
    (ny, nx), ``grad_amp`` (nsrc,) and the forward ``trace``.
    """
    n = p.nsteps if nsteps is None else int(nsteps)
    lam, mu, rho0 = (medium if medium is not None else p.medium.full(p.ny, p.nx))
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
    cfg, keep = _cfg(p)
    shape = (9, p.ny, p.nx)
    adj = np.zeros(shape)
    gk = np.zeros((p.ny, p.nx))
    ga = np.zeros(max(len(p.sources), 1))
    trace = np.zeros((max(n, 1), max(p.nrec, 1), max(p.ncomp, 1)))
    res = None
    if residual is not None and p.nrec > 0:
        res = np.ascontiguousarray(residual, dtype=np.float64).reshape(n, p.nrec, p.ncomp)
    ai = None if adj_init is None else np.ascontiguousarray(adj_init, dtype=np.float64).reshape(shape)
    init, kind = None, 0
    if fstar_init is not None:
        init = np.ascontiguousarray(fstar_init, dtype=np.float64).reshape(shape)
    elif f_init is not None:
        init, kind = np.ascontiguousarray(f_init, dtype=np.float64).reshape(shape), 1
    rc = lib().oracle_adjoint(C.byref(cfg), _ptr(lam), _ptr(mu), _ptr(rho0), _ptr(init), kind,
                              int(t0), n, _ptr(res), _ptr(ai), _ptr(adj), _ptr(gk), _ptr(ga),
                              _ptr(trace) if p.nrec > 0 else _ptr(None))
    if rc != 0:
        raise MemoryError("oracle_adjoint failed with %d" % rc)
    del keep
    return {"adj": adj, "grad_kappa": gk, "grad_amp": ga[:len(p.sources)],
            "trace": trace[:n, :p.nrec, :p.ncomp]}


def misfit(trace: np.ndarray, d_obs: np.ndarray):
    """L = 1/2 sum (v - d)^2 and the residual e = v - d."""
    e = np.asarray(trace, dtype=np.float64) - np.asarray(d_obs, dtype=np.float64)
    return 0.5 * float(np.sum(e * e)), e


def lame_gradients(grad_kappa: np.ndarray, lam: np.ndarray, mu: np.ndarray):
    """dL/dlambda and dL/dmu from dL/dkappa with kappa = b^2 (mu - lambda)/mu
    (Sec. 4): dkappa/dlambda = -b^2/mu, dkappa/dmu = b^2 lambda/mu^2."""
    b2 = 1.0 / 3.0
    lam = np.asarray(lam, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    return -b2 * grad_kappa / mu, b2 * grad_kappa * lam / (mu * mu)
