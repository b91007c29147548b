"""Drive the host code of the three-dimensional step, built against the stub
HIP runtime in this folder, through the call sequences of the GPU tests:
volumes with ragged tails on both lattices and both dtypes, every face mix,
sources by and across faces, receivers on face cells, several tile shapes,
stepping, timed steps, 64- and 128-column lean tiles, fields, state copies and
argument errors. The stub
checks every launch's tiles (see stub3.cpp). Run as a script by
tests/test_host_code_cpu.py with the built library's path."""
import ctypes as C
import os
import sys
import warnings

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import paper_2009_06404_amd._lib as L  # noqa: E402

L.LIB_PATH = sys.argv[1]
L._lib = None
import paper_2009_06404_amd._lib3d as L3  # noqa: E402

L3.lib()
sim = C.CDLL(sys.argv[1])
sim.sim_register.argtypes = [C.c_void_p, C.c_size_t]
sim.sim3_steps_checked.restype = C.c_longlong
sim.sim3_lean_tiles.restype = C.c_longlong
sim.sim3_general_tiles.restype = C.c_longlong
sim.sim3_wide_launches.restype = C.c_longlong
sim.sim3_lean_src_tiles.restype = C.c_longlong

from workloads.problem import BC_FREE, BC_FREE0, BC_PERIODIC, BC_RIGID, default_sponge_profile  # noqa: E402
from workloads.problem3 import Source3  # noqa: E402

keep = []
warnings.simplefilter("ignore", RuntimeWarning)   # LBM_WARN_UNSTABLE of unstable media or LBM_FREE


def dev(a):
    a = np.ascontiguousarray(a)
    keep.append(a)
    sim.sim_register(a.ctypes.data, a.nbytes)
    return a


def run(shape, faces, q, dtype, tile, sources, receivers, thick=(0, 4, 3, 0, 2, 0)):
    nz, ny, nx = shape
    code, npdt = (L.LBM_F32, np.float32) if dtype == "f32" else (L.LBM_F64, np.float64)
    rng = np.random.default_rng(nx * ny + nz)
    mu = rng.uniform(0.036, 0.044, shape)
    nu = rng.uniform(0.15, 0.3, shape)
    lam = dev((2 * nu * mu / (1 - 2 * nu)).astype(npdt))
    mu = dev(mu.astype(npdt))
    rho = dev(np.ones(shape, npdt))
    nb = L3.lbm3_workspace_bytes(nx, ny, nz, q, code)
    ws = dev(np.zeros(nb + 512, np.uint8))
    wp = (ws.ctypes.data + 255) // 256 * 256
    ext = (nz, nz, nx, nx, ny, ny)
    th = tuple(min(t, e) for t, e in zip(thick, ext))
    bc, kb = L3.make_bc(faces, th, [default_sponge_profile(t) for t in th])
    ctx = L3.lbm3_init(nx, ny, nz, q, code, lam.ctypes.data, mu.ctypes.data, rho.ctypes.data, 0.9,
                       bc, wp, nb, None)
    g, stable = L3.lbm3_stability(ctx)
    assert 0.99 < g < 1.5, g
    if BC_FREE in faces[:2]:
        assert not stable                    # the printed free surface is always reported
    L3.lbm3_set_sources(ctx, [s.as_tuple() for s in sources])
    T = 12
    rec = np.asarray(receivers, np.int32).reshape(-1, 3)
    tr = dev(np.zeros((T, max(len(rec), 1), 3), npdt))
    L3.lbm3_set_receivers(ctx, rec, 7, tr.ctypes.data, T)
    if tile is not None:
        L3.lbm3_set_tile(ctx, *tile)
    L3.lbm3_step(ctx, 3)
    kt = L3.lbm3_step_timed(ctx, 2)
    assert kt["lean_cells"] + kt["general_cells"] == nx * ny * nz, kt
    # width of the lean tiles: 128 columns by default for FP32
    wide = dtype == "f32"
    rows = 6 if tile is None else tile[0]
    assert L3.lbm3_get_lean_width(ctx) == (128 if wide and rows != 14 else 64)
    L3.lbm3_set_lean_width(ctx, 64)
    assert L3.lbm3_get_lean_width(ctx) == 64
    L3.lbm3_step(ctx, 1)
    if wide:
        L3.lbm3_set_lean_width(ctx, 128)
        L3.lbm3_step(ctx, 1)
    else:
        try:
            L3.lbm3_set_lean_width(ctx, 128)
        except L.LBMError:
            pass
        else:
            raise AssertionError("128-column tiles accepted for FP64")
    out10 = dev(np.zeros((10,) + shape, npdt))
    L3.lbm3_moments(ctx, out10.ctypes.data)
    st = dev(np.zeros((q,) + shape, npdt))
    L3.lbm3_get_state(ctx, st.ctypes.data)
    L3.lbm3_set_state(ctx, st.ctypes.data, 40)
    L3.lbm3_set_tile(ctx, 2, 1)
    L3.lbm3_step(ctx, 2)
    L3.lbm3_set_receivers(ctx, rec[:0], 7, None, 0)
    L3.lbm3_step(ctx, 1)
    assert L3.lbm3_get_time(ctx) == 43
    for bad in (lambda: L3.lbm3_set_sources(ctx, [(nx + 1.0, 0, 0, 1, 0, 0, 1, 1, 10, 10)]),
                lambda: L3.lbm3_set_tile(ctx, 5, 0),
                lambda: L3.lbm3_set_receivers(ctx, [(0, 0, nz)], 1, tr.ctypes.data, T)):
        try:
            bad()
        except L.LBMError:
            pass
        else:
            raise AssertionError("invalid call accepted")
    L3.lbm3_destroy(ctx)
    del kb


P = BC_PERIODIC
MIXES = [(P,) * 6, (BC_FREE0, BC_RIGID, P, P, P, P), (BC_FREE, BC_FREE0, BC_RIGID, BC_RIGID, P, P),
         (BC_RIGID,) * 6, (P, P, BC_RIGID, BC_RIGID, BC_RIGID, BC_RIGID)]
SHAPES = [(3, 3, 3), (5, 7, 70), (11, 13, 67), (20, 9, 130), (37, 15, 64)]
n = 0
for si, shape in enumerate(SHAPES):
    nz, ny, nx = shape
    for mi, faces in enumerate(MIXES):
        for q in (19, 27):
            dtype = "f32" if (si + mi + q) % 2 else "f64"
            tile = [None, (6, 0), (14, 5), (2, 3), (6, nz)][(si + mi) % 5]
            srcs = [Source3(nx * 0.5, ny * 0.5, nz * 0.5, 1.0, 0, 0, 1),
                    Source3(0.0, ny - 1.0, 0.0, 1.5, 1, 0, 0),            # a corner: wraps where periodic
                    Source3(nx - 1.0, 0.0, nz * 0.3, 0.4, 0, 1, 0)][: 1 + (si + mi) % 3]
            recs = [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (nx // 3, ny // 2, 0), (nx // 3, ny // 2, 0),
                    (nx // 2, 0, nz // 2)]
            run(shape, faces, q, dtype, tile, srcs, recs)
            n += 1
print(f"volumes {n}, steps checked {sim.sim3_steps_checked()}, lean tiles {sim.sim3_lean_tiles()}, "
      f"general tiles {sim.sim3_general_tiles()}, 128-column launches {sim.sim3_wide_launches()}, "
      f"lean tiles near sources {sim.sim3_lean_src_tiles()}")
assert sim.sim3_lean_tiles() > 0 and sim.sim3_general_tiles() > 0 and sim.sim3_wide_launches() > 0
assert sim.sim3_lean_src_tiles() > 0, "no lean tile near a source was launched"
print("ALL OK")
