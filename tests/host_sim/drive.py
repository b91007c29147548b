"""Drive the library's host code, built against the stub HIP runtime in this
folder, through the same C-ABI call sequences as the GPU tests: forward
stepping with launch changes, moments, state copies, and adjoint runs with
checkpoints, uneven segments and batched grids. Run as a script by
tests/test_host_code_cpu.py with the built library's path."""
import ctypes as C
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

import paper_2009_06404_amd._lib as L  # noqa: E402

L.LIB_PATH = sys.argv[1]
L._lib = None
lib = L.lib()
sim = C.CDLL(sys.argv[1])
sim.sim_register.argtypes = [C.c_void_p, C.c_size_t]

from workloads import BC_FREE, BC_FREE0, BC_PERIODIC, BC_RIGID, Medium, Problem, Source  # noqa: E402
from workloads.problem import default_sponge_profile  # noqa: E402

keep = []


def dev(a):
    a = np.ascontiguousarray(a)
    keep.append(a)
    sim.sim_register(a.ctypes.data, a.nbytes)
    return a


def problem(bc, rr, nx, ny, seed, sources=None, receivers=None):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(0.036, 0.044, (ny, nx))
    nu = rng.uniform(0.15, 0.3, (ny, nx))
    lam = 2 * nu * mu / (1 - 2 * nu)
    prof = default_sponge_profile(6)
    thick = (0, 6, 6, 0)
    src = sources or [Source(nx * 0.3, ny * 0.4, 2.0, 0.0, 1.0, 1.0, 12.0, 16.0)]
    rec = receivers or ([(x, 0) for x in range(0, nx, 3)] + [(x, ny // 2) for x in range(1, nx, 7)])
    return Problem(nx=nx, ny=ny, bc=bc, medium=Medium("field", lam, mu, np.ones((ny, nx))),
                   tau=0.9, rigid_row=rr, sponge_thick=thick,
                   sponge_profiles=tuple(prof if t else None for t in thick), sources=src,
                   receivers=np.asarray(rec, np.int32), comp_mask=3)


def run(probs, T, seg, dtype, launch=None, chunks=None, resident=0):
    code, npdt = (L.LBM_F32, np.float32) if dtype == "f32" else (L.LBM_F64, np.float64)
    grids = [(p.nx, p.ny) for p in probs]
    fields = [np.concatenate([p.medium.full(p.ny, p.nx)[k].ravel() for p in probs]).astype(npdt)
              for k in range(3)]
    lam, mu, rho = (dev(f) for f in fields)
    nb = L.lbm_workspace_bytes(grids, code)
    ws = dev(np.zeros(nb + 512, np.uint8))
    wp = (ws.ctypes.data + 255) // 256 * 256
    bcs = [(p.bc[0], p.bc[1], p.bc[2], p.bc[3], p.rigid_row) for p in probs]
    sps = [(tuple(p.sponge_thick), tuple(p.profile(e) for e in range(4))) for p in probs]
    ctx = L.lbm_init(grids, code, lam.ctypes.data, mu.ctypes.data, rho.ctypes.data, probs[0].tau,
                     bcs, sps, wp, nb, 0)
    for g, p in enumerate(probs):
        L.lbm_set_sources(ctx, g, [s.as_tuple() for s in p.sources])
        tr = dev(np.zeros((T, p.nrec, p.ncomp), npdt))
        L.lbm_set_receivers(ctx, g, np.asarray(p.receivers, np.int32), p.comp_mask, tr.ctypes.data, T)
    if launch:
        lc = L.lbm_get_launch(ctx)
        lc.update(launch)
        L.lbm_set_launch(ctx, **lc)
    ab = L.lbm_adjoint_workspace_bytes_resident(ctx, seg, T, resident)
    assert (ab == L.lbm_adjoint_workspace_bytes(ctx, seg, T)) == (resident < T - (T - 1) // seg * seg)
    adj_before = sim.sim_adjoint_pairs_checked()
    aws = dev(np.zeros(ab + 512, np.uint8))
    L.lbm_adjoint_begin(ctx, seg, T, (aws.ctypes.data + 255) // 256 * 256, ab)
    # the forward in pieces that cross the checkpoints and the kept range
    for n in (3, T // 2 - 3, T - T // 2):
        L.lbm_step(ctx, n)
    for g, p in enumerate(probs):
        res = dev(np.ones((T, p.nrec, p.ncomp), npdt))
        gk = dev(np.zeros((p.ny, p.nx)))
        ga = dev(np.zeros(max(len(p.sources), 1)))
        L.lbm_adjoint_set_io(ctx, g, res.ctypes.data, gk.ctypes.data, ga.ctypes.data)
    for i, n in enumerate(chunks or [T]):
        if i % 2:
            kt = L.lbm_adjoint_step_timed(ctx, n)
            assert kt["steps"] == n, kt
        else:
            L.lbm_adjoint_step(ctx, n)
    for g, p in enumerate(probs):
        out = dev(np.zeros((9, p.ny, p.nx), npdt))
        L.lbm_adjoint_get_state(ctx, g, out.ctypes.data)
        mom = dev(np.zeros((6, p.ny, p.nx), npdt))
        L.lbm_moments(ctx, g, mom.ctypes.data)
        L.lbm_get_state(ctx, g, out.ctypes.data)
    L.lbm_destroy(ctx)
    return sim.sim_adjoint_pairs_checked() - adj_before


sim.sim_pairs_checked.restype = C.c_int64
sim.sim_adjoint_pairs_checked.restype = C.c_int64


def run_forward(probs, T, launch, steps=(5, 1, 8), tune=None):
    """Forward steps only, with the given launch (two-step path when
    fuse_rows > 0): odd and even step counts, graphs, timed steps. With tune,
    lbm_autotune first runs every candidate shape for that many steps, and a
    second call with steps = 0 must return the cached choice."""
    code, npdt = (L.LBM_F32, np.float32)
    grids = [(p.nx, p.ny) for p in probs]
    fields = [np.concatenate([p.medium.full(p.ny, p.nx)[k].ravel() for p in probs]).astype(npdt)
              for k in range(3)]
    lam, mu, rho = (dev(f) for f in fields)
    nb = L.lbm_workspace_bytes(grids, code)
    ws = dev(np.zeros(nb + 512, np.uint8))
    wp = (ws.ctypes.data + 255) // 256 * 256
    bcs = [(p.bc[0], p.bc[1], p.bc[2], p.bc[3], p.rigid_row) for p in probs]
    sps = [(tuple(p.sponge_thick), tuple(p.profile(e) for e in range(4))) for p in probs]
    ctx = L.lbm_init(grids, code, lam.ctypes.data, mu.ctypes.data, rho.ctypes.data, probs[0].tau,
                     bcs, sps, wp, nb, 0)
    T = sum(steps) + 8
    for g, p in enumerate(probs):
        L.lbm_set_sources(ctx, g, [s.as_tuple() for s in p.sources])
        tr = dev(np.zeros((T, p.nrec, p.ncomp), npdt))
        L.lbm_set_receivers(ctx, g, np.asarray(p.receivers, np.int32), p.comp_mask, tr.ctypes.data, T)
    lc = L.lbm_get_launch(ctx)
    lc.update(launch)
    L.lbm_set_launch(ctx, **lc)
    if tune is not None:
        chosen = L.lbm_autotune(ctx, tune)
        assert L.lbm_autotune(ctx, 0) == chosen == L.lbm_get_launch(ctx), chosen
        assert (chosen["fuse_rows"] > 0) == (lc["fuse_rows"] > 0), (chosen, lc)
    before = sim.sim_pairs_checked()
    L.lbm_set_finite_check(ctx, 4)
    for n in steps:
        L.lbm_step(ctx, n)
        L.lbm_filter(ctx, 0.01)
    kt = L.lbm_step_timed(ctx, 4)
    assert L.lbm_check_finite_noalloc(ctx)
    assert L.lbm_finite_status(ctx) == (True, -1)
    L.lbm_set_finite_check(ctx, 0)
    after = sim.sim_pairs_checked()
    L.lbm_destroy(ctx)
    return after - before, kt


CASES = [
    ("periodic", (BC_PERIODIC,) * 4, -1),
    ("free_rigid_interface", (BC_FREE, BC_RIGID, BC_PERIODIC, BC_PERIODIC), 17),
    ("free0_rigid_sides", (BC_FREE0, BC_FREE0, BC_RIGID, BC_RIGID), -1),
    ("rigid_box_interface", (BC_RIGID,) * 4, 9),
]
for dtype in ("f64", "f32"):
    for name, bc, rr in CASES:
        run([problem(bc, rr, 70, 40, 1)], 24, 7, dtype)
        big = problem(bc, -1 if rr < 0 else 90, 300, 200, 2,
                      sources=[Source(40.0, 30.0, 2.0, 0.3, 0.9, 1.0, 12.0, 16.0)],
                      receivers=[(x, 0) for x in range(0, 300, 5)] + [(x, 101) for x in range(3, 300, 11)])
        for launch in (dict(waves=1, rows=4), dict(waves=2, rows=8), dict(waves=8, rows=2),
                       dict(waves=2, rows=8, fuse_rows=6)):
            apairs = run([big], 20, 8, dtype, launch=launch)
            # adjoint pairs on the two-step path: in every segment of 8 steps
            assert (apairs > 0) == ("fuse_rows" in launch), (launch, apairs)
        print("ok", name, dtype, flush=True)
    run([problem(CASES[1][1], 20, 150, 37, 3), problem(CASES[3][1], -1, 64, 65, 4)], 18, 5, dtype,
        launch=dict(waves=2, rows=4), chunks=[7, 11])
# two-step path: blocks of 256 columns; every pair must write each cell once
# and the second general step may read only intermediate cells of its pair
FUSED = [
    ("periodic", (BC_PERIODIC,) * 4, -1, 600, 120),
    ("free_rigid_interface", (BC_FREE, BC_RIGID, BC_PERIODIC, BC_PERIODIC), 61, 530, 150),
    ("free0_rigid_sides", (BC_FREE0, BC_FREE0, BC_RIGID, BC_RIGID), -1, 780, 97),
]
for name, bc, rr, nx, ny in FUSED:
    p = problem(bc, rr, nx, ny, 5, sources=[Source(nx * 0.7, ny * 0.5, 2.0, 0.3, 0.9, 1.0, 12.0, 16.0)],
                receivers=[(x, 0) for x in range(0, nx, 5)] + [(x, 77) for x in range(3, nx, 11)])
    for fr in (4, 8, 13):
        for extra in (dict(), dict(overlap=0), dict(graph_chunk=6), dict(waves=8), dict(waves=1)):
            pairs, kt = run_forward([p], 0, dict(dict(waves=4, rows=8, fuse_rows=fr), **extra))
            assert pairs > 0 and kt["fused_cells"] > 0, (name, fr, extra, pairs, kt)
    print("ok fused", name, flush=True)
pairs, kt = run_forward([problem(FUSED[1][1], 40, 530, 90, 6), problem(FUSED[0][1], -1, 300, 64, 7),
                         problem(FUSED[2][1], -1, 1100, 50, 8)], 0, dict(waves=2, rows=4, fuse_rows=6))
assert pairs > 0, pairs
# three-step path: blocks of 128, 192 and 256 columns (tri_waves, or waves
# with 8 counting as 4); the
# step counts leave a pair and a single step over; every launch reads only
# cells holding the state of its starting time, and every triple writes each
# cell once
sim.sim_triples_checked.restype = C.c_int64
sim.sim_time_reads.restype = C.c_int64
for name, bc, rr, nx, ny in FUSED:
    p = problem(bc, rr, nx, ny, 5, sources=[Source(nx * 0.7, ny * 0.5, 2.0, 0.3, 0.9, 1.0, 12.0, 16.0)],
                receivers=[(x, 0) for x in range(0, nx, 5)] + [(x, 77) for x in range(3, nx, 11)])
    for fr in (4, 8, 13):
        for extra in (dict(), dict(overlap=0), dict(graph_chunk=6), dict(waves=8), dict(waves=2),
                      dict(tri_waves=3), dict(waves=8, tri_waves=3, overlap=0), dict(tri_waves=2)):
            t0 = sim.sim_triples_checked()
            pairs, kt = run_forward([p], 0, dict(dict(waves=4, rows=8, fuse_rows=fr, fuse_steps=3), **extra))
            assert sim.sim_triples_checked() > t0 and kt["fused_steps"] == 3 and kt["fused_cells"] > 0, \
                (name, fr, extra, kt)
    print("ok three-step", name, flush=True)
t0 = sim.sim_triples_checked()
pairs, kt = run_forward([problem(FUSED[1][1], 40, 530, 90, 6), problem(FUSED[0][1], -1, 300, 64, 7),
                         problem(FUSED[2][1], -1, 1100, 50, 8)], 0,
                        dict(waves=2, rows=4, fuse_rows=6, fuse_steps=3), steps=(3, 7, 12))
assert sim.sim_triples_checked() > t0, kt
t0 = sim.sim_triples_checked()
pairs, kt = run_forward([problem(FUSED[1][1], 40, 530, 90, 6), problem(FUSED[0][1], -1, 300, 64, 7),
                         problem(FUSED[2][1], -1, 1100, 50, 8)], 0,
                        dict(waves=1, rows=4, fuse_rows=6, fuse_steps=3, tri_waves=3), steps=(3, 7, 12))
assert sim.sim_triples_checked() > t0, kt
assert sim.sim_time_reads() > 0
# autotuning: every candidate shape of either path runs through the checks
# above, and each result lands in the cache file LBM_TUNE_CACHE names
cache = os.path.join(os.path.dirname(sys.argv[1]), "tune_cache.txt")
os.environ["LBM_TUNE_CACHE"] = cache
tp = problem(FUSED[1][1], 61, 530, 150, 9, sources=[Source(300.0, 75.0, 2.0, 0.3, 0.9, 1.0, 12.0, 16.0)],
             receivers=[(x, 0) for x in range(0, 530, 5)])
for fr in (6, 0):
    pairs, kt = run_forward([tp], 0, dict(waves=4, rows=8, fuse_rows=fr), tune=3)
    assert (pairs > 0) == (fr > 0), (fr, pairs)
t0 = sim.sim_triples_checked()
pairs, kt = run_forward([tp], 0, dict(waves=4, rows=8, fuse_rows=6, fuse_steps=3), tune=3)
assert sim.sim_triples_checked() > t0 and kt["fused_steps"] == 3, kt
lines = open(cache).read().splitlines()
assert len(lines) == 3 and lines[0].startswith("sim f32 ") and " pairs|" in lines[0], lines
assert " single|" in lines[1] and " triples|" in lines[2], lines
print("ok autotune", flush=True)

# densities kept from the recorded forward: none, the last (short) segment,
# a few whole segments, all of them; every plane the adjoint reads must hold
# the density of the time it reads it for
for dtype in ("f32", "f64"):
    p = problem(FUSED[1][1], 61, 530, 150, 12, sources=[Source(300.0, 75.0, 2.0, 0.3, 0.9, 1.0, 12.0, 16.0)],
                receivers=[(x, 0) for x in range(0, 530, 5)] + [(x, 77) for x in range(3, 530, 11)])
    for launch in (dict(waves=2, rows=8, fuse_rows=8), dict(waves=2, rows=8),
                   dict(waves=2, rows=8, fuse_rows=8, fuse_steps=3)):
        for resident, chunks in ((0, [23]), (2, [5, 18]), (12, [1, 22]), (23, [23]), (1000, [4, 19])):
            run([p], 23, 7, dtype, launch=launch, chunks=chunks, resident=resident)
    print("ok kept densities", dtype, flush=True)

# adjoint pairs: blocks of 128, 256 and 512 columns (256 in FP64), segments of
# odd and even lengths (a pair never spans two), adjoint steps taken in odd
# chunks, batched grids; every pair writes each cell once and its second
# general step reads only cells its first wrote
for dtype in ("f32", "f64"):
    for name, bc, rr, nx, ny in FUSED:
        p = problem(bc, rr, nx, ny, 11, sources=[Source(nx * 0.7, ny * 0.5, 2.0, 0.3, 0.9, 1.0, 12.0, 16.0)],
                    receivers=[(x, 0) for x in range(0, nx, 5)] + [(x, 77) for x in range(3, nx, 11)])
        for fr, waves, seg, chunks in ((4, 2, 7, [5, 3, 9, 4]), (13, 4, 8, [21]), (8, 8, 5, [1, 2, 18])):
            apairs = run([p], 21, seg, dtype, launch=dict(waves=waves, rows=8, fuse_rows=fr),
                         chunks=chunks)
            assert apairs > 0, (name, dtype, fr, waves, apairs)
    apairs = run([problem(FUSED[1][1], 40, 530, 90, 6), problem(FUSED[0][1], -1, 300, 64, 7),
                  problem(FUSED[2][1], -1, 1100, 50, 8)], 16, 6, dtype,
                 launch=dict(waves=2, rows=4, fuse_rows=6, overlap=0), chunks=[3, 13])
    assert apairs > 0, apairs
    print("ok adjoint pairs", dtype, flush=True)


def init_only(nx, ny, code, npdt):
    """A context on one homogeneous nx x ny grid (no steps)."""
    lam = dev(np.full(nx * ny, 0.03, npdt))
    mu = dev(np.full(nx * ny, 0.04, npdt))
    rho = dev(np.ones(nx * ny, npdt))
    nb = L.lbm_workspace_bytes([(nx, ny)], code)
    ws = dev(np.zeros(nb + 512, np.uint8))
    wp = (ws.ctypes.data + 255) // 256 * 256
    sps = [((0, 0, 0, 0), tuple(np.zeros(0) for _ in range(4)))]
    return L.lbm_init([(nx, ny)], code, lam.ctypes.data, mu.ctypes.data, rho.ctypes.data, 1.0,
                      [(BC_FREE0, BC_RIGID, BC_PERIODIC, BC_PERIODIC, -1)], sps, wp, nb, 0)


def refused(ctx, **kw):
    before = L.lbm_get_launch(ctx)
    lc = dict(before, **kw)
    try:
        L.lbm_set_launch(ctx, **lc)
    except L.LBMError as e:
        assert "descriptor" in str(e), str(e)
        assert L.lbm_get_launch(ctx) == before
        return True
    return False


# descriptor reach: a tile's rows (plus 6) and a two-step block's rows (plus
# 8; a three-step block's plus 12) of nine population runs must stay within
# 2^31 - 1 and 2^32 - 1 bytes
ctx = init_only(4096, 40, L.LBM_F64, np.float64)          # 294912 B per row
assert not refused(ctx, rows=7275) and refused(ctx, rows=7276)
L.lbm_destroy(ctx)
ctx = init_only(828544, 3, L.LBM_F64, np.float64)         # 59655168 B per row
assert not refused(ctx, rows=29, fuse_rows=63, fuse_steps=2)
assert refused(ctx, rows=30) and refused(ctx, rows=8, fuse_rows=64, fuse_steps=2)
assert not refused(ctx, rows=8, fuse_rows=59, fuse_steps=3)
assert refused(ctx, rows=8, fuse_rows=60, fuse_steps=3)
L.lbm_destroy(ctx)
# the widest FP32 grid: the default launch takes 2-row tiles and 4-row
# three-step blocks (8-row blocks on the two-step path)
ctx = init_only(7456512, 3, L.LBM_F32, np.float32)
lc = L.lbm_get_launch(ctx)
assert lc["rows"] == 2 and lc["fuse_rows"] == 4 and lc["fuse_steps"] == 3, lc
assert refused(ctx, rows=3) and refused(ctx, fuse_rows=5)
assert not refused(ctx, fuse_rows=8, fuse_steps=2) and refused(ctx, fuse_rows=9, fuse_steps=2)
L.lbm_destroy(ctx)
print("ok descriptor reach", flush=True)
# three-step block widths: 2, 3 or 4 wavefronts, 0 to follow waves
ctx = init_only(4096, 40, L.LBM_F32, np.float32)
for bad in (1, 5, -1):
    try:
        L.lbm_set_launch(ctx, **dict(L.lbm_get_launch(ctx), tri_waves=bad))
        raise AssertionError(f"tri_waves {bad} accepted")
    except L.LBMError as e:
        assert "tri_waves" in str(e), str(e)
for good in (0, 2, 3, 4):
    L.lbm_set_launch(ctx, **dict(L.lbm_get_launch(ctx), tri_waves=good))
    assert L.lbm_get_launch(ctx)["tri_waves"] == good
L.lbm_destroy(ctx)
print("ok three-step widths", flush=True)
print("ALL OK", flush=True)
