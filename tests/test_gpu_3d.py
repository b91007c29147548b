"""The three-dimensional step of liblbm.so, on both its lattices (D3Q19 and
D3Q27), against the FP64 three-dimensional oracle (oracle/lbm3d_oracle.c),
through the C ABI of include/lbm3d.h.

* parity of the state, the ten macroscopic fields and the receiver traces on
  volumes spanning several tiles with ragged x / y / z tails, for every face
  kind (periodic, rigid, FREE, FREE0), sponges on every face, uniform and
  cell-wise media, sources and random initial states: FP64 <= 1e-12, FP32
  <= 1e-5 relative L2;
* the tile shape (rows per workgroup 2 / 6 / 14, planes per segment, 64- or
  128-column lean tiles) does not change a single bit;
* the smallest volumes (3 cells on an axis) and a volume of one ragged tile;
* the full 256^3 half-space workload in the launch the benchmark times,
  against the oracle over two steps from a random state.
"""
import numpy as np
import pytest

from oracle import stepper3d as O3
from workloads.problem import BC_FREE, BC_FREE0, BC_PERIODIC, BC_RIGID, default_sponge_profile
from workloads.problem3 import Problem3, Source3, volume_field, volume_half_space
from gpu_helpers import rel_l2

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
FIELDS3 = ("rho", "j_x", "j_y", "j_z", "P_xx", "P_xy", "P_xz", "P_yy", "P_yz", "P_zz")


Q = [19, 27]


def _random_state(p, seed, scale=1e-3):
    return np.random.default_rng(seed).normal(size=(p.q,) + p.shape) * scale


def _run_gpu(p, nsteps, dtype, state=None, t0=0, tile=None, width=None):
    import torch
    from paper_2009_06404_amd.solver3d import Solver3
    s = Solver3(p, dtype=dtype, trace_steps=max(nsteps, 1), tile=tile)
    try:
        if width is not None:
            s.set_lean_width(width)
        if state is not None:
            s.set_state(torch.as_tensor(state), t0)
        s.step(nsteps)
        out = {"fstar": s.state().double().cpu().numpy(), "mom": s.moments().double().cpu().numpy(),
               "trace": s.trace.double().cpu().numpy() if s.trace is not None else None,
               "time": s.time, "tile": s.tile(), "width": s.lean_width}
        torch.cuda.synchronize()
    finally:
        s.close()
    return out


def _compare(g, r, tol, what, near_zero=()):
    """Per-field relative L2 of the ten macroscopic fields, the state and the
    traces, each within tol. Each field is measured against its own norm,
    except those named in near_zero (which the case makes vanish by symmetry):
    those against 1e-3 of the largest field's norm."""
    floor = 1e-3 * max(np.linalg.norm(r["mom"][k]) for k in range(10))
    worst = 0.0
    for name in near_zero:
        assert name in FIELDS3, name
    for k, name in enumerate(FIELDS3):
        nb = float(np.linalg.norm(r["mom"][k]))
        if name in near_zero:
            nb = max(nb, floor)
        e = float(np.linalg.norm(g["mom"][k] - r["mom"][k]) / nb) if nb > 0 else \
            float(np.abs(g["mom"][k]).max())
        assert e <= tol, f"{what} {name}: rel L2 {e:.3e}"
        worst = max(worst, e)
    e = rel_l2(g["fstar"], r["fstar"])
    assert e <= tol, f"{what} state: rel L2 {e:.3e}"
    worst = max(worst, e)
    if r["trace"] is not None and r["trace"].size:
        e = rel_l2(g["trace"], r["trace"])
        assert e <= tol, f"{what} trace: rel L2 {e:.3e}"
        worst = max(worst, e)
    return worst


def _case_field_periodic():
    return volume_field(nx=150, ny=20, nz=16, seed=21, nsteps=30)


def _case_half_space():
    return volume_half_space(n=72, nz=40, nsteps=40, sponge=8, src_depth=6, stride=5).replace(
        sources=[Source3(35.5, 36.0, 6.0, 2.0, 0.0, 0.0, 1.0, 1.0, 12.0, 16.0)])


def _case_free_box():
    rng = np.random.default_rng(3)
    prof = default_sponge_profile(4, 0.2)
    p = volume_field(nx=67, ny=13, nz=11, seed=23, nsteps=25,
                     faces=(BC_FREE, BC_RIGID, BC_RIGID, BC_RIGID, BC_RIGID, BC_RIGID), tau=0.8)
    return p.replace(sponge_thick=(0, 4, 4, 0, 0, 4), sponge_profiles=(None, prof, prof, None, None, prof),
                     receivers=np.stack([rng.integers(0, 67, 30), rng.integers(0, 13, 30),
                                         rng.integers(0, 11, 30)], 1).astype(np.int32))


def _case_mixed():
    prof = default_sponge_profile(2, 0.3)
    p = volume_field(nx=64, ny=7, nz=5, seed=24, nsteps=20,
                     faces=(BC_FREE0, BC_FREE, BC_PERIODIC, BC_PERIODIC, BC_RIGID, BC_RIGID), tau=1.3)
    return p.replace(sponge_thick=(1, 0, 2, 2, 0, 1), sponge_profiles=(np.array([0.1]), None, prof, prof,
                                                                       None, np.array([0.25])))


CASES = {"field_periodic": (_case_field_periodic, False),
         "half_space": (_case_half_space, False),
         "free_box": (_case_free_box, True),
         "mixed": (_case_mixed, True)}


@pytest.mark.parametrize("q", Q)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_parity_with_the_oracle(case, dtype, q):
    make, random_start = CASES[case]
    p = make().replace(q=q)
    n = p.nsteps
    st = _random_state(p, 5) if random_start else None
    ref = O3.run(p, n, fstar_init=st, t0=3 if random_start else 0)
    got = _run_gpu(p, n, dtype, state=st, t0=3 if random_start else 0)
    worst = _compare(got, ref, TOL[dtype], f"{case} {dtype}")
    print(f"[3d] D3Q{q} {case} {dtype}: worst rel L2 {worst:.2e}, tile {got['tile']}, "
          f"lean width {got['width']}", flush=True)
    assert got["time"] == n + (3 if random_start else 0)
    assert np.linalg.norm(ref["fstar"]) > 0


@pytest.mark.parametrize("q", Q)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_tile_shape_does_not_change_a_bit(dtype, q):
    p = _case_free_box().replace(q=q)
    st = _random_state(p, 6)
    base = _run_gpu(p, 12, dtype, state=st, tile=(6, 0))
    for tile in ((2, 1), (14, 3), (6, 11), (2, 4)):
        g = _run_gpu(p, 12, dtype, state=st, tile=tile)
        assert g["tile"][0] == tile[0]
        assert np.array_equal(g["fstar"], base["fstar"]), tile
        assert np.array_equal(g["mom"], base["mom"]), tile
        assert np.array_equal(g["trace"], base["trace"]), tile


@pytest.mark.parametrize("q", Q)
@pytest.mark.parametrize("sides", ["periodic", "rigid"])
def test_lean_tile_width_changes_no_bit(q, sides):
    """FP32 lean tiles of 128 columns (two wavefronts per row) against 64-column
    ones, bit for bit, in 6- and 2-row tiles, and against the oracle: on a
    periodic volume whose last tile is ragged (322 = 2 x 128 + 66 columns)
    with the x wrap inside lean tiles, and on a volume with rigid x and y
    faces (400 columns: the 128-column tiles next to the x faces are general,
    the two between them lean)."""
    if sides == "periodic":
        p = volume_field(nx=322, ny=23, nz=19, seed=31, nsteps=9, q=q)
    else:
        p = volume_field(nx=400, ny=23, nz=19, seed=32, nsteps=9, q=q,
                         faces=(BC_PERIODIC, BC_PERIODIC, BC_RIGID, BC_RIGID, BC_RIGID, BC_RIGID))
    p = p.replace(sources=[], receivers=p.receivers[:3])   # most tiles lean
    st = _random_state(p, 7)
    ref = O3.run(p, 9, fstar_init=st, t0=4)
    for tile in ((6, 0), (2, 5)):
        narrow = _run_gpu(p, 9, "f32", state=st, t0=4, tile=tile, width=64)
        wide = _run_gpu(p, 9, "f32", state=st, t0=4, tile=tile, width=128)
        assert narrow["width"] == 64 and wide["width"] == 128
        for k in ("fstar", "mom", "trace"):
            assert np.array_equal(narrow[k], wide[k]), (tile, k)
        w = _compare(wide, ref, TOL["f32"], f"128 columns {tile}")
        print(f"[3d] D3Q{q} {sides} 128-column lean tiles, tile {tile}: bitwise equal to 64 columns, "
              f"worst rel L2 against the oracle {w:.2e}", flush=True)


@pytest.mark.parametrize("faces", [(BC_PERIODIC,) * 6, (BC_FREE0, BC_RIGID) + (BC_RIGID,) * 4,
                                   (BC_FREE, BC_FREE0, BC_PERIODIC, BC_PERIODIC, BC_RIGID, BC_RIGID)])
@pytest.mark.parametrize("shape", [(3, 3, 3), (3, 5, 4), (5, 3, 70)])
@pytest.mark.parametrize("q", Q)
def test_smallest_volumes(faces, shape, q):
    nz, ny, nx = shape
    p = volume_field(nx=nx, ny=ny, nz=nz, seed=30, nsteps=9, faces=faces, tau=0.9, q=q)
    p = p.replace(receivers=np.array([[0, 0, 0], [nx - 1, ny - 1, nz - 1], [nx // 2, ny // 2, nz // 2]],
                                     np.int32), sources=[])
    st = _random_state(p, 7)
    ref = O3.run(p, 9, fstar_init=st)
    got = _run_gpu(p, 9, "f64", state=st)
    _compare(got, ref, 1e-12, f"{shape} {faces}")


@pytest.mark.parametrize("q", Q)
def test_receivers_restart_with_set_state_and_two_calls_of_step(q):
    """Steps in two calls equal one call; set_state at a new time restarts the
    trace at row 0 (rows hold steps t0, t0+1, ...)."""
    import torch
    from paper_2009_06404_amd.solver3d import Solver3
    p = _case_mixed().replace(q=q)
    st = _random_state(p, 8)
    ref = O3.run(p, 14, fstar_init=st, t0=10)
    s = Solver3(p, dtype="f64", trace_steps=14)
    try:
        s.set_state(torch.as_tensor(st), 10)
        s.step(5)
        s.step(9)
        got = {"fstar": s.state().double().cpu().numpy(), "mom": s.moments().double().cpu().numpy(),
               "trace": s.trace.double().cpu().numpy()}
        assert s.time == 24
    finally:
        s.close()
    _compare(got, ref, 1e-12, "two calls")


@pytest.mark.parametrize("q", Q)
def test_full_size_half_space_against_the_oracle(q):
    """The 256^3 half-space workload (free surface, rigid bottom behind its
    sponge, periodic sides behind theirs, source, 4096 surface receivers) in
    FP32 with the default tile: two steps from a random state at t = 60 (the
    Ricker peak) against the oracle, cell by cell."""
    p = volume_half_space(n=256, q=q)
    st = _random_state(p, 9, 1e-4)
    got = _run_gpu(p, 2, "f32", state=st, t0=60)
    ref = O3.run(p, 2, fstar_init=st, t0=60)
    w = _compare(got, ref, TOL["f32"], "256^3 f32")
    err = np.abs(got["fstar"] - ref["fstar"]).max() / np.abs(ref["fstar"]).max()
    print(f"[3d] D3Q{q} 256^3 f32: worst rel L2 {w:.2e}, max rel {err:.2e}, tile {got['tile']}", flush=True)
    assert err < 1e-4


@pytest.mark.parametrize("q", Q)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_timed_steps_equal_overlapped_steps(dtype, q):
    """lbm3_step (general kernel on the second stream beside the lean one)
    and lbm3_step_timed (one after the other) give the same bits; the timing
    reports both kernels and their cells add up to the volume."""
    import torch
    from paper_2009_06404_amd.solver3d import Solver3
    p = volume_half_space(n=96, nz=70, sponge=8, src_depth=9, stride=3, q=q)
    outs = []
    for timed in (False, True):
        s = Solver3(p, dtype=dtype, trace_steps=30)
        try:
            s.step(5)
            kt = s.step_timed(25) if timed else s.step(25)
            outs.append((s.state().double().cpu().numpy(), s.trace.double().cpu().numpy()))
            torch.cuda.synchronize()
        finally:
            s.close()
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    assert kt["steps"] == 25 and kt["lean_ms"] > 0 and kt["general_ms"] > 0
    assert kt["lean_cells"] + kt["general_cells"] == p.cells
    assert kt["lean_cells"] > kt["general_cells"]
