"""The two-step path (temporal blocking, launch fuse_rows > 0) against single
steps and the FP64 oracle.

The two-step kernel performs the single-step kernels' per-cell operations in
the same order, so a run on the two-step path must equal the single-step run
bit for bit: state and traces, for odd and even step counts, with and without
the general kernel on the second stream, for several block widths and
heights, boundary mixes, media and a batch of uneven grids, launched directly
and as captured HIP graphs (graph_chunk / 2 pairs per graph, replayed several
times, with chunks of an even and an odd number of pairs and direct steps
after the last whole chunk). One run per case is also compared with the
oracle.
"""
import numpy as np
import pytest

import workloads as w
from workloads import BC_FREE0, BC_PERIODIC, BC_RIGID, Medium, Problem, Source
from workloads.configs import lame_from_poisson
from workloads.problem import default_sponge_profile
from oracle import stepper
from gpu_helpers import compare, run_gpu

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
NSTEPS = 61


def _field_periodic(nx=700, ny=200, seed=11, tau=0.8):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(0.036, 0.044, (ny, nx))
    nu = rng.uniform(0.1, 0.3, (ny, nx))
    lam = 2 * nu * mu / (1 - 2 * nu)
    rec = [(x, ny // 5) for x in range(0, nx, 9)] + [(x, 3 * ny // 4) for x in range(5, nx, 31)]
    return Problem(nx=nx, ny=ny, bc=(BC_PERIODIC,) * 4,
                   medium=Medium("field", lam, mu, np.ones((ny, nx))), tau=tau,
                   sources=[Source(nx * 0.6, ny * 0.55, 2.5, 0.6, 0.8, 1.0, 14.0, 20.0)],
                   receivers=np.asarray(rec, np.int32), comp_mask=3, nsteps=NSTEPS,
                   name="field_periodic")


def _rigid_sides(nx=530, ny=150, tau=0.9):
    lam, mu = lame_from_poisson(0.3)
    prof = default_sponge_profile(10)
    rec = [(x, 0) for x in range(0, nx, 4)]
    return Problem(nx=nx, ny=ny, bc=(BC_FREE0, BC_RIGID, BC_RIGID, BC_RIGID), rigid_row=90,
                   medium=Medium("homogeneous", lam, mu, 1.0), tau=tau,
                   sponge_thick=(0, 10, 0, 0), sponge_profiles=(None, prof, None, None),
                   sources=[Source(120.0, 40.0, 2.0, 0.0, 1.0, 1.0, 12.0, 18.0)],
                   receivers=np.asarray(rec, np.int32), comp_mask=3, nsteps=NSTEPS,
                   name="rigid_sides")


CASES = {
    "surface_sponges": lambda: w.plain_large(n=600, nsteps=NSTEPS, sponge=24, src_depth=30),
    "layered_interface": lambda: w.hbm_scale(n=640, nsteps=NSTEPS, sponge=32),
    "field_periodic": _field_periodic,
    "rigid_sides": _rigid_sides,
}

FUSED = [
    dict(waves=4, rows=8, fuse_rows=8),
    dict(waves=4, rows=8, fuse_rows=4, overlap=0),
    dict(waves=2, rows=4, fuse_rows=13, graph_chunk=8),
    dict(waves=8, rows=8, fuse_rows=32, graph_chunk=14, overlap=0),
    dict(waves=2, rows=4, fuse_rows=16, graph_chunk=6),
]


def _fused_cells(p, dtype, launch):
    from paper_2009_06404_amd import Solver
    s = Solver(p, dtype=dtype, trace_steps=1, launch=launch)
    try:
        return s.step_timed(0)["fused_cells"]
    finally:
        s.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_two_step_path_equals_single_steps(case, dtype):
    p = CASES[case]()
    ref = run_gpu(p, NSTEPS, dtype, launch=dict(waves=4, rows=8))
    compare(ref, stepper.run(p, nsteps=NSTEPS), TOL[dtype], f"{case} {dtype}")
    for launch in FUSED:
        assert _fused_cells(p, dtype, launch) > 0, (case, launch)
        g = run_gpu(p, NSTEPS, dtype, launch=launch)
        assert np.array_equal(ref["fstar"], g["fstar"]), (case, launch)
        assert np.array_equal(ref["trace"], g["trace"]), (case, launch)
        assert np.array_equal(ref["mom"], g["mom"]), (case, launch)
    print(f"[two-step] {case} {dtype}: {len(FUSED)} launch shapes bitwise equal", flush=True)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_two_step_path_batched_uneven_grids(dtype):
    probs = [_field_periodic(nx=560, ny=120, seed=12, tau=1.0), _rigid_sides(nx=600, ny=96, tau=1.0),
             w.hbm_scale(n=300, nsteps=NSTEPS, sponge=16), w.plain_small(n=96, nsteps=NSTEPS).replace(tau=1.0)]
    ref = run_gpu(probs, NSTEPS, dtype, launch=dict(waves=2, rows=4))
    for launch in (dict(waves=2, rows=4, fuse_rows=6), dict(waves=4, rows=8, fuse_rows=16, graph_chunk=8),
                   dict(waves=2, rows=8, fuse_rows=32, graph_chunk=10)):
        got = run_gpu(probs, NSTEPS, dtype, launch=launch)
        for g, (a, b) in enumerate(zip(ref, got)):
            assert np.array_equal(a["fstar"], b["fstar"]), (g, launch)
            if a["trace"] is not None:
                assert np.array_equal(a["trace"], b["trace"]), (g, launch)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_two_step_timed_steps_equal_plain_steps(dtype):
    """lbm_step_timed on the two-step path (pairs plus an odd last step)
    advances the state like lbm_step and reports the two-step kernel."""
    import torch
    from paper_2009_06404_amd import Solver
    p = _field_periodic()
    launch = dict(waves=4, rows=8, fuse_rows=16)
    outs = []
    for timed in (False, True):
        s = Solver(p, dtype=dtype, trace_steps=40, launch=launch)
        try:
            s.step(9)
            if timed:
                kt = s.step_timed(31)
            else:
                s.step(31)
            outs.append((s.state().double().cpu().numpy(), s.traces[0].double().cpu().numpy()))
            assert s.time == 40
            torch.cuda.synchronize()
        finally:
            s.close()
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    assert kt["steps"] == 31 and kt["fused_ms"] > 0 and kt["fused_cells"] > 0
    assert kt["general_ms"] > 0


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_adjoint_with_two_step_forward(dtype):
    """The adjoint's recorded forward, its recompute and the adjoint steps
    themselves may run on the two-step path (pairs, and single steps up to
    each checkpoint; the recompute also stashes rho of both steps of a pair):
    the checkpoints, traces, adjoint state and dL/dkappa equal those of
    single steps bit for bit."""
    from test_gpu_adjoint import _gpu_adjoint, _problem
    p = _problem((BC_FREE0, BC_RIGID, BC_PERIODIC, BC_PERIODIC), -1, nx=600, ny=90, seed=5)
    T = 31
    res = np.random.default_rng(6).standard_normal((T, p.nrec, p.ncomp))
    assert _fused_cells(p, dtype, dict(waves=4, rows=8, fuse_rows=16)) > 0
    a = _gpu_adjoint([p], T, 7, dtype, [res], launch=dict(waves=4, rows=8))[0]
    b = _gpu_adjoint([p], T, 7, dtype, [res], launch=dict(waves=4, rows=8, fuse_rows=16))[0]
    for k in ("trace", "adj", "grad_kappa"):
        assert np.array_equal(a[k], b[k]), k
    assert np.allclose(a["grad_amp"], b["grad_amp"], rtol=1e-13, atol=0)
