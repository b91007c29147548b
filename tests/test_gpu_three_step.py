"""The three-step path (launch fuse_steps = 3) against single steps and the
FP64 oracle.

The three-step kernel performs the single-step kernels' per-cell operations in
the same order, so a run on the three-step path must equal the single-step
run bit for bit: state, traces and moments, for step counts that leave a pair
and a single step over, with and without the general kernel's first step on
the second stream, for blocks of 128, 192 and 256 columns (tri_waves 2, 3 and
4; without tri_waves the width follows waves, 8 counting as 4) and
several heights, the boundary mixes and media of the two-step tests and a
batch of uneven grids, launched directly and as captured HIP graphs
(graph_chunk / 3 triples per graph, replayed several times, with direct steps
after the last whole chunk). One run per case is also compared with the
oracle.
"""
import numpy as np
import pytest

import workloads as w
from oracle import stepper
from gpu_helpers import compare, run_gpu
from test_gpu_two_step import CASES, NSTEPS, TOL, _field_periodic, _fused_cells, _rigid_sides

pytestmark = pytest.mark.gpu

TRIPLES = [
    dict(waves=4, rows=8, fuse_rows=8, fuse_steps=3),
    dict(waves=2, rows=4, fuse_rows=4, fuse_steps=3, overlap=0),
    dict(waves=2, rows=4, fuse_rows=13, fuse_steps=3, graph_chunk=9),
    dict(waves=8, rows=8, fuse_rows=32, fuse_steps=3, graph_chunk=15, overlap=0),
    dict(waves=4, rows=4, fuse_rows=16, fuse_steps=3, graph_chunk=6),
    dict(waves=2, rows=4, fuse_rows=7, fuse_steps=3, tri_waves=3),
    dict(waves=4, rows=8, fuse_rows=24, fuse_steps=3, tri_waves=3, graph_chunk=9, overlap=0),
    dict(waves=8, rows=8, fuse_rows=10, fuse_steps=3, tri_waves=2),
]


def _kernel_times(p, dtype, launch, steps):
    from paper_2009_06404_amd import Solver
    s = Solver(p, dtype=dtype, trace_steps=max(steps, 1), launch=launch)
    try:
        return s.step_timed(steps)
    finally:
        s.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_three_step_path_equals_single_steps(case, dtype):
    p = CASES[case]()
    ref = run_gpu(p, NSTEPS, dtype, launch=dict(waves=4, rows=8))
    for k, launch in enumerate(TRIPLES):
        kt = _kernel_times(p, dtype, launch, 3)
        assert kt["fused_steps"] == 3 and kt["fused_cells"] > 0, (case, launch, kt)
        g = run_gpu(p, NSTEPS, dtype, launch=launch)
        if k == 0:
            compare(g, stepper.run(p, nsteps=NSTEPS), TOL[dtype], f"{case} {dtype} three-step")
        assert np.array_equal(ref["fstar"], g["fstar"]), (case, launch)
        assert np.array_equal(ref["trace"], g["trace"]), (case, launch)
        assert np.array_equal(ref["mom"], g["mom"]), (case, launch)
    print(f"[three-step] {case} {dtype}: {len(TRIPLES)} launch shapes bitwise equal", flush=True)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_three_step_path_batched_uneven_grids(dtype):
    probs = [_field_periodic(nx=560, ny=120, seed=12, tau=1.0), _rigid_sides(nx=600, ny=96, tau=1.0),
             w.hbm_scale(n=300, nsteps=NSTEPS, sponge=16), w.plain_small(n=96, nsteps=NSTEPS).replace(tau=1.0)]
    ref = run_gpu(probs, NSTEPS, dtype, launch=dict(waves=2, rows=4))
    for launch in (dict(waves=2, rows=4, fuse_rows=6, fuse_steps=3),
                   dict(waves=4, rows=8, fuse_rows=16, fuse_steps=3, graph_chunk=12),
                   dict(waves=2, rows=8, fuse_rows=32, fuse_steps=3, graph_chunk=9),
                   dict(waves=2, rows=8, fuse_rows=32, fuse_steps=3, tri_waves=3, graph_chunk=9),
                   dict(waves=1, rows=4, fuse_rows=5, fuse_steps=3, tri_waves=3)):
        got = run_gpu(probs, NSTEPS, dtype, launch=launch)
        for g, (a, b) in enumerate(zip(ref, got)):
            assert np.array_equal(a["fstar"], b["fstar"]), (g, launch)
            if a["trace"] is not None:
                assert np.array_equal(a["trace"], b["trace"]), (g, launch)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_three_step_leftover_pairs_and_timed_steps(dtype):
    """Step counts of every remainder modulo 3, through lbm_step and
    lbm_step_timed, give the single-step bits; the timed steps report the
    three-step kernel."""
    import torch
    from paper_2009_06404_amd import Solver
    p = _field_periodic()
    chunks = (5, 4, 9, 1, 11, 2, 8)   # 40 steps
    outs = []
    for launch, timed in ((dict(waves=4, rows=8), False),
                          (dict(waves=4, rows=8, fuse_rows=16, fuse_steps=3), False),
                          (dict(waves=4, rows=8, fuse_rows=16, fuse_steps=3), True)):
        s = Solver(p, dtype=dtype, trace_steps=40, launch=launch)
        try:
            for n in chunks:
                if timed:
                    kt = s.step_timed(n)
                else:
                    s.step(n)
            outs.append((s.state().double().cpu().numpy(), s.traces[0].double().cpu().numpy()))
            assert s.time == 40
            torch.cuda.synchronize()
        finally:
            s.close()
    for o in outs[1:]:
        assert np.array_equal(outs[0][0], o[0])
        assert np.array_equal(outs[0][1], o[1])
    assert kt["steps"] == 8 and kt["fused_steps"] == 3 and kt["fused_ms"] > 0
    assert kt["general_ms"] > 0


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_adjoint_with_three_step_launch(dtype):
    """With fuse_steps = 3 the adjoint's recorded forward and recompute keep
    to pairs: checkpoints, traces, adjoint state and dL/dkappa equal those of
    single steps bit for bit."""
    from test_gpu_adjoint import _gpu_adjoint, _problem
    from workloads import BC_FREE0, BC_PERIODIC, BC_RIGID
    p = _problem((BC_FREE0, BC_RIGID, BC_PERIODIC, BC_PERIODIC), -1, nx=600, ny=90, seed=5)
    T = 31
    res = np.random.default_rng(6).standard_normal((T, p.nrec, p.ncomp))
    launch = dict(waves=4, rows=8, fuse_rows=16, fuse_steps=3)
    assert _fused_cells(p, dtype, launch) > 0
    a = _gpu_adjoint([p], T, 7, dtype, [res], launch=dict(waves=4, rows=8))[0]
    b = _gpu_adjoint([p], T, 7, dtype, [res], launch=launch)[0]
    for k in ("trace", "adj", "grad_kappa"):
        assert np.array_equal(a[k], b[k]), k
    assert np.allclose(a["grad_amp"], b["grad_amp"], rtol=1e-13, atol=0)


def _short_grid(nx=600, ny=11, tau=0.9):
    from workloads import BC_FREE0, BC_PERIODIC, BC_RIGID, Medium, Problem, Source
    from workloads.configs import lame_from_poisson
    lam, mu = lame_from_poisson(0.25)
    rec = [(x, 0) for x in range(0, nx, 7)]
    return Problem(nx=nx, ny=ny, bc=(BC_FREE0, BC_RIGID, BC_PERIODIC, BC_PERIODIC),
                   medium=Medium("homogeneous", lam, mu, 1.0), tau=tau,
                   sources=[Source(60.0, 5.0, 1.5, 0.0, 1.0, 1.0, 12.0, 18.0)],
                   receivers=np.asarray(rec, np.int32), comp_mask=3, nsteps=NSTEPS,
                   name="short")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_three_step_launch_on_grids_without_three_step_blocks(dtype):
    """An 11-row grid holds two-step blocks (own rows 4..6) but no three-step
    blocks (six rows of reach each side): under fuse_steps = 3 it runs pairs.
    A graph chunk of 9 steps is then not whole pairs and the steps run
    launched directly; a chunk of 12 runs as graphs of 6 pairs. Both give the
    single-step bits."""
    p = _short_grid()
    launch = dict(waves=2, rows=4, fuse_rows=8, fuse_steps=3, graph_chunk=9)
    kt = _kernel_times(p, dtype, launch, 2)
    assert kt["fused_steps"] == 2 and kt["fused_cells"] > 0, kt
    ref = run_gpu(p, NSTEPS, dtype, launch=dict(waves=2, rows=4))
    for lc in (launch, dict(launch, graph_chunk=12)):
        g = run_gpu(p, NSTEPS, dtype, launch=lc)
        assert np.array_equal(ref["fstar"], g["fstar"]), lc
        assert np.array_equal(ref["trace"], g["trace"]), lc
