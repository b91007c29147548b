"""The high-wavenumber filter (lbm_filter) against the oracle's filter, and
the stability it restores, on the GPU through the C ABI.

Tolerances as for the step: relative L2 1e-12 (FP64) and 1e-5 (FP32). An
FP32 case filters the FP32-rounded state on both sides."""
import numpy as np
import pytest

from workloads import BC_FREE0, BC_PERIODIC, BC_RIGID, Medium, Problem, Source
from oracle import stepper, theory as T
from oracle.filter import filter_state
from gpu_helpers import rel_l2

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def _box(nx, ny, bc=(BC_PERIODIC,) * 4, rr=-1, nu=0.25, tau=1.0):
    lam = 0.04 * T.lame_ratio(nu)
    return Problem(nx=nx, ny=ny, bc=bc, rigid_row=rr, medium=Medium("homogeneous", lam, 0.04, 1.0), tau=tau)


CASES = [
    ("periodic", lambda: _box(70, 40)),
    ("walls_and_rigid_row", lambda: _box(66, 50, bc=(BC_FREE0, BC_RIGID, BC_RIGID, BC_RIGID), rr=21)),
    ("periodic_x_walls_y", lambda: _box(300, 37, bc=(BC_FREE0, BC_RIGID, BC_PERIODIC, BC_PERIODIC))),
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_filter_matches_oracle(name, make, dtype):
    import torch
    import warnings
    from paper_2009_06404_amd import Solver
    p = make()
    rng = np.random.default_rng(len(name))
    f0 = rng.standard_normal((9, p.ny, p.nx))
    if dtype == "f32":
        f0 = f0.astype(np.float32).astype(np.float64)
    sigma = 0.04
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        s = Solver(p, dtype=dtype, trace_steps=1)
    try:
        s.set_state(0, torch.as_tensor(f0), 7)
        s.filter(sigma)
        got = s.state(0).double().cpu().numpy()
        assert s.time == 7
    finally:
        s.close()
    ref = filter_state(p, f0, sigma)
    e = rel_l2(got, ref)
    assert e <= TOL[dtype], e
    print(f"[filter] {name} {dtype}: {e:.2e}", flush=True)


def test_filter_batched_grids_and_between_graph_chunks():
    """Two grids in one context; a filter between captured chunks of steps
    leaves the run equal to the same run with direct launches, and both equal
    the oracle's steps and filters."""
    import torch
    import warnings
    from paper_2009_06404_amd import Solver
    probs = [_box(70, 40, nu=0.3).replace(sources=[Source(30.0, 20.0, 2.0, 0.0, 1.0, 1.0, 12.0, 16.0)]),
             _box(44, 52, bc=(BC_FREE0, BC_RIGID, BC_PERIODIC, BC_PERIODIC), nu=0.3)
             .replace(sources=[Source(20.0, 10.0, 2.0, 0.0, 1.0, 1.0, 12.0, 16.0)])]
    outs = []
    for chunk in (0, 8):
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            s = Solver(probs, dtype="f64", trace_steps=1, launch=dict(waves=1, rows=4, graph_chunk=chunk))
        try:
            for _ in range(3):
                s.step(16)
                s.filter(0.02)
            outs.append([s.state(g).double().cpu().numpy() for g in range(2)])
            torch.cuda.synchronize()
        finally:
            s.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
    for g, p in enumerate(probs):
        f, t = None, 0
        for _ in range(3):
            f = stepper.run(p, nsteps=16, t0=t, fstar_init=f, want_trace=False)["fstar"]
            t += 16
            f = filter_state(p, f, 0.02)
        assert rel_l2(outs[0][g], f) <= TOL["f64"]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_filter_stabilises_an_unstable_ratio(dtype):
    """nu = 0.37 at tau = 1 grows on the GPU as the von Neumann factor says;
    filtered every 4 steps with sigma = 0.02 it decays, and the filtered run
    equals the oracle's."""
    import torch
    import warnings
    from paper_2009_06404_amd import Solver, _lib as L
    p = _box(22, 22, nu=0.37)
    f0 = np.random.default_rng(7).standard_normal((9, 22, 22))
    if dtype == "f32":
        f0 = f0.astype(np.float32).astype(np.float64)
    res = {}
    for filt in (False, True):
        with warnings.catch_warnings(record=True) as rec:
            warnings.simplefilter("always")
            s = Solver(p, dtype=dtype, trace_steps=1)
        try:
            assert any("liblbm" in str(r.message) for r in rec)      # lbm_init warns
            s.set_state(0, torch.as_tensor(f0), 0)
            for _ in range(100):
                s.step(4)
                if filt:
                    s.filter(0.02)
            res[filt] = s.state(0).double().cpu().numpy()
            torch.cuda.synchronize()
        finally:
            s.close()
    n0 = np.linalg.norm(f0)
    assert np.linalg.norm(res[False]) > 2 * n0
    assert np.linalg.norm(res[True]) < 0.5 * n0
    assert L.lbm_vn_growth_filtered(0.37, 1.0, 0.02, 4, 33) <= 1.0 + 1e-9
    f, t = f0, 0
    for _ in range(100):
        f = stepper.run(p, nsteps=4, t0=t, fstar_init=f, want_trace=False)["fstar"]
        t += 4
        f = filter_state(p, f, 0.02)
    assert rel_l2(res[True], f) <= TOL[dtype]


def test_filter_refused_while_recording_and_bad_sigma():
    import warnings
    from paper_2009_06404_amd import Solver, _lib as L
    p = _box(40, 30)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        s = Solver(p, dtype="f32", trace_steps=10)
    try:
        for bad in (0.0, -0.1, 0.07):
            with pytest.raises(L.LBMError):
                s.filter(bad)
        s.adjoint_begin(10, 5)
        with pytest.raises(L.LBMError) as ei:
            s.filter(0.01)
        assert ei.value.code == L.LBM_E_STATE
        s.step(10)
        s.filter(0.01)        # the recording is complete: allowed
    finally:
        s.close()


def test_filter_throughput_full_size():
    """One filter pass over the 4096^2 FP32 state: timed with HIP events on
    the solver's stream (a measurement; the bar is only that it keeps more
    than 3.5 TB/s of its 72 algorithmic bytes per cell)."""
    import torch
    import warnings
    import workloads as w
    from paper_2009_06404_amd import Solver
    p = w.plain_large(nsteps=2)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        s = Solver(p, dtype="f32", trace_steps=4)
    try:
        s.step(2)
        for _ in range(3):
            s.filter(0.01)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            s.filter(0.01)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 20
        gbs = 72 * p.nx * p.ny / (ms / 1e3) / 1e9
        print(f"[filter] 4096^2 f32: {ms * 1e3:.1f} us per pass, {gbs:.0f} GB/s algorithmic", flush=True)
        assert gbs > 3500
        assert s.check_finite()
    finally:
        s.close()
