"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle, element
by element on the same seeded inputs.

Tolerances (relative L2 per field, per state and per trace set): FP64 1e-12,
FP32 1e-5 against the FP64 oracle.
"""
import numpy as np
import pytest

import workloads as w
from workloads import BC_FREE, BC_FREE0, BC_PERIODIC, BC_RIGID, Medium, Problem, Source
from oracle import stepper
from gpu_helpers import compare, rel_l2, run_gpu

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def _oracle(p, nsteps, fstar_init=None, t0=0):
    return stepper.run(p, nsteps=nsteps, fstar_init=fstar_init, t0=t0)


def _print(name, worst):
    print(f"[parity] {name}: worst rel L2 {worst:.3e}", flush=True)


def test_plain_small_full_config_f64():
    """128x128 periodic box, nu = 0.25, x-force, 16-station ring, 600 steps:
    the full small configuration, FP64."""
    p = w.plain_small()
    g = run_gpu(p, p.nsteps, "f64")
    worst = compare(g, _oracle(p, p.nsteps), TOL["f64"], "plain_small f64")
    _print("plain_small f64 600 steps", worst)


def test_plain_small_f32():
    p = w.plain_small()
    g = run_gpu(p, p.nsteps, "f32")
    worst = compare(g, _oracle(p, p.nsteps), TOL["f32"], "plain_small f32")
    _print("plain_small f32 600 steps", worst)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_plain_large_reduced(dtype):
    """Free surface, sponges, rigid bottom, nu = 0.33 (elastic force active),
    surface receivers: the large configuration at 256x256."""
    p = w.plain_large(n=256, nsteps=700, sponge=24, src_depth=20)
    g = run_gpu(p, p.nsteps, dtype)
    worst = compare(g, _oracle(p, p.nsteps), TOL[dtype], f"plain_large/256 {dtype}")
    _print(f"plain_large 256 {dtype}", worst)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_free_surface_as_printed_short_run(dtype):
    """The printed free-surface rule (linear extrapolation), over a run short
    enough that its growing surface modes stay below the tolerance."""
    p = w.plain_large(n=256, nsteps=110, sponge=24, src_depth=20, top_bc=BC_FREE)
    g = run_gpu(p, p.nsteps, dtype)
    worst = compare(g, _oracle(p, p.nsteps), TOL[dtype], f"printed free surface {dtype}")
    _print(f"printed free surface 256 {dtype}", worst)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_hbm_scale_reduced(dtype):
    """8 layers (per-row kappa), rigid internal interface, 3 sources."""
    p = w.hbm_scale(n=256, nsteps=500, sponge=32)
    assert p.rigid_row > 0
    p = p.replace(receivers=np.array([[x, 0] for x in range(0, 256, 5)] +
                                     [[x, p.rigid_row - 1] for x in range(3, 256, 7)] +
                                     [[x, p.rigid_row] for x in range(1, 256, 9)], np.int32),
                  comp_mask=3)
    g = run_gpu(p, p.nsteps, dtype)
    worst = compare(g, _oracle(p, p.nsteps), TOL[dtype], f"hbm_scale/256 {dtype}")
    _print(f"hbm_scale 256 {dtype}", worst)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_field_medium_shots_batched(dtype):
    """Per-cell kappa (random-field medium) with several shots in one batch."""
    probs = w.adjoint_shots(n=128, shots=3, nsteps=300, sponge=16)
    gs = run_gpu(probs, 300, dtype)
    for s, (p, g) in enumerate(zip(probs, gs)):
        worst = compare(g, _oracle(p, 300), TOL[dtype], f"shot {s} {dtype}")
        _print(f"field medium shot {s} {dtype}", worst)


def test_batched_uneven_grids_match_oracle_and_single_runs():
    """Grids of uneven, ragged sizes in one launch: each matches the oracle and
    is bitwise equal to the same grid run alone."""
    probs = w.batched_shots(count=4, nsteps=250, sponge=16, sides=[70, 96, 131, 200])
    probs = [p.replace(receivers=np.array([[x, 0] for x in range(0, p.nx, 3)], np.int32),
                       comp_mask=2) for p in probs]
    gb = run_gpu(probs, 250, "f32")
    for p, g in zip(probs, gb):
        compare(g, _oracle(p, 250), TOL["f32"], f"batched {p.nx}")
        single = run_gpu(p, 250, "f32")
        assert np.array_equal(single["fstar"], g["fstar"])
        assert np.array_equal(single["mom"], g["mom"])
        assert np.array_equal(single["trace"], g["trace"])


def _feature_problem(nx=150, ny=77):
    prof = w.default_sponge_profile(9)
    lam = np.linspace(0.01, 0.05, ny)
    mu = np.full(ny, 0.04)
    return Problem(nx=nx, ny=ny, bc=(BC_FREE, BC_RIGID, BC_PERIODIC, BC_PERIODIC),
                   medium=Medium("layered", lam, mu, np.ones(ny)), tau=0.9, rigid_row=40,
                   sponge_thick=(0, 9, 7, 9), sponge_profiles=(None, prof, prof[:7] * 2, prof),
                   sources=[Source(20.0, 5.0, 2.5, 0.3, 1.0, 1.0, 14.0, 10.0),
                            Source(140.0, 60.0, 2.0, -1.0, 0.2, 0.5, 10.0, 12.0)],
                   receivers=np.array([[0, 0], [149, 0], [75, 39], [75, 40], [3, 76], [3, 76]], np.int32),
                   comp_mask=3, dtype="f64")


def test_launch_configurations_agree_bitwise():
    """Ragged grid (nx not a multiple of 64, odd ny), every wall type: all tile
    shapes give bitwise the same state, and one of them matches the oracle."""
    p = _feature_problem()
    ref = None
    for waves in (1, 2, 4):
        for rows in (1, 5, 64):
            for prefetch, split in ((1, 1), (2, 0), (2, 1)):
                cfg = dict(waves=waves, rows=rows, prefetch=prefetch, split=split)
                g = run_gpu(p, 60, "f64", launch=cfg)
                if ref is None:
                    ref = g
                    compare(g, _oracle(p, 60), TOL["f64"], "feature problem")
                else:
                    assert np.array_equal(ref["fstar"], g["fstar"]), cfg
                    assert np.array_equal(ref["trace"], g["trace"]), cfg


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_interior_kernel_split_is_bitwise_neutral(dtype):
    """A periodic box large enough to have interior tiles: the run with the
    interior/general split equals the run with one kernel, and the oracle."""
    p = w.plain_large(n=192, nsteps=150, sponge=20, src_depth=30)
    a = run_gpu(p, 150, dtype, launch=dict(waves=1, rows=8, split=1))
    b = run_gpu(p, 150, dtype, launch=dict(waves=1, rows=8, split=0))
    c = run_gpu(p, 150, dtype, launch=dict(waves=2, rows=4, split=1, pair=1))
    # the general kernel on the second stream, with direct launches and inside
    # captured graphs (fork and join as graph edges), and without the overlap
    d = run_gpu(p, 150, dtype, launch=dict(waves=1, rows=8, split=1, overlap=0))
    e = run_gpu(p, 150, dtype, launch=dict(waves=1, rows=8, split=1, overlap=1, graph_chunk=10))
    for other in (b, c, d, e):
        assert np.array_equal(a["fstar"], other["fstar"])
        assert np.array_equal(a["trace"], other["trace"])
    compare(a, _oracle(p, 150), TOL[dtype], f"split {dtype}")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_timed_steps_equal_plain_steps(dtype):
    """lbm_step_timed advances the state exactly like lbm_step, and its two
    kernels' tile lists cover every cell once."""
    import torch
    from paper_2009_06404_amd import Solver
    p = w.plain_large(n=320, nsteps=40, sponge=20, src_depth=30)
    outs = []
    for timed in (False, True):
        s = Solver(p, dtype=dtype, trace_steps=40, launch=dict(waves=2, rows=4, split=1))
        try:
            s.step(10)
            if timed:
                kt = s.step_timed(30)
            else:
                s.step(30)
            outs.append((s.state().double().cpu().numpy(), s.traces[0].double().cpu().numpy()))
            assert s.time == 40
            torch.cuda.synchronize()
        finally:
            s.close()
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    assert kt["steps"] == 30
    assert kt["interior_cells"] > 0 and kt["general_cells"] > 0
    assert kt["interior_cells"] + kt["general_cells"] == p.nx * p.ny
    assert kt["interior_ms"] > 0 and kt["general_ms"] > 0


BC_CASES = [
    ("periodic", (BC_PERIODIC,) * 4, -1),
    ("free_rigid", (BC_FREE, BC_RIGID, BC_PERIODIC, BC_PERIODIC), -1),
    ("free0_rigid", (BC_FREE0, BC_RIGID, BC_PERIODIC, BC_PERIODIC), 7),
    ("free0_free0_rigid_sides", (BC_FREE0, BC_FREE0, BC_RIGID, BC_RIGID), -1),
    ("rigid_box", (BC_RIGID,) * 4, -1),
    ("free_free_rigid_sides", (BC_FREE, BC_FREE, BC_RIGID, BC_RIGID), 6),
    ("rigid_free", (BC_RIGID, BC_FREE, BC_PERIODIC, BC_PERIODIC), 5),
    ("periodic_y_rigid_x", (BC_PERIODIC, BC_PERIODIC, BC_RIGID, BC_RIGID), -1),
]


@pytest.mark.parametrize("name,bc,rr", BC_CASES, ids=[c[0] for c in BC_CASES])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_random_state_every_link(name, bc, rr, dtype):
    """From a random state every population and every wall link is active."""
    rng = np.random.default_rng(7)
    nx, ny = 67, 13
    lam = rng.uniform(0.0, 0.06, size=(ny, nx))
    mu = rng.uniform(0.035, 0.045, size=(ny, nx))
    prof = w.default_sponge_profile(3, 0.3)
    p = Problem(nx=nx, ny=ny, bc=bc, medium=Medium("field", lam, mu, rng.uniform(0.8, 1.2, (ny, nx))),
                tau=0.8, rigid_row=rr, sponge_thick=(2, 3, 3, 2),
                sponge_profiles=(prof, prof, prof, prof),
                sources=[Source(33.0, 6.0, 2.0, 0.6, -0.8, 1.0, 6.0, 2.0)],
                receivers=np.array([[x, y] for y in range(ny) for x in range(0, nx, 11)], np.int32),
                comp_mask=3)
    f0 = rng.normal(size=(9, ny, nx))
    if dtype == "f32":
        f0 = f0.astype(np.float32).astype(np.float64)
    g = run_gpu(p, 6, dtype, state=f0, t0=3)
    ref = _oracle(p, 6, fstar_init=f0, t0=3)
    compare(g, ref, TOL[dtype], f"random state {name} {dtype}")


def test_minimal_grid_and_zero_steps():
    p = Problem(nx=3, ny=3, bc=(BC_PERIODIC,) * 4, medium=Medium("homogeneous", 0.02, 0.04, 1.0),
                sources=[Source(1.0, 1.0, 1.0, 1.0, 0.0, 1.0, 4.0, 2.0)],
                receivers=np.array([[1, 1]], np.int32), comp_mask=3, dtype="f64")
    g = run_gpu(p, 9, "f64")
    # P_xy is odd in y about the source row and 4e-6 of the largest field here
    compare(g, _oracle(p, 9), TOL["f64"], "3x3", near_zero=("P_xy",))
    # zero steps: the state is the rest state; the fields at t = 0 already
    # carry the source's half-step contribution to j (j = m + S/2)
    g0 = run_gpu(p, 0, "f64")
    assert np.all(g0["fstar"] == 0)
    compare(g0, _oracle(p, 0), TOL["f64"], "3x3 t=0", near_zero=("P_xy",))


def test_restart_and_graph_are_bitwise():
    """n steps in one call == k steps, get/set state, n-k steps; and the
    HIP-graph-captured loop == direct launches."""
    import torch
    from paper_2009_06404_amd import Solver
    p = _feature_problem().replace(dtype="f32")
    a = run_gpu(p, 40, "f32")
    s = Solver(p, dtype="f32", trace_steps=40)
    s.step(17)
    st = s.state(0).clone()
    s.close()
    s2 = Solver(p, dtype="f32", trace_steps=40)
    s2.set_state(0, st, 17)
    s2.step(23)
    fs = s2.state(0).double().cpu().numpy()
    s2.close()
    assert np.array_equal(fs, a["fstar"])
    g = run_gpu(p, 40, "f32", launch=dict(waves=2, rows=16, graph_chunk=8))
    d = run_gpu(p, 40, "f32", launch=dict(waves=2, rows=16, graph_chunk=0))
    assert np.array_equal(g["fstar"], d["fstar"])
    assert np.array_equal(g["trace"], d["trace"])
    torch.cuda.synchronize()


def test_plain_large_full_size_random_state_f32():
    """The large configuration at its full 4096x4096 size, in the default
    launch configuration, from a random state (all cells active): 12 steps
    against the oracle, all fields, state and the 4096 surface traces."""
    p = w.plain_large()
    rng = np.random.default_rng(11)
    f0 = rng.standard_normal(size=(9, p.ny, p.nx), dtype=np.float32).astype(np.float64) * 1e-3
    g = run_gpu(p, 12, "f32", state=f0, t0=50)
    ref = _oracle(p, 12, fstar_init=f0, t0=50)
    worst = compare(g, ref, TOL["f32"], "plain_large 4096 random state")
    _print("plain_large 4096 f32 random state 12 steps", worst)


def test_hbm_scale_full_size_light_cone_windows():
    """The 16384^2 FP32 HBM-scale configuration (8 layers, rigid interface,
    3 sources, 128-cell sponges) at full size in its default launch shape,
    80 steps from rest. A cell's value after n steps depends only on cells
    within 2n (Chebyshev) -- one cell per step from streaming, one from the
    density-gradient stencil -- so every field is exactly zero outside the
    sources' reach (9 sigma + 2n + 1), and inside a window around each source
    the oracle reproduces the fields on a small periodic box carrying the
    same medium rows (the fields never reach the box's edges)."""
    import torch
    from paper_2009_06404_amd import Solver
    p = w.hbm_scale()
    n = 80
    R = 200
    reach = int(np.ceil(9 * 3.0)) + 2 * n + 1
    assert reach < R
    lam_r, mu_r, rho_r = p.medium.rows(p.ny)
    s = Solver(p, dtype="f32", trace_steps=1)
    try:
        s.step(n)
        mom = s.moments(0)
        torch.cuda.synchronize()
        mask = torch.ones((p.ny, p.nx), dtype=torch.bool, device=mom.device)
        for q in p.sources:
            xs, ys = int(q.x), int(q.y)
            x0, x1, y0, y1 = xs - R, xs + R + 1, ys - R, ys + R + 1
            assert 128 < x0 and x1 < p.nx - 128 and 0 < y0 and y1 < p.rigid_row
            mask[y0:y1, x0:x1] = False
            win = Problem(nx=x1 - x0, ny=y1 - y0, bc=(BC_PERIODIC,) * 4,
                          medium=Medium("layered", lam_r[y0:y1], mu_r[y0:y1], rho_r[y0:y1]),
                          tau=p.tau, sources=[Source(q.x - x0, q.y - y0, q.sigma, q.dir_x, q.dir_y,
                                                     q.amp, q.period, q.t0)])
            ref = stepper.run(win, nsteps=n, want_trace=False)["mom"]
            got = mom[:, y0:y1, x0:x1].double().cpu().numpy()
            floor = 1e-3 * max(np.linalg.norm(ref[k]) for k in range(6))
            for k in range(6):
                e = np.linalg.norm(got[k] - ref[k]) / max(np.linalg.norm(ref[k]), floor)
                assert e <= TOL["f32"], (q.x, q.y, k, e)
            _print(f"hbm_scale window at ({xs}, {ys})", e)
        outside = torch.where(mask, mom.abs().amax(dim=0), torch.zeros((), device=mom.device))
        assert float(outside.max().item()) == 0.0
    finally:
        s.close()


def test_init_reports_the_stability_window():
    """lbm_init returns LBM_WARN_UNSTABLE (the context is still made) when a
    bulk mode grows for the media's Poisson ratios at tau, or when an edge
    uses the printed free-surface rule; lbm_stability reports the factor."""
    import warnings
    from paper_2009_06404_amd import Solver, _lib as L
    from oracle import theory as T
    base = w.plain_small(n=64, nsteps=1)
    cases = []
    for nu, tau, bc in ((0.25, 1.0, base.bc), (0.33, 1.0, base.bc), (0.37, 1.0, base.bc),
                        (0.0, 0.55, base.bc), (0.25, 1.0, (BC_FREE, BC_RIGID, BC_PERIODIC, BC_PERIODIC))):
        lam = 0.04 * T.lame_ratio(nu)
        cases.append((base.replace(medium=Medium("homogeneous", lam, 0.04, 1.0), tau=tau, bc=bc), nu, tau,
                      bc == base.bc))
    for p, nu, tau, bulk_only in cases:
        with warnings.catch_warnings(record=True) as rec:
            warnings.simplefilter("always")
            s = Solver(p, dtype="f32", trace_steps=1)
        try:
            g, stable = L.lbm_stability(s.ctx)
        finally:
            s.close()
        expect = T.max_growth(nu, tau, n=33) <= 1.0 + 1e-6 and bulk_only
        assert stable == expect, (nu, tau, g)
        assert abs(g - T.max_growth(nu, tau, n=33)) < 1e-7
        assert (len([r for r in rec if "liblbm" in str(r.message)]) > 0) == (not expect)
    # a cell-wise medium: its sampled range decides
    rng = np.random.default_rng(3)
    mu = np.full((48, 64), 0.04)
    nu_f = rng.uniform(0.3, 0.39, (48, 64))
    lam = 2 * nu_f * mu / (1 - 2 * nu_f)
    p = base.replace(nx=64, ny=48, medium=Medium("field", lam, mu, np.ones((48, 64))), tau=1.0,
                     sources=[], receivers=np.zeros((0, 2), np.int32))
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        s = Solver(p, dtype="f32", trace_steps=1)
    try:
        g, stable = L.lbm_stability(s.ctx)
    finally:
        s.close()
    assert not stable and g >= T.max_growth(float(nu_f.max()), 1.0, n=33) - 1e-3


def test_batched_full_size_sampled_grids():
    """The batched configuration at full size (512 grids of side 256..2048,
    860 M cells, FP32) in the launch the benchmark times, 8 steps (four pairs
    on the two-step path). The 8 smallest and the 2 largest grids start from
    random states, the others from rest. The grids are independent, so each
    sampled grid must match the oracle run on that grid alone: fields and
    state. Every grid's state stays finite."""
    import torch
    import bench
    from paper_2009_06404_amd import Solver
    probs = w.batched_shots()
    order = np.argsort([p.nx for p in probs], kind="stable")
    pick = [int(g) for g in list(order[:8]) + list(order[-2:])]
    starts = {}
    s = Solver(probs, dtype="f32", trace_steps=1, launch=dict(bench.BATCHED_LAUNCH))
    try:
        assert s.launch()["fuse_rows"] > 0
        for g in pick:
            p = probs[g]
            rng = np.random.default_rng(100 + g)
            f0 = rng.standard_normal(size=(9, p.ny, p.nx), dtype=np.float32)
            starts[g] = f0.astype(np.float64) * 1e-3
            s.set_state(g, torch.as_tensor(starts[g], dtype=torch.float32), 0)
        s.step(8)
        got = {g: {"mom": s.moments(g).double().cpu().numpy(),
                   "fstar": s.state(g).double().cpu().numpy(), "trace": None} for g in pick}
        assert s.check_finite()
    finally:
        s.close()
    worst = 0.0
    for g in pick:
        ref = stepper.run(probs[g], nsteps=8, fstar_init=starts[g], want_trace=False)
        worst = max(worst, compare(got[g], ref, TOL["f32"], f"batched grid {g} ({probs[g].nx}^2)"))
    _print("batched_shots full size, 10 sampled grids, 8 steps", worst)
