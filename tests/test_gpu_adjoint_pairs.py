"""GPU parity of the adjoint's two-step path (launch fuse_rows > 0): steps t
and t-1 of a checkpoint segment in one pass of the two-step adjoint kernel
over blocks clear of walls, sources and receivers, with the general adjoint
kernel taking the other cells one step at a time (its first step also over
the blocks' border strips).

Compared, as for the single-step adjoint: the adjoint state at t0, dL/dkappa
per cell and dL/damp per source against the FP64 oracle adjoint (relative L2,
FP64 1e-11, FP32 1e-4), and against the single-step GPU adjoint of the same
launch without pairs: the state and dL/dkappa bit for bit (every adjoint
kernel forms a cell's terms in the same order), dL/damp to 1e-12 (its FP64
atomic sums come in another order). Segments of odd length and adjoint steps
taken in odd chunks leave single steps between the pairs; every run checks
through the timed adjoint step that its two-step kernel ran.
"""
import numpy as np
import pytest

from workloads import BC_FREE, BC_FREE0, BC_PERIODIC, BC_RIGID, Medium, Problem, Source
from workloads.problem import default_sponge_profile
from oracle import stepper
from gpu_helpers import rel_l2

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-11, "f32": 1e-4}


def _problem(bc, rr, nx, ny, seed, medium="field", tau=0.9, sponge=6, rec_rows=(0, 101)):
    rng = np.random.default_rng(seed)
    if medium == "field":
        mu = rng.uniform(0.036, 0.044, (ny, nx))
        nu = rng.uniform(0.15, 0.3, (ny, nx))
        rho = rng.uniform(0.9, 1.1, (ny, nx))
    elif medium == "layers":        # moduli constant along rows: a per-row kappa
        mu = np.repeat(rng.uniform(0.036, 0.044, (ny, 1)), nx, axis=1)
        nu = np.repeat(rng.uniform(0.15, 0.3, (ny, 1)), nx, axis=1)
        rho = np.repeat(rng.uniform(0.9, 1.1, (ny, 1)), nx, axis=1)
    else:                           # homogeneous: one kappa
        mu = np.full((ny, nx), 0.04)
        nu = np.full((ny, nx), 0.25)
        rho = np.ones((ny, nx))
    lam = 2 * nu * mu / (1 - 2 * nu)
    prof = default_sponge_profile(sponge)
    thick = (0, sponge, sponge, 0)
    src = [Source(nx * 0.15, ny * 0.2, 2.0, 0.3, 0.9, 1.0, 12.0, 16.0),
           Source(nx * 0.8, ny * 0.75, 1.5, 0.6, 0.8, 0.8, 10.0, 14.0)]
    rec = [(x, r) for r in rec_rows for x in range(r % 5, nx, 5)]
    return Problem(nx=nx, ny=ny, bc=bc, medium=Medium("field", lam, mu, rho), tau=tau,
                   rigid_row=rr, sponge_thick=thick,
                   sponge_profiles=tuple(prof if t else None for t in thick),
                   sources=src, receivers=np.asarray(rec, np.int32), comp_mask=3, nsteps=0)


def _gpu_adjoint(probs, T, seg, dtype, residuals, launch, chunks, resident=0):
    """The adjoint through the C ABI; every other chunk through the timed
    adjoint step, whose kernel counts come back with the results."""
    import torch
    from paper_2009_06404_amd import Solver
    s = Solver(probs, dtype=dtype, trace_steps=T, launch=launch)
    fused_launches = 0
    try:
        s.adjoint_begin(T, seg, resident_steps=resident)
        s.step(T)
        keep = []
        for g, p in enumerate(probs):
            res = torch.as_tensor(residuals[g], dtype=s.tdtype, device=s.device).contiguous()
            gk = torch.zeros((p.ny, p.nx), dtype=torch.float64, device=s.device)
            ga = torch.zeros(max(len(p.sources), 1), dtype=torch.float64, device=s.device)
            s.adjoint_set_io(g, res, gk, ga)
            keep.append((res, gk, ga))
        for i, n in enumerate(chunks):
            if i % 2:
                kt = s.adjoint_step_timed(n)
                if kt["fused_ms"] > 0:
                    assert kt["fused_cells"] > 0
                    fused_launches += 1
            else:
                s.adjoint_step(n)
        assert s.adjoint_time == 0
        out = [{"adj": s.adjoint_state(g).double().cpu().numpy(),
                "grad_kappa": keep[g][1].cpu().numpy(),
                "grad_amp": keep[g][2].cpu().numpy()[:len(p.sources)],
                "trace": s.traces[g].double().cpu().numpy()}
               for g, p in enumerate(probs)]
        torch.cuda.synchronize()
    finally:
        s.close()
    return out, fused_launches


def _errors(a, b):
    return tuple(rel_l2(a[k], b[k]) for k in ("adj", "grad_kappa", "grad_amp"))


def _check(what, dtype, got, ref, single):
    e_ref = _errors(got, ref)
    e_one = _errors(got, single)
    print(f"[adjoint pairs] {what}: vs oracle state {e_ref[0]:.2e} grad_kappa {e_ref[1]:.2e} "
          f"grad_amp {e_ref[2]:.2e}; vs single steps {e_one[0]:.2e} {e_one[1]:.2e} "
          f"{e_one[2]:.2e}", flush=True)
    assert np.linalg.norm(ref["adj"]) > 0 and np.linalg.norm(ref["grad_kappa"]) > 0
    assert max(e_ref) <= TOL[dtype], (what, e_ref)
    assert np.array_equal(got["adj"], single["adj"]), what
    assert np.array_equal(got["grad_kappa"], single["grad_kappa"]), what
    assert e_one[2] <= 1e-12, (what, e_one)


CASES = [
    ("free_rigid_interface", (BC_FREE, BC_RIGID, BC_PERIODIC, BC_PERIODIC), 150),
    ("free0_rigid_sides", (BC_FREE0, BC_FREE0, BC_RIGID, BC_RIGID), -1),
    ("periodic", (BC_PERIODIC,) * 4, -1),
]
LAUNCHES = [dict(waves=2, rows=8, fuse_rows=8), dict(waves=4, rows=4, fuse_rows=13)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name,bc,rr", CASES, ids=[c[0] for c in CASES])
def test_adjoint_pairs_match_oracle_and_single_steps(name, bc, rr, dtype):
    """A 300 x 200 grid: cell-wise moduli, two sources, receivers along the
    top row and through row 101 (whose neighbourhood goes to the general
    kernel), segments of 7 steps; 128- and 256-column blocks."""
    p = _problem(bc, rr, 300, 200, seed=len(name))
    T, seg = 40, 7
    res = np.random.default_rng(5).standard_normal((T, p.nrec, p.ncomp))
    ref = stepper.adjoint(p, nsteps=T, residual=res)
    for launch in LAUNCHES:
        single = dict(launch, fuse_rows=0)
        one, _ = _gpu_adjoint([p], T, seg, dtype, [res], single, [T])
        got, nf = _gpu_adjoint([p], T, seg, dtype, [res], launch, [3, 17, 9, 11])
        assert nf > 0, "the two-step adjoint kernel did not run"
        _check(f"{name} {launch} {dtype}", dtype, got[0], ref, one[0])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("medium", ["layers", "homogeneous"])
def test_adjoint_pairs_per_row_and_scalar_moduli(medium, dtype):
    """The two-step adjoint kernel reads kappa from its per-row table (moduli
    constant along rows) or as one value (homogeneous medium)."""
    p = _problem((BC_FREE0, BC_RIGID, BC_PERIODIC, BC_PERIODIC), -1, 260, 120, seed=3,
                 medium=medium, rec_rows=(0,))
    T, seg = 30, 10
    res = np.random.default_rng(6).standard_normal((T, p.nrec, p.ncomp))
    ref = stepper.adjoint(p, nsteps=T, residual=res)
    launch = dict(waves=2, rows=8, fuse_rows=16)
    one, _ = _gpu_adjoint([p], T, seg, dtype, [res], dict(launch, fuse_rows=0), [T])
    got, nf = _gpu_adjoint([p], T, seg, dtype, [res], launch, [4, 26])
    assert nf > 0
    _check(f"{medium} {dtype}", dtype, got[0], ref, one[0])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batched_adjoint_pairs_and_partial_blocks(dtype):
    """Three grids of different widths in one context (blocks narrower than
    the launch's at the right edge of non-periodic grids), with 512-column
    blocks asked for (256 in FP64)."""
    p1 = _problem((BC_FREE, BC_RIGID, BC_PERIODIC, BC_PERIODIC), 40, 530, 90, seed=1,
                  rec_rows=(0,))
    p2 = _problem((BC_PERIODIC,) * 4, -1, 300, 64, seed=2, rec_rows=(0, 33))
    p3 = _problem((BC_FREE0, BC_FREE0, BC_RIGID, BC_RIGID), -1, 1100, 50, seed=3, rec_rows=(0,))
    probs = [p1, p2, p3]
    T, seg = 24, 12
    rng = np.random.default_rng(9)
    res = [rng.standard_normal((T, p.nrec, p.ncomp)) for p in probs]
    launch = dict(waves=8, rows=4, fuse_rows=6)
    one, _ = _gpu_adjoint(probs, T, seg, dtype, res, dict(launch, fuse_rows=0), [T])
    got, nf = _gpu_adjoint(probs, T, seg, dtype, res, launch, [5, 19])
    assert nf > 0
    for g, p in enumerate(probs):
        ref = stepper.adjoint(p, nsteps=T, residual=res[g])
        _check(f"batched grid {g} ({p.nx}x{p.ny}) {dtype}", dtype, got[g], ref, one[g])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("fuse_rows", [8, 0], ids=["pairs", "single_steps"])
def test_kept_densities_equal_the_recompute(fuse_rows, dtype):
    """A workspace beyond the minimum keeps the densities of the last
    segments from the recorded forward run (written as it goes, receivers
    recorded as usual), and the adjoint skips their recompute: traces, adjoint
    state and dL/dkappa are those of the run that recomputes every segment,
    bit for bit; dL/damp to rounding (pairs may then span two kept segments).
    Kept: none, the last (short) segment, three segments, all."""
    p = _problem((BC_FREE, BC_RIGID, BC_PERIODIC, BC_PERIODIC), 150, 300, 200, seed=21)
    T, seg = 40, 7
    res = np.random.default_rng(8).standard_normal((T, p.nrec, p.ncomp))
    launch = dict(waves=2, rows=8, fuse_rows=fuse_rows)
    base, _ = _gpu_adjoint([p], T, seg, dtype, [res], launch, [3, 37])
    for resident in (5, 19, T):
        got, _ = _gpu_adjoint([p], T, seg, dtype, [res], launch, [3, 37], resident=resident)
        for k in ("trace", "adj", "grad_kappa"):
            assert np.array_equal(got[0][k], base[0][k]), (resident, k)
        e = rel_l2(got[0]["grad_amp"], base[0]["grad_amp"])
        print(f"[kept densities] {dtype} fuse_rows={fuse_rows} resident={resident}: bitwise; "
              f"dL/damp {e:.1e}", flush=True)
        assert e <= 1e-12, (resident, e)


def test_gradient_matches_central_differences_of_the_gpu_misfit():
    """dL/dlambda and dL/dmu of the GPU adjoint (two-step path, FP64) against
    central differences of the GPU forward's own misfit, at six cells within
    the wavefield's reach: beside the sources, under the free surface, near
    the receiver row through the grid. Independent of the oracle: both sides
    come from the kernels."""
    import torch
    from paper_2009_06404_amd import Solver
    p = _problem((BC_FREE0, BC_RIGID, BC_PERIODIC, BC_PERIODIC), -1, 300, 100, seed=31,
                 rec_rows=(0, 50))
    T, seg = 60, 13
    launch = dict(waves=2, rows=8, fuse_rows=8)
    lam, mu, rho = p.medium.full(p.ny, p.nx)
    d_obs = np.random.default_rng(2).standard_normal((T, p.nrec, p.ncomp)) * 1e-3

    def misfit(lam_, mu_):
        q = p.replace(medium=Medium("field", lam_, mu_, rho))
        s = Solver(q, dtype="f64", trace_steps=T, launch=launch)
        try:
            s.step(T)
            m, _ = s.misfit(0, torch.as_tensor(d_obs))
            return float(m.item())
        finally:
            s.close()

    s = Solver(p, dtype="f64", trace_steps=T, launch=launch)
    try:
        s.adjoint_begin(T, seg)
        s.step(T)
        _, res = s.misfit(0, torch.as_tensor(d_obs))
        gk = torch.zeros((p.ny, p.nx), dtype=torch.float64, device=s.device)
        s.adjoint_set_io(0, res, gk, None)
        kt = s.adjoint_step_timed(T)
        assert kt["fused_cells"] > 0
        gl = torch.zeros_like(gk)
        gm = torch.zeros_like(gk)
        s.lame_gradient(0, gk, gl, gm)
        gl, gm = gl.cpu().numpy(), gm.cpu().numpy()
    finally:
        s.close()
    # within the wavefield's reach over 60 steps: near the sources (45, 20)
    # and (240, 75), under the surface, beside the receiver row 50, in a block
    cells = [(45, 22), (30, 6), (60, 42), (230, 80), (246, 68), (240, 56)]
    for x, y in cells:
        for name, field, g in (("lambda", lam, gl), ("mu", mu, gm)):
            h = 1e-5 * field[y, x]
            plus, minus = field.copy(), field.copy()
            plus[y, x] += h
            minus[y, x] -= h
            if name == "lambda":
                fd = (misfit(plus, mu) - misfit(minus, mu)) / (2 * h)
            else:
                fd = (misfit(lam, plus) - misfit(lam, minus)) / (2 * h)
            e = abs(g[y, x] - fd) / max(abs(fd), 1e-30)
            print(f"[central differences] dL/d{name} at ({x},{y}): adjoint {g[y, x]:.6e}, "
                  f"differences {fd:.6e}, rel {e:.1e}", flush=True)
            assert abs(fd) > 0 and e <= 1e-5, (name, x, y, g[y, x], fd)
