"""GPU parity of the discrete adjoint (lbm_adjoint_* through the C ABI)
against the FP64 oracle adjoint, on the same seeded inputs.

Compared: the adjoint state dL/df(t0) after stepping back to the start, the
per-cell dL/dkappa and the per-source dL/damp. Tolerances (relative L2):
FP64 1e-11; FP32 1e-4 (an FP32 forward and adjoint against the FP64
oracle). Every observed-data input comes from the oracle.
"""
import numpy as np
import pytest

from workloads import BC_FREE, BC_FREE0, BC_PERIODIC, BC_RIGID, Medium, Problem, Source
from workloads.problem import default_sponge_profile
import workloads as w
from oracle import stepper
from gpu_helpers import rel_l2

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-11, "f32": 1e-4}

BC_CASES = [
    ("periodic", (BC_PERIODIC,) * 4, -1),
    ("free_rigid_interface", (BC_FREE, BC_RIGID, BC_PERIODIC, BC_PERIODIC), 17),
    ("free0_both_rigid_sides", (BC_FREE0, BC_FREE0, BC_RIGID, BC_RIGID), -1),
    ("rigid_box_interface", (BC_RIGID,) * 4, 9),
    ("rigid_top_free_bottom", (BC_RIGID, BC_FREE, BC_PERIODIC, BC_PERIODIC), -1),
]


def _problem(bc, rr, nx=70, ny=40, seed=0, tau=0.9, sponge=6):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(0.036, 0.044, (ny, nx))
    nu = rng.uniform(0.15, 0.3, (ny, nx))
    lam = 2 * nu * mu / (1 - 2 * nu)
    rho = rng.uniform(0.9, 1.1, (ny, nx))
    prof = default_sponge_profile(sponge)
    thick = (0, sponge, sponge, 0)
    src = [Source(nx * 0.3, ny * 0.4, 2.0, 0.0, 1.0, 1.0, 12.0, 16.0),
           Source(nx * 0.7, ny * 0.6, 1.5, 0.6, 0.8, 0.8, 10.0, 14.0)]
    rec = [(x, 0) for x in range(0, nx, 3)] + [(x, ny // 2) for x in range(1, nx, 7)] + [(5, 0)]
    return Problem(nx=nx, ny=ny, bc=bc, medium=Medium("field", lam, mu, rho), tau=tau,
                   rigid_row=rr, sponge_thick=thick,
                   sponge_profiles=tuple(prof if t else None for t in thick),
                   sources=src, receivers=np.asarray(rec, np.int32), comp_mask=3, nsteps=0)


def _gpu_adjoint(probs, T, seg, dtype, residuals, launch=None, chunks=None):
    import torch
    from paper_2009_06404_amd import Solver
    s = Solver(probs, dtype=dtype, trace_steps=T, launch=launch)
    try:
        s.adjoint_begin(T, seg)
        s.step(T)
        td = s.tdtype
        keep = []
        for g, p in enumerate(probs):
            res = torch.as_tensor(residuals[g], dtype=td, device=s.device).contiguous()
            gk = torch.zeros((p.ny, p.nx), dtype=torch.float64, device=s.device)
            ga = torch.zeros(max(len(p.sources), 1), dtype=torch.float64, device=s.device)
            s.adjoint_set_io(g, res, gk, ga)
            keep.append((res, gk, ga))
        for n in (chunks or [T]):
            s.adjoint_step(n)
        assert s.adjoint_time == 0
        out = []
        for g, p in enumerate(probs):
            out.append({"adj": s.adjoint_state(g).double().cpu().numpy(),
                        "grad_kappa": keep[g][1].cpu().numpy(),
                        "grad_amp": keep[g][2].cpu().numpy()[:len(p.sources)],
                        "trace": s.traces[g].double().cpu().numpy()})
        torch.cuda.synchronize()
    finally:
        s.close()
    return out


def _compare(gpu, ref, tol, what):
    e1 = rel_l2(gpu["adj"], ref["adj"])
    e2 = rel_l2(gpu["grad_kappa"], ref["grad_kappa"])
    e3 = rel_l2(gpu["grad_amp"], ref["grad_amp"])
    print(f"[adjoint] {what}: state {e1:.2e} grad_kappa {e2:.2e} grad_amp {e3:.2e}", flush=True)
    assert np.linalg.norm(ref["adj"]) > 0 and np.linalg.norm(ref["grad_kappa"]) > 0
    assert e1 <= tol, f"{what}: adjoint state {e1:.3e}"
    assert e2 <= tol, f"{what}: grad_kappa {e2:.3e}"
    assert e3 <= tol, f"{what}: grad_amp {e3:.3e}"


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name,bc,rr", BC_CASES, ids=[c[0] for c in BC_CASES])
def test_adjoint_matches_oracle(name, bc, rr, dtype):
    p = _problem(bc, rr, seed=len(name))
    T, seg = 40, 7
    rng = np.random.default_rng(7)
    res = rng.standard_normal((T, p.nrec, p.ncomp))
    ref = stepper.adjoint(p, nsteps=T, residual=res)
    g = _gpu_adjoint([p], T, seg, dtype, [res])[0]
    _compare(g, ref, TOL[dtype], f"{name} {dtype}")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("bc", [(BC_FREE0, BC_RIGID, BC_PERIODIC, BC_PERIODIC),
                                (BC_PERIODIC,) * 4, (BC_FREE, BC_FREE, BC_RIGID, BC_RIGID)],
                         ids=["free0_rigid_periodic_x", "periodic", "free_rigid_sides"])
def test_adjoint_interior_tiles_match_oracle(bc, dtype):
    """A grid large enough for interior tiles of the adjoint (source band in a
    corner, a receiver row through the middle that sends the tiles beside it
    to the general kernel). The two launch shapes split the cells differently
    between the interior and the general kernel, which form a cell's terms in
    the same order: the state and dL/dkappa agree bit for bit."""
    p = _problem(bc, -1, nx=300, ny=200, seed=11)
    p = p.replace(sources=[Source(40.0, 30.0, 2.0, 0.3, 0.9, 1.0, 12.0, 16.0)],
                  receivers=np.asarray([(x, 0) for x in range(0, 300, 5)] +
                                       [(x, 101) for x in range(3, 300, 11)], np.int32))
    T, seg = 40, 16
    res = np.random.default_rng(4).standard_normal((T, p.nrec, p.ncomp))
    ref = stepper.adjoint(p, nsteps=T, residual=res)
    got = []
    for launch in (dict(waves=1, rows=4), dict(waves=2, rows=8)):
        g = _gpu_adjoint([p], T, seg, dtype, [res], launch=launch)[0]
        _compare(g, ref, TOL[dtype], f"interior tiles {bc} {launch} {dtype}")
        got.append(g)
    for k in ("adj", "grad_kappa"):
        assert np.array_equal(got[0][k], got[1][k]), k


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_adjoint_chunks_and_segments_are_neutral(dtype):
    """Stepping the adjoint back in uneven pieces, and any checkpoint
    spacing, gives bitwise the same state, dL/dkappa and dL/damp (each step's
    dL/damp is summed over workgroups in a fixed order, with no atomics)."""
    p = _problem((BC_FREE0, BC_RIGID, BC_PERIODIC, BC_PERIODIC), -1, nx=90, ny=33, seed=3)
    T = 30
    res = np.random.default_rng(2).standard_normal((T, p.nrec, p.ncomp))
    a = _gpu_adjoint([p], T, 30, dtype, [res])[0]
    for seg, chunks in ((1, [30]), (4, [13, 17]), (11, [1, 28, 1]), (64, [29, 1])):
        b = _gpu_adjoint([p], T, seg, dtype, [res], chunks=chunks)[0]
        for k in ("adj", "grad_kappa", "grad_amp"):
            assert np.array_equal(a[k], b[k]), (seg, chunks, k)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batched_adjoint_matches_oracle(dtype):
    """Grids of different sizes and boundary types in one context."""
    p1 = _problem((BC_FREE, BC_RIGID, BC_PERIODIC, BC_PERIODIC), 20, nx=150, ny=37, seed=1)
    p2 = _problem((BC_RIGID,) * 4, -1, nx=64, ny=65, seed=2)
    T, seg = 36, 10
    rng = np.random.default_rng(9)
    r1 = rng.standard_normal((T, p1.nrec, p1.ncomp))
    r2 = rng.standard_normal((T, p2.nrec, p2.ncomp))
    g1, g2 = _gpu_adjoint([p1, p2], T, seg, dtype, [r1, r2], launch=dict(waves=2, rows=4))
    _compare(g1, stepper.adjoint(p1, nsteps=T, residual=r1), TOL[dtype], f"batched grid 0 {dtype}")
    _compare(g2, stepper.adjoint(p2, nsteps=T, residual=r2), TOL[dtype], f"batched grid 1 {dtype}")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gradients_and_misfit_are_reproducible(dtype):
    """The same run twice, on the two-step path with pairs and single steps
    mixed: the adjoint state, dL/dkappa, dL/damp and the misfit agree bit for
    bit (their sums over workgroups run in a fixed order, with no atomics)."""
    import torch
    from paper_2009_06404_amd import Solver
    p = _problem((BC_FREE, BC_RIGID, BC_PERIODIC, BC_PERIODIC), 20, nx=300, ny=90, seed=8)
    T = 26
    d_obs = np.random.default_rng(4).standard_normal((T, p.nrec, p.ncomp)) * 1e-3
    runs = []
    for _ in range(2):
        s = Solver(p, dtype=dtype, trace_steps=T, launch=dict(waves=2, rows=4, fuse_rows=8))
        try:
            s.adjoint_begin(T, 9)
            s.step(T)
            mis, res = s.misfit(0, torch.as_tensor(d_obs))
            gk = torch.zeros((p.ny, p.nx), dtype=torch.float64, device=s.device)
            ga = torch.zeros(len(p.sources), dtype=torch.float64, device=s.device)
            s.adjoint_set_io(0, res, gk, ga)
            s.adjoint_step(5)
            s.adjoint_step(T - 5)
            runs.append([mis.cpu().numpy(), s.adjoint_state(0).cpu().numpy(), gk.cpu().numpy(),
                         ga.cpu().numpy()])
            torch.cuda.synchronize()
        finally:
            s.close()
    assert np.abs(runs[0][3]).max() > 0
    for a, b, what in zip(runs[0], runs[1], ("misfit", "state", "grad_kappa", "grad_amp")):
        assert np.array_equal(a, b), what


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_misfit_and_lame_gradient(dtype):
    import torch
    from paper_2009_06404_amd import Solver
    p = _problem((BC_FREE0, BC_RIGID, BC_PERIODIC, BC_PERIODIC), -1, seed=4)
    T = 25
    d_obs = np.random.default_rng(3).standard_normal((T, p.nrec, p.ncomp)) * 1e-4
    ref_tr = stepper.run(p, nsteps=T)["trace"]
    ref_L, ref_e = stepper.misfit(ref_tr, d_obs)
    s = Solver(p, dtype=dtype, trace_steps=T)
    try:
        s.step(T)
        mis, res = s.misfit(0, torch.as_tensor(d_obs))
        gk = torch.as_tensor(np.random.default_rng(5).standard_normal((p.ny, p.nx)),
                             device=s.device).contiguous()
        gl = torch.zeros_like(gk)
        gm = torch.zeros_like(gk)
        s.lame_gradient(0, gk, gl, gm)
        s.lame_gradient(0, gk, gl, gm)              # accumulates
        torch.cuda.synchronize()
        tol = TOL[dtype]
        assert abs(mis.item() - ref_L) <= tol * ref_L
        assert rel_l2(res.double().cpu().numpy(), ref_e) <= tol
        lam, mu, _ = p.medium.full(p.ny, p.nx)
        wl, wm = stepper.lame_gradients(gk.cpu().numpy(), lam, mu)
        ftol = 1e-15 if dtype == "f64" else 1e-6
        assert rel_l2(gl.cpu().numpy(), 2 * wl) <= ftol
        assert rel_l2(gm.cpu().numpy(), 2 * wm) <= ftol
    finally:
        s.close()


def test_reduced_adjoint_workload_gradients():
    """The adjoint workload at 256^2 with 4 shots and 1000 steps, checkpoints
    every 100 steps, FP32: misfit gradients with respect to lambda, mu and
    the amplitudes against the FP64 oracle adjoint (observed data: the same
    shots through the homogeneous background, computed by the oracle)."""
    import torch
    from paper_2009_06404_amd import Solver
    n, shots, T = 256, 4, 1000
    probs = [p.replace(nsteps=T) for p in w.adjoint_shots(n=n, shots=shots, nsteps=T)]
    bg = w.adjoint_shots(n=n, shots=shots, nsteps=T, homogeneous=True)
    lam, mu, rho = probs[0].medium.full(n, n)
    ref_gl = np.zeros((n, n))
    ref_gm = np.zeros((n, n))
    ref_ga = []
    d_obs = []
    for p, q in zip(probs, bg):
        d = stepper.run(q, nsteps=T)["trace"]
        d_obs.append(d)
        fw = stepper.run(p, nsteps=T)["trace"]
        _, e = stepper.misfit(fw, d)
        ad = stepper.adjoint(p, nsteps=T, residual=e)
        gl, gm = stepper.lame_gradients(ad["grad_kappa"], lam, mu)
        ref_gl += gl
        ref_gm += gm
        ref_ga.append(ad["grad_amp"][0])
    print(f"[adjoint] oracle done for {shots} shots", flush=True)
    s = Solver(probs, dtype="f32", trace_steps=T)
    try:
        s.adjoint_begin(T, 100)
        s.step(T)
        gk = torch.zeros((shots, n, n), dtype=torch.float64, device=s.device)
        ga = torch.zeros((shots, 1), dtype=torch.float64, device=s.device)
        keep = []
        for g in range(shots):
            mis, res = s.misfit(g, torch.as_tensor(d_obs[g]))
            keep.append(res)
            s.adjoint_set_io(g, res, gk[g], ga[g])
        s.adjoint_step(T)
        gl = torch.zeros((n, n), dtype=torch.float64, device=s.device)
        gm = torch.zeros_like(gl)
        for g in range(shots):
            s.lame_gradient(g, gk[g], gl, gm)
        torch.cuda.synchronize()
        e_l = rel_l2(gl.cpu().numpy(), ref_gl)
        e_m = rel_l2(gm.cpu().numpy(), ref_gm)
        e_a = rel_l2(ga[:, 0].cpu().numpy(), np.array(ref_ga))
        print(f"[adjoint] reduced workload: grad_lam {e_l:.2e} grad_mu {e_m:.2e} "
              f"grad_amp {e_a:.2e}", flush=True)
        assert e_l <= 1e-4 and e_m <= 1e-4 and e_a <= 1e-4
    finally:
        s.close()


def test_autograd_shot_traces():
    """torch.autograd through ShotTraces: the gradient of a trace misfit with
    respect to lambda, mu and the amplitudes equals the oracle's."""
    import torch
    from paper_2009_06404_amd import shot_traces
    n, shots, T = 96, 2, 160
    probs = [p.replace(nsteps=T) for p in w.adjoint_shots(n=n, shots=shots, nsteps=T, sponge=16)]
    lam0, mu0, rho0 = probs[0].medium.full(n, n)
    d_obs = np.random.default_rng(1).standard_normal((shots, T, n, 1)) * 1e-6
    lam = torch.tensor(lam0, dtype=torch.float64, device="cuda", requires_grad=True)
    mu = torch.tensor(mu0, dtype=torch.float64, device="cuda", requires_grad=True)
    amp = torch.tensor([1.0, 0.7], dtype=torch.float64, device="cuda", requires_grad=True)
    tr = shot_traces(lam, mu, amp, probs, T, seg_steps=32, dtype="f64")
    loss = 0.5 * ((tr - torch.as_tensor(d_obs, device="cuda")) ** 2).sum()
    loss.backward()
    ref_gl = np.zeros((n, n))
    ref_gm = np.zeros((n, n))
    ref_ga = []
    for g, (p, a) in enumerate(zip(probs, [1.0, 0.7])):
        q = p.sources[0]
        pa = p.replace(sources=[Source(q.x, q.y, q.sigma, q.dir_x, q.dir_y, a, q.period, q.t0)])
        fw = stepper.run(pa, nsteps=T)["trace"]
        _, e = stepper.misfit(fw, d_obs[g])
        ad = stepper.adjoint(pa, nsteps=T, residual=e)
        gl, gm = stepper.lame_gradients(ad["grad_kappa"], lam0, mu0)
        ref_gl += gl
        ref_gm += gm
        ref_ga.append(ad["grad_amp"][0])
    assert rel_l2(lam.grad.cpu().numpy(), ref_gl) <= 1e-11
    assert rel_l2(mu.grad.cpu().numpy(), ref_gm) <= 1e-11
    assert rel_l2(amp.grad.cpu().numpy(), np.array(ref_ga)) <= 1e-11


def test_full_size_adjoint_one_shot_against_the_oracle():
    """The adjoint workload on its full grid (16 shots of 1024^2, FP32,
    cell-wise moduli, checkpoints every 100 steps) in the launch the benchmark
    times, over 200 steps. Shot 0 takes its residual against the observed
    data of the homogeneous background (computed by the oracle) and is
    compared with the FP64 oracle adjoint: dL/dkappa, dL/damp and the adjoint
    state at t = 0. The other 15 shots take zero observed data and must give
    finite gradients."""
    import torch
    import bench
    from paper_2009_06404_amd import Solver
    n, shots, T = 1024, 16, 200
    probs = [p.replace(nsteps=T) for p in w.adjoint_shots(n=n, shots=shots, nsteps=T)]
    bg0 = w.adjoint_shots(n=n, shots=shots, nsteps=T, homogeneous=True)[0]
    d0 = stepper.run(bg0, nsteps=T)["trace"]
    _, e0 = stepper.misfit(stepper.run(probs[0], nsteps=T)["trace"], d0)
    ref = stepper.adjoint(probs[0], nsteps=T, residual=e0)
    print("[adjoint] oracle done for shot 0 at 1024^2", flush=True)
    s = Solver(probs, dtype="f32", trace_steps=T, launch=dict(bench.ADJOINT_LAUNCH))
    try:
        assert s.launch()["fuse_rows"] > 0
        s.adjoint_begin(T, 100)
        s.step(T)
        gk = torch.zeros((shots, n, n), dtype=torch.float64, device=s.device)
        ga = torch.zeros((shots, 1), dtype=torch.float64, device=s.device)
        keep = []
        for g in range(shots):
            d = torch.as_tensor(d0) if g == 0 else torch.zeros_like(s.traces[g])
            _, res = s.misfit(g, d)
            keep.append(res)
            s.adjoint_set_io(g, res, gk[g], ga[g])
        s.adjoint_step(T)
        got = {"adj": s.adjoint_state(0).double().cpu().numpy(), "grad_kappa": gk[0].cpu().numpy(),
               "grad_amp": ga[0].cpu().numpy()}
        assert bool(torch.isfinite(gk).all()) and bool(torch.isfinite(ga).all())
    finally:
        s.close()
    _compare(got, ref, TOL["f32"], "full-size shot 0 (1024^2, 200 steps, 16 shots batched)")
