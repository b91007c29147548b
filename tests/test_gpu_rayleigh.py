"""Sec. 7's surface-wave experiment on the GPU (300 x 100 grid, free
surface, 30-cell absorbing layers on the other sides for 400 steps, then
periodic sides): the state handed from the first context to the second
through lbm_get_state / lbm_set_state at step 400, surface traces to step
2400 and the fields at step 1800 equal the FP64 oracle's (FP64 1e-12, FP32
1e-5, relative L2), and the GPU run's own surface-wave speed (two turns)
and depth profile meet the same bars as the oracle's."""
import numpy as np
import pytest

from oracle import stepper
from gpu_helpers import rel_l2
import _rayleigh as RY

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def _oracle():
    p1, p2 = RY.problems()
    a = stepper.run(p1, nsteps=RY.SWITCH)
    b = stepper.run(p2, nsteps=RY.PROFILE_STEP - RY.SWITCH, t0=RY.SWITCH, fstar_init=a["fstar"])
    c = stepper.run(p2, nsteps=RY.END - RY.PROFILE_STEP, t0=RY.PROFILE_STEP, fstar_init=b["fstar"])
    trace = np.concatenate([a["trace"][:, :, 0], b["trace"][:, :, 0], c["trace"][:, :, 0]])
    return trace, b["mom"]


def _gpu(dtype):
    import torch
    from paper_2009_06404_amd import Solver
    p1, p2 = RY.problems()
    s1 = Solver(p1, dtype=dtype, trace_steps=RY.SWITCH)
    try:
        s1.step(RY.SWITCH)
        st = s1.state(0).clone()
        tr1 = s1.traces[0][:, :, 0].double().cpu().numpy()
    finally:
        s1.close()
    s2 = Solver(p2, dtype=dtype, trace_steps=RY.END - RY.SWITCH)
    try:
        s2.set_state(0, st, RY.SWITCH)
        s2.step(RY.PROFILE_STEP - RY.SWITCH)
        mom = s2.moments(0).double().cpu().numpy()
        s2.step(RY.END - RY.PROFILE_STEP)
        tr2 = s2.traces[0][:, :, 0].double().cpu().numpy()
        torch.cuda.synchronize()
    finally:
        s2.close()
    return np.concatenate([tr1, tr2]), mom


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_rayleigh_experiment_on_gpu(dtype):
    ref_trace, ref_mom = _oracle()
    trace, mom = _gpu(dtype)
    e_tr = rel_l2(trace, ref_trace)
    e_j = rel_l2(mom[2], ref_mom[2])
    assert e_tr <= TOL[dtype] and e_j <= TOL[dtype], (e_tr, e_j)
    vr, _, _ = RY.speeds()
    v, spread, n = RY.two_turn_speed(trace)
    fits = RY.depth_fits(mom[2])
    print(f"[rayleigh] {dtype}: traces {e_tr:.2e}, j_y(1800) {e_j:.2e}; v_R two turns {v:.5f} "
          f"(theory {vr:.5f}, {100 * (v - vr) / vr:+.2f}%, spread {spread:.4f} over {n} stations); "
          f"depth fit at x={fits['x']}: lambda_R {fits['rayleigh'][0][1]:.1f}, residuals "
          f"Rayleigh {fits['rayleigh'][1]:.2e} exponential {fits['exp'][1]:.2e} "
          f"(d = {fits['exp'][0][1]:.1f}) printed form {fits['printed'][1]:.2e}", flush=True)
    assert n >= 20 and abs(v - vr) / vr < 0.005
    assert fits["rayleigh"][1] < 0.5 * fits["exp"][1]
    assert fits["rayleigh"][1] < 0.1 * fits["printed"][1]
