"""The periodic finite check of lbm_step (lbm_set_finite_check) on the GPU:
a run that blows up (Poisson ratio 0.4, unstable at every tau, Sec. 4) is
reported at the first checked time whose state holds NaN or Inf -- the same
time a synchronous lbm_check_finite after every block of steps finds --
while lbm_step itself stays asynchronous; the next lbm_step refuses to step;
lbm_set_state clears the record. A stable run with the check on is bitwise
the run without it, on the single-step and the two-step paths (with
captured graphs between checks)."""
import numpy as np
import pytest

import workloads as w
from workloads import Medium
from oracle import theory as T
from gpu_helpers import run_gpu

pytestmark = pytest.mark.gpu


def _unstable():
    p = w.plain_small(n=64, nsteps=600, nu=0.25, tau=1.0)
    return p.replace(medium=Medium("homogeneous", 0.04 * T.lame_ratio(0.4), 0.04, 1.0))


def test_blow_up_reported_at_the_first_failing_check():
    import warnings
    import torch
    from paper_2009_06404_amd import Solver, _lib as L
    p = _unstable()
    every = 10
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        ref = Solver(p, dtype="f32", trace_steps=1)
        s = Solver(p, dtype="f32", trace_steps=1)
    try:
        first = -1
        for k in range(1, 61):
            ref.step(every)
            if first < 0 and not ref.check_finite():
                first = k * every
        assert 0 < first <= 600, first
        L.lbm_set_finite_check(s.ctx, every)
        s.step(600)                           # asynchronous: no verdict yet
        ok, t_bad = L.lbm_finite_status(s.ctx)
        assert not ok and t_bad == first, (t_bad, first)
        with pytest.raises(L.LBMError, match=f"t = {first}"):
            s.step(1)
        assert s.time == 600
        s.set_state(0, torch.zeros((9, p.ny, p.nx), dtype=torch.float32), 0)
        assert L.lbm_finite_status(s.ctx) == (True, -1)
        s.step(every)
        print(f"[finite check] nu 0.4 blew up by t = {first}; reported at t = {t_bad}", flush=True)
    finally:
        ref.close()
        s.close()


@pytest.mark.parametrize("launch", [None, dict(waves=2, rows=8, fuse_rows=16, graph_chunk=6)],
                         ids=["single_step", "two_step_graphs"])
def test_check_leaves_a_stable_run_unchanged(launch):
    from paper_2009_06404_amd import Solver, _lib as L
    p = w.plain_large(n=600, nsteps=90, sponge=24, src_depth=30)
    a = run_gpu(p, 90, "f32", launch=launch)
    s = Solver(p, dtype="f32", trace_steps=90, launch=launch)
    try:
        L.lbm_set_finite_check(s.ctx, 12)
        s.step(50)
        s.step(40)
        assert L.lbm_finite_status(s.ctx) == (True, -1)
        st = s.state(0).double().cpu().numpy()
        tr = s.traces[0].double().cpu().numpy()
    finally:
        s.close()
    assert np.array_equal(st, a["fstar"]) and np.array_equal(tr, a["trace"])
