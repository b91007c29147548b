"""The allocation-free finite check (lbm_check_finite_noalloc) against
lbm_check_finite through the C ABI: the same verdict on finite states, on
NaN and on Inf in one or two grids of a batch, on two calls in a row with
the second on a smaller context (its scratch must have been cleared after a
non-finite result), and a clear refusal beyond its 4096-grid scratch."""
import numpy as np
import pytest

import workloads as w
from workloads import BC_FREE0, BC_PERIODIC, BC_RIGID, Medium, Problem

pytestmark = pytest.mark.gpu


def _both(s):
    from paper_2009_06404_amd import _lib as L
    rc_a = L.lib().lbm_check_finite(s.ctx)
    rc_b = L.lib().lbm_check_finite_noalloc(s.ctx)
    return rc_a, rc_b, L.last_error()


def _poison(s, g, value, where):
    import torch
    st = s.state(g).clone()
    st[where] = value
    s.set_state(g, st, s.time)
    torch.cuda.synchronize()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_noalloc_finite_check_matches_the_allocating_one(dtype):
    from paper_2009_06404_amd import Solver, _lib as L
    ok, bad = L.LBM_OK, L.LBM_E_NONFINITE
    probs = w.batched_shots(count=3, nsteps=20, sponge=16, sides=[70, 131, 96])
    s = Solver(probs, dtype=dtype, trace_steps=1)
    try:
        s.step(20)
        assert _both(s)[:2] == (ok, ok)
        _poison(s, 1, float("nan"), (4, 100, 33))
        rc_a, rc_b, msg = _both(s)
        assert (rc_a, rc_b) == (bad, bad) and "1 grid(s), the first is grid 1" in msg, msg
        _poison(s, 2, float("inf"), (8, 95, 0))
        rc_a, rc_b, msg = _both(s)
        assert (rc_a, rc_b) == (bad, bad) and "2 grid(s), the first is grid 1" in msg, msg
        _poison(s, 1, 0.0, (4, 100, 33))
        rc_a, rc_b, msg = _both(s)
        assert (rc_a, rc_b) == (bad, bad) and "1 grid(s), the first is grid 2" in msg, msg
    finally:
        s.close()
    # second call, smaller input: one grid, finite, then -inf in its last cell
    p = Problem(nx=40, ny=24, bc=(BC_FREE0, BC_RIGID, BC_PERIODIC, BC_PERIODIC),
                medium=Medium("homogeneous", 0.03, 0.04, 1.0))
    s = Solver(p, dtype=dtype, trace_steps=1)
    try:
        s.step(3)
        assert _both(s)[:2] == (ok, ok)
        _poison(s, 0, float("-inf"), (8, 23, 39))
        rc_a, rc_b, msg = _both(s)
        assert (rc_a, rc_b) == (bad, bad) and "1 grid(s), the first is grid 0" in msg, msg
    finally:
        s.close()


def test_noalloc_finite_check_refuses_more_grids_than_its_scratch():
    from paper_2009_06404_amd import Solver, _lib as L
    p = Problem(nx=3, ny=3, bc=(BC_PERIODIC,) * 4, medium=Medium("homogeneous", 0.04, 0.04, 1.0))
    s = Solver([p] * 4097, dtype="f32", trace_steps=1)
    try:
        assert L.lib().lbm_check_finite(s.ctx) == L.LBM_OK
        assert L.lib().lbm_check_finite_noalloc(s.ctx) == L.LBM_E_INVALID
        assert "at most 4096 grids" in L.last_error()
    finally:
        s.close()
    s = Solver([p] * 4096, dtype="f32", trace_steps=1)
    try:
        assert L.lib().lbm_check_finite_noalloc(s.ctx) == L.LBM_OK
    finally:
        s.close()
