"""lbm_autotune on the GPU, through the C ABI of include/lbm.h.

On the two-step path it picks a block shape (waves 2 / 4 / 8, fuse_rows 16 ..
64), on the single-step path a tile shape. The state and the time are left
as they were and no launch shape changes a bit of the result, so steps after
tuning equal steps without it, state and traces, bit for bit. A second call
with steps = 0 returns the cached choice for the context's key.
"""
import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu


def _run(p, dtype, tune):
    import torch
    from paper_2009_06404_amd import Solver
    s = Solver(p, dtype=dtype, trace_steps=40)
    try:
        st = np.random.default_rng(4).normal(size=(9, p.ny, p.nx)) * 1e-3
        s.set_state(0, torch.as_tensor(st, dtype=s.tdtype, device="cuda"), 0)
        s.step(3)
        chosen = None
        if tune is not None:
            chosen = s.autotune(tune)
            assert s.time == 3
            assert s.autotune(0) == chosen == s.launch()
        s.step(11)
        assert s.time == 14
        # trace rows of later times may hold the tuning runs' (equal) values
        out = (s.state().cpu().numpy(), s.traces[0][:14].cpu().numpy())
    finally:
        s.close()
    return chosen, out


@pytest.mark.parametrize("n,dtype,pairs", [(2048, "f32", True), (512, "f64", False)])
def test_autotune_keeps_the_state_and_the_bits(n, dtype, pairs):
    p = w.plain_large(n=n, nsteps=20, dtype=dtype)
    chosen, tuned = _run(p, dtype, 4)
    _, plain = _run(p, dtype, None)
    print(f"[autotune] {n}^2 {dtype}: {chosen}", flush=True)
    if pairs:
        assert chosen["fuse_rows"] >= 16 and chosen["waves"] in (2, 4, 8)
    else:
        assert chosen["fuse_rows"] == 0
    assert np.array_equal(tuned[0], plain[0])
    assert np.array_equal(tuned[1], plain[1])
    assert np.abs(plain[1]).max() > 0   # the random start reaches the receivers at once
