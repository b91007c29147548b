"""Shared helpers for the GPU parity tests: run a problem through the C ABI
and compare with the oracle."""
import numpy as np


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return float(np.linalg.norm(a))
    return float(np.linalg.norm(a - b) / nb)


FIELDS = ("rho", "j_x", "j_y", "P_xx", "P_xy", "P_yy")


def run_gpu(problems, nsteps, dtype=None, launch=None, state=None, t0=0):
    """Run one problem (or a batch) for nsteps through liblbm; returns a list of
    dicts with numpy float64 'mom', 'fstar', 'trace'."""
    import torch
    from paper_2009_06404_amd import Solver
    single = not isinstance(problems, (list, tuple))
    probs = [problems] if single else list(problems)
    s = Solver(probs, dtype=dtype, trace_steps=max(nsteps, 1), launch=launch)
    try:
        if state is not None:
            for g, st in enumerate(state if not single else [state]):
                s.set_state(g, torch.as_tensor(st), t0)
        s.step(nsteps)
        out = []
        for g, p in enumerate(probs):
            d = {"mom": s.moments(g).double().cpu().numpy(),
                 "fstar": s.state(g).double().cpu().numpy()}
            tr = s.traces[g]
            d["trace"] = tr.double().cpu().numpy() if tr is not None else None
            out.append(d)
        torch.cuda.synchronize()
    finally:
        s.close()
    return out[0] if single else out


def compare(gpu, ref, tol, what="", near_zero=()):
    """Per-field relative L2 of the macroscopic fields, the state and the
    traces; asserts each is within tol. Returns the worst value. Each field is
    measured against its own norm, except the fields named in near_zero
    (which the test's problem makes vanish, or nearly vanish, by symmetry;
    each test says why): those are measured against 1e-3 of the largest
    field's norm."""
    worst = 0.0
    floor = 1e-3 * max(np.linalg.norm(ref["mom"][k]) for k in range(6))
    for name in near_zero:
        assert name in FIELDS, name
    for k, name in enumerate(FIELDS):
        nb = np.linalg.norm(ref["mom"][k])
        if name in near_zero:
            nb = max(nb, floor)
        e = float(np.linalg.norm(gpu["mom"][k] - ref["mom"][k]) / nb) if nb > 0 \
            else rel_l2(gpu["mom"][k], ref["mom"][k])
        assert e <= tol, f"{what} field {name}: rel L2 {e:.3e} > {tol:.1e}"
        worst = max(worst, e)
    e = rel_l2(gpu["fstar"], ref["fstar"])
    assert e <= tol, f"{what} state f*: rel L2 {e:.3e} > {tol:.1e}"
    worst = max(worst, e)
    if gpu.get("trace") is not None and ref.get("trace") is not None and ref["trace"].size:
        e = rel_l2(gpu["trace"], ref["trace"])
        assert e <= tol, f"{what} traces: rel L2 {e:.3e} > {tol:.1e}"
        worst = max(worst, e)
    return worst
