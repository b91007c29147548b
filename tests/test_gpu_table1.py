"""The paper's bulk-wave validation (Sec. 5, the Table of j_x misfits) run on
the GPU: periodic boxes of 64^2 .. 512^2, Poisson ratios 0 .. 0.3, tau = 0.55,
a centred x-directed Gaussian x Ricker force, compared with the App. B Fourier
spectral Crank-Nicolson solution of the Navier equation.

At 128^2 the configuration is the paper's (sigma 4, period 20, 70 steps); the
other sizes scale the source, the period, the delay and the step count with
the grid (the paper does not state its scaling). Checked: the GPU fields equal
the FP64 oracle's at every size (1e-12); against the reference at the same
time, the 128^2 misfits lie within 1.5x of the printed row and the misfit falls
by at least 1.8x per refinement (faster than the printed first order); against
the reference half a step later, every size lies within 1.5x of the printed
row and the misfit falls at first order, as printed: the printed table is
consistent with a half-step offset between the two solutions compared."""
import numpy as np
import pytest

import workloads as w
from workloads import Source
from oracle import spectral, stepper
from _golden import TABLE1_NUS, table1
from gpu_helpers import rel_l2, run_gpu

pytestmark = pytest.mark.gpu


def _case(n, nu):
    s = n / 128
    p = w.plain_small(n=n, nsteps=int(round(70 * s)), nu=nu, tau=0.55)
    return p.replace(sources=[Source(n / 2, n / 2, 4.0 * s, 1.0, 0.0, 1.0, 20.0 * s, 30.0 * s)],
                     receivers=np.zeros((0, 2), np.int32))


def test_table1_sweep_on_gpu():
    tab = table1()
    errs, half = {}, {}
    for n in (64, 128, 256, 512):
        row, row_h = [], []
        for nu in TABLE1_NUS:
            p = _case(n, nu)
            g = run_gpu(p, p.nsteps, "f64")
            jx = g["mom"][1]
            ref = stepper.run(p, want_trace=False)["mom"][1]
            assert rel_l2(jx, ref) <= 1e-12, (n, nu)
            j0, _ = spectral.solve(n, nu, p.nsteps, p.sources[0])
            j1, _ = spectral.solve(n, nu, p.nsteps + 1, p.sources[0])
            row.append(spectral.rel_l2(jx, j0))
            row_h.append(spectral.rel_l2(jx, 0.5 * (j0 + j1)))
        errs[n], half[n] = row, row_h
        print(f"[table1] {n:4d}: same time " + " ".join(f"{e:.4f}" for e in row)
              + " | half a step later " + " ".join(f"{e:.4f}" for e in row_h)
              + " | printed " + " ".join(f"{v:.4f}" for v in tab[n]), flush=True)
    for e, printed in zip(errs[128], tab[128]):
        assert printed / 1.5 < e < printed * 1.5
    for a, b in ((64, 128), (128, 256), (256, 512)):
        for ea, eb in zip(errs[a], errs[b]):
            assert ea > 1.8 * eb, (a, b, ea, eb)
    for n in (64, 128, 256, 512):
        for e, printed in zip(half[n], tab[n]):
            assert printed / 1.5 < e < printed * 1.5, (n, e, printed)
    for a, b in ((128, 256), (256, 512)):
        for ea, eb in zip(half[a], half[b]):
            assert 1.4 < ea / eb < 2.2, (a, b, ea, eb)
