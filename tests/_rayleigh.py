"""The surface-wave experiment of Sec. 7 (shared by the oracle test and the
GPU test): a 300 x 100 grid with a free surface on top and 30-cell absorbing
layers on the three other sides for the first 400 steps, then periodic sides
(bottom layer kept), so that the surface wave circles the grid. A vertical
Gaussian x Ricker force near the upper-left corner (the paper does not print
its parameters: x = 45, 3 cells deep, sigma 2, period 40, delay 60 here).

Analysis of the outputs (not of the method): the surface-wave speed from the
time two complete turns take at each surface station (the paper's
measurement), and least-squares fits of the depth profile of j_y at step
1800 under the surface maximum: an exponential A exp(-y/d), and the
vertical-displacement profile of a Rayleigh wave,
    A [exp(-k a_P y) - 2/(1 + a_S^2) exp(-k a_S y)],
a_P = sqrt(1 - v_R^2/v_P^2), a_S = sqrt(1 - v_R^2/v_S^2), k = 2 pi / lambda_R,
which follows from the two traction-free conditions of the half-space
solution. The paper prints this profile with a_P and a_S exchanged; that
form is fitted as well, for comparison."""
import numpy as np

import workloads as w
from workloads import BC_FREE0, BC_PERIODIC, BC_RIGID, Medium, Problem, Source
from oracle import theory as T
from _golden import paper_values

NU = 0.25
PV = paper_values()
NX, NY = int(PV["rayleigh_grid_nx"]), int(PV["rayleigh_grid_ny"])
L = int(PV["rayleigh_sponge"])
SWITCH = int(PV["rayleigh_switch_step"])
PROFILE_STEP = int(PV["rayleigh_profile_step"])
END = 2400


def problems(tau=1.0, free=BC_FREE0):
    """(phase 1 with side layers, phase 2 with periodic sides). The paper
    does not print the experiment's tau or which extrapolation its free
    surface used; the defaults are tau = 1 and the zero-order surface, and
    (0.55, BC_FREE) is the printed rule at the tau of the bulk-wave tests."""
    prof = w.default_sponge_profile(L)
    med = Medium("homogeneous", 0.04 * T.lame_ratio(NU), 0.04, 1.0)
    rec = np.array([[x, 0] for x in range(NX)], np.int32)
    p1 = Problem(nx=NX, ny=NY, bc=(free, BC_RIGID, BC_PERIODIC, BC_PERIODIC), medium=med,
                 tau=tau, sponge_thick=(0, L, L, L), sponge_profiles=(None, prof, prof, prof),
                 sources=[Source(45.0, 3.0, 2.0, 0.0, 1.0, 1.0, 40.0, 60.0)],
                 receivers=rec, comp_mask=2, name="rayleigh")
    p2 = p1.replace(sponge_thick=(0, L, 0, 0), sponge_profiles=(None, prof, None, None))
    return p1, p2


def speeds():
    vr = T.rayleigh_speed(NU)
    vp, vs = T.wave_speeds(NU)
    return vr, vp, vs


def two_turn_speed(trace):
    """trace: (END, NX) surface v_y for steps 0..END-1. At every tenth station,
    the lag that best aligns a 101-step window around a passage of the
    surface pulse after the switch with the signal two turns later (sub-step
    by a parabola through the correlation peak); v = 2 NX / lag. Returns the
    mean and the spread over stations."""
    vr, _, _ = speeds()
    half = 50
    out = []
    for x in range(0, NX, 10):
        tp = 60.0 + ((x - 45) % NX) / vr
        while tp < SWITCH + 80:
            tp += NX / vr
        t1 = int(round(tp))
        lag0 = 2 * NX / vr
        if t1 + int(lag0) + half + 45 >= trace.shape[0]:
            continue
        seg = trace[t1 - half:t1 + half + 1, x]
        lags = np.arange(int(lag0) - 40, int(lag0) + 41)
        c = np.array([np.dot(seg, trace[t1 - half + g:t1 + half + 1 + g, x]) for g in lags])
        k = int(np.argmax(c))
        y0, y1, y2 = c[k - 1], c[k], c[k + 1]
        out.append(2 * NX / (lags[k] + 0.5 * (y0 - y2) / (y0 - 2 * y1 + y2)))
    out = np.array(out)
    return float(out.mean()), float(out.std()), len(out)


def depth_fits(jy, depth=60):
    """Least-squares fits of j_y(y) under the surface maximum of jy (ny, nx)."""
    from scipy.optimize import curve_fit
    vr, vp, vs = speeds()
    aS, aP = np.sqrt(1 - (vr / vs) ** 2), np.sqrt(1 - (vr / vp) ** 2)
    xm = int(np.argmax(np.abs(jy[0])))
    y = np.arange(depth, dtype=np.float64)
    prof = jy[:depth, xm]

    def expo(y, A, d):
        return A * np.exp(-y / d)

    def rayleigh(y, A, lam):
        k = 2 * np.pi / lam
        return A * (np.exp(-k * aP * y) - 2 / (1 + aS ** 2) * np.exp(-k * aS * y))

    def printed(y, A, lam):
        k = 2 * np.pi / lam
        return A * (np.exp(-k * aS * y) - 2 / (1 + aP ** 2) * np.exp(-k * aP * y))

    out = {"x": xm}
    for name, f, p0 in (("exp", expo, (prof[0], 20.0)), ("rayleigh", rayleigh, (-prof[0], 40.0)),
                        ("printed", printed, (prof[0], 40.0))):
        popt, _ = curve_fit(f, y, prof, p0=p0, maxfev=20000)
        out[name] = (popt, float(np.sum((f(y, *popt) - prof) ** 2)))
    return out
