#!/usr/bin/env python3
"""Benchmark of the fused D2Q9 elastic-wave LBM step on one MI355X.

Workload (default): the large plain configuration -- 4096 x 4096 FP32 grid,
free surface on top, 96-cell absorbing layers on the other three sides (rigid
bottom behind its layer, periodic sides behind theirs), homogeneous solid with
Poisson ratio 0.33, one vertical Gaussian x Ricker source 20 cells below the
surface, 4096 surface receivers recording v_y. A step is one time step of the
whole grid (pull streaming with the wall rules, moments, density gradient,
source and sponge, collision, receivers).

Steps run in pairs on the two-step path (the default for this size): the
general kernel advances the cells near walls, sources and receivers by one
step into an intermediate buffer while the two-step kernel takes the rest of
the grid (blocks of 256 columns) through both steps in one pass; then the
general kernel takes its cells through the second step. Prints ONE JSON line:
GLUPS (cell updates per second / 1e9) over the timed steps, the roofline of the
dominant kernel -- HBM-bound; algorithmic bytes per launch = one read and one
write of each population word of each cell the launch covers (for the two-step
kernel, once per two steps), divided by its mean launch duration from HIP
events around each of its launches on the solver's stream in a short pass
after the timed steps -- and the FP64 oracle timed on this host's cores on a
bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GLUPS (D2Q9 cell updates/s) and % HBM roofline; batched & adjoint vs plain"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ("paper_2009_06404_amd/csrc/lbm_kernels.hip",
                  "paper_2009_06404_amd/csrc/lbm_adjoint.hip",
                  "paper_2009_06404_amd/csrc/lbm_device.h",
                  "paper_2009_06404_amd/csrc/lbm_internal.h")
FUSED_KERNEL = "fused2_kernel"
FUSED3_KERNEL = "fused3_kernel"
INTERIOR_KERNEL = "interior_kernel"


def traffic_file(kernel: str, workload: str, dtype: str) -> str:
    """profiles/traffic_<kernel>_<workload>_<dtype>.txt, e.g. workload
    plain_large_4096 or hbm_scale_16384."""
    return os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}_{dtype}.txt")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(path: str, cells=None):
    """Bytes per launch from a committed rocprofv3 counter summary, or None
    when the kernel source has changed since the counters were taken or the
    launch covers another number of cells."""
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if "=" in line:
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_hash") != kernel_hash():
        return None
    if cells is not None and vals.get("cells_per_launch") != str(cells):
        return None                      # counters taken for another launch shape
    try:
        return float(vals["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _sample_steps(run, target_s: float, cap: int) -> int:
    """Steps for a sample of about target_s seconds: after one untimed run
    (first-touch and library loading), a run of 1 step and one of 3 separate
    the per-step time from the fixed setup time."""
    run(1)
    t = time.perf_counter()
    run(1)
    t1 = time.perf_counter() - t
    t = time.perf_counter()
    run(3)
    t3 = time.perf_counter() - t
    per = max((t3 - t1) / 2, 1e-3)
    setup = max(t1 - per, 0.0)
    return max(1, min(cap, int((target_s - setup) / per)))


def cpu_baseline(problem, target_s: float = 15.0):
    """The FP64 oracle as it stands, on this host's cores, on the first steps
    of the same workload; steps chosen so the sample takes ~target_s."""
    from oracle import stepper
    cells = problem.nx * problem.ny
    n = _sample_steps(lambda k: stepper.run(problem, nsteps=k, want_trace=False), target_s, 400)
    t = time.perf_counter()
    stepper.run(problem, nsteps=n, want_trace=False)
    el = time.perf_counter() - t
    cores = stepper.num_threads()
    # the same oracle on one thread, over 2 steps (setup included)
    stepper.set_num_threads(1)
    try:
        t = time.perf_counter()
        stepper.run(problem, nsteps=2, want_trace=False)
        el1 = time.perf_counter() - t
    finally:
        stepper.set_num_threads(cores)
    return {"value": cells * n / el / 1e9, "unit": "GLUPS", "cores": cores,
            "kind": "oracle",
            "sample": f"{n} steps of the full {problem.nx}x{problem.ny} grid from the rest "
                      f"state, FP64, OpenMP over rows ({el:.1f} s incl. setup)",
            "one_thread": {"value": cells * 2 / el1 / 1e9, "unit": "GLUPS",
                           "sample": f"2 steps of the same grid on 1 thread ({el1:.1f} s incl. setup)"}}


# hipDeviceAttribute_t values of the HIP runtime's enum (ROCm 7 headers)
_HIP_ATTR = {"clock_khz": 5, "mem_bus_bits": 59, "mem_clock_khz": 60, "compute_units": 63}


def device_report(torch) -> dict:
    """What the device reports (hipDeviceGetAttribute) and a measured plain
    copy of one population buffer's size (9 x 4096^2 FP32): the published
    peaks the roofline uses are checked against both."""
    import ctypes as C
    out = {"name": torch.cuda.get_device_name(0)}
    try:
        hip = C.CDLL("libamdhip64.so")
        for k, a in _HIP_ATTR.items():
            v = C.c_int(0)
            if hip.hipDeviceGetAttribute(C.byref(v), a, 0) == 0:
                out[k] = v.value
        if "mem_clock_khz" in out and "mem_bus_bits" in out:
            # HBM3E moves four bits per pin and reported memory clock (2 GHz
            # reported, 8 Gb/s per pin)
            out["hbm_peak_from_attributes_GBps"] = round(
                4 * out["mem_clock_khz"] * 1e3 * out["mem_bus_bits"] / 8 / 1e9, 1)
            out["hbm_peak_note"] = "4 transfers per reported memory clock x bus width"
    except OSError:
        pass
    src = torch.ones(9 * 4096 * 4096, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    out["copy_GBps"] = round(2 * src.numel() * 4 / (ms / 1e3) / 1e9, 1)
    out["copy_note"] = "torch copy of 604 MB, read + write bytes per second"
    del src, dst
    torch.cuda.empty_cache()
    return out


def cpu_baseline3(problem, target_s: float = 10.0):
    """The FP64 three-dimensional oracle as it stands, on this host's cores,
    on the first steps of the same volume from the rest state; steps chosen
    so the sample takes ~target_s."""
    from oracle import stepper, stepper3d
    steps = _sample_steps(lambda k: stepper3d.run(problem, nsteps=k, want_trace=False), target_s, 40)
    t = time.perf_counter()
    stepper3d.run(problem, nsteps=steps, want_trace=False)
    el = time.perf_counter() - t
    return {"value": problem.cells * steps / el / 1e9, "unit": "GLUPS", "cores": stepper.num_threads(),
            "kind": "oracle",
            "sample": f"{steps} steps of the full {problem.nx}x{problem.ny}x{problem.nz} volume "
                      f"(D3Q{problem.q}) from the rest state, FP64, OpenMP ({el:.1f} s incl. setup)"}


def _timed_steps(s, steps: int, warmup: int, torch) -> float:
    """ms per step over `steps` steps after `warmup`, HIP events on the stream."""
    s.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    s.step(steps)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def roofline_block(kt: dict, esize: int, workload: str, dtype: str) -> dict:
    """The HBM roofline of the dominant kernel (the one covering most cells)
    from its per-launch event timing kt (lbm_step_timed). Algorithmic bytes
    per launch: each population word of each cell the launch covers read once
    from its input state and written once to its output state, 18 words per
    cell (72 B in FP32). The two- and three-step kernels do this once for two
    or three steps, so their `frac` is per pass; `per_update` counts the same
    launch at 18 words per cell update (the survey's per-update figure), which
    on those paths exceeds the HBM peak because the intermediate updates
    never touch HBM."""
    if kt["fused_cells"] > 0:
        ksteps = kt.get("fused_steps") or 2
        kname = FUSED3_KERNEL if ksteps == 3 else FUSED_KERNEL
        kcells, kms = kt["fused_cells"], kt["fused_ms"]
    elif kt["interior_cells"] > 0:
        kname, kcells, kms, ksteps = INTERIOR_KERNEL, kt["interior_cells"], kt["interior_ms"], 1
    else:
        kname, kcells, kms, ksteps = "step_kernel", kt["general_cells"], kt["general_ms"], 1
    per_cell = 18 * esize
    alg_bytes = per_cell * kcells
    achieved = alg_bytes / (kms / 1e3) / 1e9 if kms > 0 else float("nan")
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4),
           "traffic": measured_traffic(traffic_file(kname, workload, dtype), kcells),
           "kernel": kname, "bytes_per_launch": alg_bytes, "cells_per_launch": kcells,
           "steps_per_launch": ksteps, "ms_per_launch": round(kms, 5), "timed_steps": kt["steps"],
           "general_kernel": {"cells_per_launch": kt["general_cells"],
                              "ms_per_launch": round(kt["general_ms"], 5)}}
    if ksteps > 1:
        word = {2: "two", 3: "three"}[ksteps]
        out["counting"] = (f"frac per {word}-step pass: 18 population words per cell per launch, "
                           f"the launch advancing its cells by {word} steps")
        out["per_update"] = {"achieved": round(ksteps * achieved, 1),
                             "frac": round(ksteps * achieved / HBM_PEAK_GBS, 4),
                             "counting": f"18 population words per cell update, {word} updates per "
                                         "cell and launch"}
    else:
        out["counting"] = "18 population words per cell update, one update per cell and launch"
    return out


def _dominant_gbps(kt: dict, esize: int) -> dict:
    """Algorithmic GB/s of the kernel covering most cells (72 B per cell and
    launch in FP32; the two-step kernel moves them once per two steps)."""
    if kt["fused_cells"] > 0:
        name = FUSED3_KERNEL if kt.get("fused_steps") == 3 else FUSED_KERNEL
        cells, ms = kt["fused_cells"], kt["fused_ms"]
    else:
        name, cells, ms = INTERIOR_KERNEL, kt["interior_cells"], kt["interior_ms"]
    return {"kernel": name, "GBps": round(18 * esize * cells / ms / 1e6, 1) if ms > 0 else None}


def bench_plain_variant(torch, w, Solver, dtype: str, launch_over: dict, label: str,
                        steps: int = 600, warmup: int = 20) -> dict:
    """The plain 4096^2 workload in another dtype or launch (the single-step
    path, FP64): GLUPS over `steps` steps and the roofline of its dominant
    kernel."""
    p = w.plain_large(dtype=dtype)
    s = Solver(p, dtype=dtype, trace_steps=warmup + steps + 64)
    launch = s.launch()
    launch.update(launch_over)
    launch["graph_chunk"] = 0 if launch.get("fuse_rows", 0) else 100
    s.set_launch(**launch)
    ms = _timed_steps(s, steps, warmup, torch)
    kt = s.step_timed(40)
    ok = s.check_finite()
    launch = s.launch()
    s.close()
    cells = p.nx * p.ny
    esize = 4 if dtype == "f32" else 8
    return {"workload": f"plain_large {p.nx}x{p.ny} {dtype.upper()} ({label})",
            "GLUPS": round(cells / ms / 1e6, 3), "ms_per_step": round(ms, 5), "steps": steps,
            "warmup": warmup,
            "roofline": roofline_block(kt, esize, f"plain_large_{p.nx}", dtype),
            "launch": launch, "state_finite": bool(ok)}


def bench_filter(torch, w, Solver, steps_ms: float, passes: int = 20) -> dict:
    """The high-wavenumber filter (lbm_filter) on the 4096^2 FP32 state: one
    pass reads and writes every population word (72 B per cell)."""
    import warnings
    p = w.plain_large(nsteps=2)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        s = Solver(p, dtype="f32", trace_steps=4)
    s.step(2)
    for _ in range(3):
        s.filter(0.01)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(passes):
        s.filter(0.01)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / passes
    s.close()
    return {"workload": "lbm_filter on the plain_large 4096x4096 FP32 state", "ms_per_pass": round(ms, 4),
            "GBps": round(72 * p.nx * p.ny / (ms / 1e3) / 1e9, 1), "passes": passes,
            "vs_one_step": round(ms / steps_ms, 3)}


def bench_volume(torch, dtype: str = "f32", n: int = 256, steps: int = 400, warmup: int = 20,
                 q: int = 19, cpu: bool = False) -> dict:
    """The three-dimensional step (D3Q19 or D3Q27) on the 256^3 half-space
    (free surface, sponges, source, 4096 surface receivers): a lean and a
    general launch per step, 2 x q population words per cell (152 B / 216 B
    in FP32)."""
    from workloads.problem3 import volume_half_space
    from paper_2009_06404_amd.solver3d import Solver3
    p = volume_half_space(n=n, nsteps=warmup + steps, q=q)
    s = Solver3(p, dtype=dtype, trace_steps=warmup + steps + 50)
    s.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    s.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    kt = s.step_timed(50)
    ok = bool(torch.isfinite(s.state()).all().item())
    tile = s.tile()
    width = s.lean_width
    s.close()
    esize = 4 if dtype == "f32" else 8
    per_cell = 2 * q * esize
    kms, kcells = kt["lean_ms"], kt["lean_cells"]
    gbps = per_cell * kcells / (kms / 1e3) / 1e9
    return {"workload": f"volume_half_space {n}^3 {dtype.upper()} (D3Q{q}): free surface top, "
                        f"24-cell sponges (rigid bottom, periodic sides), nu=0.25, vertical Ricker "
                        f"source at depth 12, {p.nrec} surface receivers",
            "GLUPS": round(p.cells / ms / 1e6, 3), "ms_per_step": round(ms, 4), "steps": steps,
            "warmup": warmup, "kernel": "step3_kernel (lean)", "kernel_ms": round(kms, 5),
            "cells_per_launch": kcells, "bytes_per_launch": per_cell * kcells,
            "kernel_GBps": round(gbps, 1), "frac": round(gbps / HBM_PEAK_GBS, 4),
            "general_kernel": {"cells_per_launch": kt["general_cells"],
                               "ms_per_launch": round(kt["general_ms"], 5)},
            "tile": list(tile), "lean_tile_columns": width, "state_finite": ok,
            **({"cpu_baseline": cpu_baseline3(p)} if cpu else {})}


def hbm_scale_band(p, rows: int = 2048):
    """The top `rows` rows of the HBM-scale grid as a grid of their own (free
    surface, the side sponges, the first layer's medium, the sources in the
    band), closed by a rigid edge: the oracle's per-cell work is that of the
    full grid, on 1/8 of its cells."""
    import numpy as np
    lam, mu, rho = p.medium.rows(p.ny)
    from workloads import BC_RIGID, Medium
    return p.replace(ny=rows, medium=Medium("layered", lam[:rows], mu[:rows], rho[:rows]),
                     rigid_row=-1, bc=(p.bc[0], BC_RIGID, p.bc[2], p.bc[3]),
                     sponge_thick=(p.sponge_thick[0], 0, p.sponge_thick[2], p.sponge_thick[3]),
                     sources=[q for q in p.sources if q.y < rows - 40],
                     receivers=np.zeros((0, 2), np.int32))


def bench_hbm_scale(torch, w, Solver, steps: int = 200, warmup: int = 20,
                    cpu: bool = False) -> dict:
    """16384^2 FP32, 8 layers, rigid interface, 3 sources (the HBM-scale
    configuration), timed over a window of its 4000 steps, with the roofline
    of its dominant kernel and the oracle timed on a band of the grid."""
    p = w.hbm_scale()
    s = Solver(p, dtype="f32", trace_steps=1)
    ms = _timed_steps(s, steps, warmup, torch)
    kt = s.step_timed(20)
    ok = s.check_finite()
    launch = s.launch()
    s.close()
    cells = p.nx * p.ny
    out = {"workload": f"hbm_scale {p.nx}x{p.ny} FP32, 8 layers, rigid interface at row "
                       f"{p.rigid_row}, 3 sources", "GLUPS": round(cells / ms / 1e6, 3),
           "ms_per_step": round(ms, 4), "steps": steps, "warmup": warmup,
           "roofline": roofline_block(kt, 4, f"hbm_scale_{p.nx}", "f32"),
           "launch": launch, "state_finite": bool(ok)}
    if cpu:
        band = hbm_scale_band(p)
        cb = cpu_baseline(band, target_s=10.0)
        cb["sample"] = (f"top {band.ny} rows of the {p.nx}x{p.ny} grid as a grid of their own "
                        f"(free surface, side sponges, first layer, rigid edge below): " + cb["sample"])
        out["cpu_baseline"] = cb
    return out


# triples of steps on the three-step path (blocks of 192 columns by 32 rows),
# 10 triples per captured HIP graph
BATCHED_LAUNCH = {"waves": 2, "rows": 8, "fuse_rows": 32, "fuse_steps": 3, "tri_waves": 3,
                  "graph_chunk": 30}
# 1024-column grids: narrow, short tiles for the adjoint kernels; the recorded
# forward (captured graphs of 10 pairs) and the recompute run on the two-step
# path (128-column blocks)
ADJOINT_LAUNCH = {"waves": 2, "rows": 4, "fuse_rows": 32, "graph_chunk": 20}


def bench_batched(torch, w, Solver, plain_glups: float, steps: int = 60,
                  warmup: int = 20, launch=None) -> dict:
    """512 grids of uneven side (256..2048) in one context, one launch of each
    kernel per triple of steps over the flat tile lists, the time loop captured
    in HIP graphs of 10 triples; then the same context launched directly (the
    same workspace: its placement in HBM moves the rate by several percent
    between allocations, so both forms are timed on one)."""
    probs = w.batched_shots()
    cells = sum(p.nx * p.ny for p in probs)
    lc = dict(launch or BATCHED_LAUNCH)
    t0 = time.perf_counter()
    s = Solver(probs, dtype="f32", trace_steps=1, launch=lc)
    setup = time.perf_counter() - t0
    ms = _timed_steps(s, steps, warmup, torch)
    graph_launch = s.launch()
    direct = dict(graph_launch)
    direct["graph_chunk"] = 0
    s.set_launch(**direct)
    ms_direct = _timed_steps(s, steps, warmup, torch)
    ok = s.check_finite()
    s.close()
    g = cells / ms / 1e6
    gd = cells / ms_direct / 1e6
    return {"workload": f"batched_shots: {len(probs)} grids, sides 256..2048, {cells} cells, FP32",
            "GLUPS": round(g, 3), "ms_per_step": round(ms, 4), "steps": steps,
            "warmup": warmup, "vs_plain": round(g / plain_glups, 4), "setup_s": round(setup, 1),
            "launch": graph_launch, "state_finite": bool(ok),
            "direct_launches": {"GLUPS": round(gd, 3), "ms_per_step": round(ms_direct, 4)},
            "graph_vs_direct": round(g / gd, 4)}


def kept_density_steps(torch, s, seg: int, nsteps: int, margin_gib: float = 16.0) -> int:
    """Steps whose densities an adjoint recording of nsteps steps can keep in
    the HBM left free, `margin_gib` GiB held back."""
    from paper_2009_06404_amd import _lib as L
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    base = L.lbm_adjoint_workspace_bytes(s.ctx, seg, nsteps)
    plane = (L.lbm_adjoint_workspace_bytes_resident(s.ctx, seg, nsteps, nsteps) - base) / nsteps
    avail = free - base - margin_gib * 2 ** 30
    return int(max(0, min(nsteps, avail // plane)))


def bench_adjoint(torch, w, Solver, plain_glups: float, nsteps: int = 5000,
                  seg: int = 100, launch=None) -> dict:
    """16 shots of 1024^2 FP32 through the perturbed medium, 5000 steps,
    checkpoints every 100: the full gradient (recorded forward, misfit,
    adjoint, Lame gradients) timed end to end, against the observed data of
    the homogeneous background (computed beforehand). Timed twice: with the
    densities of as many trailing segments as the free HBM holds kept from
    the recorded forward (no recompute there), and with every segment
    recomputed from its checkpoint; the gradients agree bit for bit except
    dL/damp, to rounding."""
    shots = w.adjoint_shots(nsteps=nsteps)
    bg = w.adjoint_shots(nsteps=nsteps, homogeneous=True)
    sb = Solver(bg, dtype="f32", trace_steps=nsteps)
    sb.step(nsteps)
    d_obs = [t.clone() for t in sb.traces]
    sb.close()
    del sb
    s = Solver(shots, dtype="f32", trace_steps=nsteps, launch=dict(launch or ADJOINT_LAUNCH))
    n = shots[0].nx
    G = len(shots)
    gk = torch.zeros((G, n, n), dtype=torch.float64, device="cuda")
    ga = torch.zeros((G, 1), dtype=torch.float64, device="cuda")
    gl = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    gm = torch.zeros_like(gl)
    cells = G * n * n

    init = [s.state(g).clone() for g in range(G)]   # the rest state at t = 0

    def gradient(kept: int) -> dict:
        for t_ in (gk, ga, gl, gm):
            t_.zero_()
        for g in range(G):
            s.set_state(g, init[g], 0)
        # the workspace is allocated once, outside the timed region (a 245 GB
        # allocation can take seconds after other workloads freed theirs);
        # fewer kept steps if the device refuses it
        while True:
            try:
                s.adjoint_reserve(nsteps, seg, kept)
                break
            except torch.cuda.OutOfMemoryError:
                if kept == 0:
                    raise
                kept //= 2
                torch.cuda.empty_cache()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e2 = torch.cuda.Event(enable_timing=True)
        e0.record()
        s.adjoint_begin(nsteps, seg, resident_steps=kept)
        s.step(nsteps)
        e1.record()
        mis = []
        for g in range(G):
            m, r = s.misfit(g, d_obs[g])
            mis.append(m)
            s.adjoint_set_io(g, r, gk[g], ga[g])
        s.adjoint_step(nsteps)
        for g in range(G):
            s.lame_gradient(g, gk[g], gl, gm)
        e2.record()
        torch.cuda.synchronize()
        t_all = e0.elapsed_time(e2)
        return {"kept_density_steps": kept,
                "gradient_GLUPS": round(cells * nsteps / (t_all / 1e3) / 1e9, 3),
                "ms_total": round(t_all, 1), "ms_forward_recorded": round(e0.elapsed_time(e1), 1),
                "misfit": float(sum(m.item() for m in mis)),
                "gradients_finite": bool(torch.isfinite(gl).all().item()
                                         and torch.isfinite(gm).all().item()),
                "gl": gl.clone()}

    with_kept = gradient(kept_density_steps(torch, s, seg, nsteps))
    kept = with_kept.pop("kept_density_steps")
    recompute = gradient(0)
    recompute.pop("kept_density_steps")
    same = bool(torch.equal(with_kept.pop("gl"), recompute.pop("gl")))
    del init
    kernels = adjoint_kernel_roofline(torch, s, seg)
    s.close()
    plane_gb = cells * 4 / 1e9
    return {"workload": f"adjoint_shots: {G} shots of {n}x{n} FP32, {nsteps} steps, "
                        f"checkpoints every {seg}",
            **with_kept, "vs_plain": round(with_kept["gradient_GLUPS"] / plain_glups, 4),
            "kept_density_steps": kept, "kept_density_GB": round(kept * plane_gb, 1),
            "recompute_every_segment": recompute, "dL_dlambda_bitwise_equal": same,
            "adjoint_kernels": kernels,
            "note": "gradient_GLUPS = cell-steps of the forward per second of forward + "
                    "misfit + adjoint (kept densities for the last kept_density_steps steps, "
                    "recompute from checkpoints for the others) + Lame gradients"}


# Algorithmic bytes per cell and launch of the adjoint kernels (FP32, cell-wise
# moduli, dL/dkappa asked): the two-step kernel reads fh(t+1) and writes
# fh(t-1) (9 + 9 words), reads rho(t), rho(t-1) and kappa (3 words) and
# reads and writes dL/dkappa (FP64, 16 B); the single-step interior kernel
# reads fh(t+1), writes fh(t) (18 words), reads rho(t) and kappa (2 words)
# and dL/dkappa (16 B).
ADJ_FUSED_BYTES = 21 * 4 + 16
ADJ_INTERIOR_BYTES = 20 * 4 + 16


def adjoint_kernel_roofline(torch, s, seg: int, nsteps: int = 400, timed: int = 200) -> dict:
    """Per-launch event timing of the adjoint kernels (lbm_adjoint_step_timed)
    over the last `timed` adjoint steps of a fresh recording of `nsteps` steps
    on the same context, and their HBM roofline on algorithmic bytes."""
    n_g = len(s.problems)
    gk = [torch.zeros((p.ny, p.nx), dtype=torch.float64, device="cuda") for p in s.problems]
    s.adjoint_begin(nsteps, seg)
    s.step(nsteps)
    for g in range(n_g):
        r = torch.randn_like(s.traces[g])
        s.adjoint_set_io(g, r, gk[g], None)
    s.adjoint_step(nsteps - timed)
    torch.cuda.synchronize()
    kt = s.adjoint_step_timed(timed)
    out = {"timed_steps": kt["steps"]}
    for name, cells, ms, per_cell, steps in (
            ("adjoint_fused2_kernel", kt["fused_cells"], kt["fused_ms"], ADJ_FUSED_BYTES, 2),
            ("adjoint_interior_kernel", kt["interior_cells"], kt["interior_ms"],
             ADJ_INTERIOR_BYTES, 1)):
        if cells <= 0 or ms <= 0:
            continue
        achieved = per_cell * cells / (ms / 1e3) / 1e9
        n = s.problems[0].nx
        out[name] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(traffic_file(name, f"adjoint_shots_{n}", "f32"),
                                                 cells),
                     "bytes_per_cell": per_cell, "cells_per_launch": cells,
                     "steps_per_launch": steps, "ms_per_launch": round(ms, 5)}
    out["adjoint_kernel_general"] = {"cells_per_launch": kt["general_cells"],
                                     "ms_per_launch": round(kt["general_ms"], 5)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=11900)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--n", type=int, default=4096, help="grid side")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--rows", type=int, default=0)
    ap.add_argument("--graph-chunk", type=int, default=-1,
                    help="steps per captured HIP graph; -1 keeps the library's default launch")
    ap.add_argument("--timed-launches", type=int, default=200,
                    help="steps of the per-kernel event-timing pass after the timed region")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the HBM-scale, batched and adjoint measurements")
    ap.add_argument("--only", choices=["hbm_scale", "single_step", "plain_f64", "batched",
                                       "adjoint", "filter", "volume", "volume27"],
                    help="run only this one of the extra measurements and print it")
    ap.add_argument("--adjoint-steps", type=int, default=5000)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 9 x n^2 floats (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the slab decomposition over xGMI is a design note); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as w
    from paper_2009_06404_amd import Solver

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        # A plain device copy of one population buffer's size: the reference for
        # the counter scale factors and the achievable read+write bandwidth.
        src = torch.ones(9 * args.n * args.n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 20
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4,
                          "launches": 25, "ms_per_copy": round(ms, 5),
                          "copy_GBps": round(2 * src.numel() * 4 / (ms / 1e3) / 1e9, 1)}), flush=True)
        return
    if args.only:
        fn = {"hbm_scale": lambda: bench_hbm_scale(torch, w, Solver, cpu=not args.no_cpu_baseline),
              "single_step": lambda: bench_plain_variant(torch, w, Solver, "f32",
                                                         {"fuse_rows": 0, "waves": 8, "rows": 8},
                                                         "single-step path"),
              "plain_f64": lambda: bench_plain_variant(torch, w, Solver, "f64", {},
                                                       "FP64, default launch"),
              "batched": lambda: bench_batched(torch, w, Solver, float("nan")),
              "adjoint": lambda: bench_adjoint(torch, w, Solver, float("nan"),
                                               nsteps=args.adjoint_steps),
              "filter": lambda: bench_filter(torch, w, Solver, float("nan")),
              "volume": lambda: bench_volume(torch, args.dtype, cpu=not args.no_cpu_baseline),
              "volume27": lambda: bench_volume(torch, args.dtype, q=27,
                                               cpu=not args.no_cpu_baseline)}[args.only]
        print(json.dumps({args.only: fn()}), flush=True)
        return
    p = w.plain_large(n=args.n, dtype=args.dtype)
    total = args.warmup + args.steps
    s = Solver(p, dtype=args.dtype, trace_steps=total)
    if args.autotune:
        s.autotune()
    launch = s.launch()
    if args.waves or args.rows:
        launch.update({k: v for k, v in (("waves", args.waves), ("rows", args.rows)) if v})
    if args.graph_chunk >= 0:
        launch["graph_chunk"] = args.graph_chunk
    s.set_launch(**launch)
    launch = s.launch()

    stream = torch.cuda.current_stream()
    s.step(args.warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    s.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    kt = s.step_timed(args.timed_launches)
    ok = s.check_finite()
    s.close()

    cells = p.nx * p.ny
    esize = 4 if args.dtype == "f32" else 8
    ms_step = ms / args.steps
    glups = cells * args.steps / (ms / 1e3) / 1e9
    rl = roofline_block(kt, esize, f"plain_large_{args.n}", args.dtype)
    step_gbs = 18 * esize * cells / (ms_step / 1e3) / 1e9
    rl["whole_step_GBps"] = round(step_gbs, 1)
    rl["note"] = ("whole_step_GBps: 18 population words per cell and step over the timed "
                  "steps -- above the HBM peak when several steps share one pass")
    out = {
        "metric": METRIC, "value": round(glups, 3), "unit": "GLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": f"plain_large {p.nx}x{p.ny} {args.dtype.upper()}: free surface top, "
                               f"96-cell sponges (rigid bottom, periodic sides), nu=0.33, "
                               f"vertical Ricker source at depth 20, {p.nx} surface receivers",
                   "nx": p.nx, "ny": p.ny, "tau": p.tau, "launch": launch,
                   "state_finite": bool(ok)},
        "roofline": rl,
    }
    if not args.no_extras and args.n == 4096 and args.dtype == "f32":
        extras = {}
        for name, fn in (("hbm_scale", lambda: bench_hbm_scale(torch, w, Solver,
                                                               cpu=not args.no_cpu_baseline)),
                         ("single_step", lambda: bench_plain_variant(
                             torch, w, Solver, "f32", {"fuse_rows": 0, "waves": 8, "rows": 8},
                             "single-step path")),
                         ("plain_f64", lambda: bench_plain_variant(
                             torch, w, Solver, "f64", {}, "FP64, default launch")),
                         ("batched", lambda: bench_batched(torch, w, Solver, glups)),
                         ("adjoint", lambda: bench_adjoint(torch, w, Solver, glups)),
                         ("filter", lambda: bench_filter(torch, w, Solver, ms_step)),
                         ("volume_d3q19", lambda: bench_volume(torch, cpu=not args.no_cpu_baseline)),
                         ("volume_d3q27", lambda: bench_volume(torch, q=27, cpu=not args.no_cpu_baseline))):
            print(f"[bench] {name} ...", file=sys.stderr, flush=True)
            extras[name] = fn()
            torch.cuda.empty_cache()
        out["extras"] = extras
    out["device"] = device_report(torch)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
