"""Benchmark: GDOF/s per SSP-RK3 stage of the P3 Euler DG hot path on one MI355X.

Workload (the precision-form configuration): isentropic vortex (strength 5, Mach 0.5) on
the periodic [0,10]^3 cube split into 64^3 hexahedra x 6 = 1,572,864 tets, P3 (20 modes,
5 variables: 157,286,400 DOF), element order shuffled from a seed and renumbered along a
Hilbert curve.  One step = one SSP-RK3 step = three fused residual+update launches.

The headline value is the mixed fp16 path (fp16 MFMA contractions with fp32 accumulation,
fp32 fluxes, fp64 state); the same workload is also timed in fp32, bf16-mixed and fp64, the
residual entry point is timed, and each precision's result is compared with the fp64 GPU
result: the state after the timed steps (relative to the whole state and to the increment)
and one residual of the initial state.  cpu_baseline is the FP64 CPU oracle at the 48^3 x 6
size (all host threads: one residual by dual-phase timing and one SSP-RK3 step; one thread on
a 14^3 x 6 sample).  stream_ceiling is the practical bandwidth of the box; counters are the
committed shader-counter summary of the stage kernel (when its sources are unchanged); the
extra workloads (--extras) are P4, the adjoint, the viscous terms, Roe's flux, temporal mixed
precision, graph replay on the smallest mesh and the element-renumbering ablation.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from synthetic import fields, kuhn_cube  # noqa: E402

HBM_PEAK_GBS = 8000.0
ALU_PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}  # MI355X vector (fp64 = its MFMA rate)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stage_kernel_p3_64cube_traffic.json")
KERNEL_SOURCES = ["dg_stage.hip", "dg_kernels.hpp", "dg_common.hpp", "dg_launch.hpp", "dg_tile.hpp"]


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2209_01877_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(precision: str):
    """HBM bytes per stage launch from the committed counter summary (FETCH_SIZE + WRITE_SIZE,
    scaled by the copy-kernel calibration), or None when the kernel sources changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("source_sha256") != kernel_source_hash() or precision not in d.get("per_precision", {}):
        return None
    r = d["per_precision"][precision]
    return (r["fetch_kib_per_dispatch"] * d["copy_fetch_factor"] + r["write_kib_per_dispatch"] * d["copy_write_factor"]) * 1024.0


def measured_counters():
    """Per precision, the stage kernel's MFMA utilisation, VALU busy fraction, L2 hit rate and
    wave wait fraction from the committed counter summary (rocprofv3 passes over the same
    benchmark; MFMA utilisation = SQ_VALU_MFMA_BUSY_CYCLES over the SIMD-cycles of the
    dispatch, 32 x SQ_CYCLES), or None when the kernel sources changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("source_sha256") != kernel_source_hash():
        return None
    out = {}
    for prec, r in d.get("per_precision", {}).items():
        if "mfma_util" in r:
            out[prec] = {k: r[k] for k in ("mfma_util", "valu_busy", "wait_frac", "tcc_hit_rate", "avg_kernel_us")
                         if k in r}
    return {"per_precision": out, "source": os.path.relpath(TRAFFIC_FILE, ROOT),
            "definition": "mfma_util = SQ_VALU_MFMA_BUSY_CYCLES / (32 SQ_CYCLES); valu_busy = 4 SQ_ACTIVE_INST_VALU / "
                          "(32 SQ_CYCLES); wait_frac = SQ_WAIT_ANY / SQ_WAVE_CYCLES; tcc_hit_rate = TCC_HIT / "
                          "(TCC_HIT + TCC_MISS)"} if out else None


def stage_flops(p: int) -> float:
    """Flops per element and stage of the element-centric path: contractions
    2 * 5 * N_p * (4 N_q + 12 N_f) (volume interpolation, 3-direction projection, own and
    neighbour traces, lift) and pointwise work 60 N_q + 100 * 4 N_f."""
    np_ = (p + 1) * (p + 2) * (p + 3) // 6
    nq, nf = (p + 1) ** 3, (p + 1) ** 2
    return 2.0 * 5 * np_ * (4 * nq + 12 * nf) + 60.0 * nq + 400.0 * nf


def stage_bytes(n_elem: int, n_modes: int, state_bytes: int) -> float:
    """Algorithmic HBM bytes of one SSP-RK3 step (three stages): per element the state read
    (U_in), the stage base U0 (stages 2 and 3), the result write, the geometry (9 + 1 fp64)
    and the topology (4 neighbour ids + packed face codes, int32)."""
    st = 5 * n_modes * state_bytes
    per_elem = (2 * st) + 2 * (3 * st) + 3 * (80 + 20)
    return float(n_elem) * per_elem


def stage_bytes_split(n_elem: int, n_modes: int, state_bytes: int) -> float:
    """The same for the mixed modes up to P3, whose rk_step regroups the update so that only
    the second stage reads U0 (it stores U0/3 + 2 U2/3 and U2's fp64 cell means, 40 B, which
    the third stage reads): one state array per step fewer, plus the means written and read."""
    st = 5 * n_modes * state_bytes
    per_elem = (2 * st) + (3 * st + 40) + (2 * st + 40) + 3 * (80 + 20)
    return float(n_elem) * per_elem


def residual_bytes(n_elem: int, n_modes: int, state_bytes: int) -> float:
    """Algorithmic HBM bytes of one residual evaluation: the state read, R written, geometry
    and topology per element (1,700 B at P3 with an fp64 state)."""
    st = 5 * n_modes * state_bytes
    return float(n_elem) * (2 * st + 80 + 20)


def progress(msg: str) -> None:
    """One line per finished part of the run, on stderr (the JSON line alone goes to stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def timed(fn, steps: int, warmup: int) -> float:
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / 1000.0


def run_gpu(args):
    from paper_2209_01877_amd import Solver

    n = args.n
    p = args.p
    mesh = kuhn_cube(n, length=10.0, shuffle_seed=2209, vid_seed=2210)
    vortex = lambda x: fields.isentropic_vortex(x, length=10.0, beta=5.0, mach=0.5)  # noqa: E731
    results = {}
    states, init_states, res_states = {}, {}, {}
    dt = None
    for prec in args.precisions:
        s = Solver(p, prec)
        t0 = time.time()
        s.upload(mesh, renumber=args.renumber)
        upload_s = time.time() - t0
        U = s.project_fn(vortex)
        if dt is None:
            # CFL 0.2 rule on the undisturbed spacing: d_K >= 0.41 h for the Kuhn split,
            # max |u| + c <= 3.1 for this vortex
            h = 10.0 / n
            dt = 0.2 * 0.41 * h / ((2 * p + 1) * 3.1)
        work = s.new_work()
        U0 = U.clone()
        # warm-up, then exactly `steps` SSP-RK3 steps in one call (the mixed modes build the
        # operand companion of U once per call; each stage writes the next one's)
        s.rk_step(U, dt, args.warmup, work)
        t = timed(lambda: s.rk_step(U, dt, args.steps, work), 1, 0)
        # dual-phase timing (difference of two run lengths, as in the paper's measurement):
        # removes the per-call fixed cost (companion build, launch of the first stage)
        t_short = timed(lambda: s.rk_step(U, dt, 10, work), 1, 0)
        t_long = timed(lambda: s.rk_step(U, dt, 10 + args.steps, work), 1, 0)
        s.sync()
        dof = mesh.n_elem * s.n_modes * 5
        stages = 3 * args.steps
        gdofs = dof * stages / t / 1e9
        R = s.new_state()
        tr = timed(lambda: s.residual(U, R), args.steps, args.warmup)
        # residual of the initial (projected) state, for the residual-level error
        s.residual(U0, R)
        res_states[prec] = s.get_state(R)
        if prec == "fp64":
            init_states[prec] = s.get_state(U0)
        # reproducible end state: restart from U0 for exactly `steps` steps
        U.copy_(U0)
        s.rk_step(U, dt, args.steps, work)
        states[prec] = s.get_state(U)
        s.sync()
        sb = 4 if prec == "fp32" else 8
        results[prec] = {
            "gdof_per_s_per_stage": gdofs,
            "ms_per_step": 1e3 * t / args.steps,
            "dual_phase_gdof_per_s_per_stage": dof * stages / (t_long - t_short) / 1e9,
            "residual_gdof_per_s": dof * args.steps / tr / 1e9,
            "residual_ms": 1e3 * tr / args.steps,
            # the residual entry point (in the mixed modes: companion pack + residual kernel)
            # against the HBM roof on its algorithmic bytes
            "residual_hbm_gb_per_s": residual_bytes(mesh.n_elem, s.n_modes, sb) * args.steps / tr / 1e9,
            "residual_hbm_frac": residual_bytes(mesh.n_elem, s.n_modes, sb) * args.steps / tr / 1e9 / HBM_PEAK_GBS,
            "stage_hbm_gb_per_s": stage_bytes(mesh.n_elem, s.n_modes, sb) * args.steps / t / 1e9,
            "upload_s": upload_s,
        }
        progress(f"{prec}: {gdofs:.1f} GDOF/s per stage")
        if prec in ALU_PEAK_TFLOPS:  # the FP64 and FP32 paths against their ALU roof
            tf = stage_flops(p) * mesh.n_elem * stages / t / 1e12
            results[prec]["alu_tflops"] = tf
            results[prec]["alu_frac"] = tf / ALU_PEAK_TFLOPS[prec]
        del s, U, U0, work, R
        torch.cuda.empty_cache()
    if "fp64" in states:
        ref, ref0, ref_r = states["fp64"], init_states["fp64"], res_states["fp64"]
        for prec, U in states.items():
            results[prec].update(l2_errors(U, ref))
            # the error that matters to a user: against what the run changed (the increment of
            # the fp64 run over the timed steps), and at the level of one residual evaluation
            inc = error_vs(U - ref0, ref - ref0)
            results[prec]["increment_rel_l2_vs_fp64"] = inc["all"]
            results[prec]["increment_rel_l2_vs_fp64_per_var"] = inc["per_var"]
            rr = error_vs(res_states[prec], ref_r)
            results[prec]["residual_rel_l2_vs_fp64"] = rr["all"]
            results[prec]["residual_rel_l2_vs_fp64_per_var"] = rr["per_var"]
    return mesh, dt, results


def l2_errors(U, ref):
    """Relative L2 difference of coefficient arrays (E, 5, N_p) against the norm of the whole
    state: over all variables, and per variable (each variable's difference over the norm of
    the whole state).  The free stream dominates that norm, so this is the smallest of the
    reported errors; see error_vs for the ones relative to the increment and the residual."""
    diff = (U - ref).pow(2).sum(dim=(0, 2)).sqrt()
    total = ref.pow(2).sum().sqrt()
    return {"rel_l2_vs_fp64": float((U - ref).pow(2).sum().sqrt() / total),
            "rel_l2_vs_fp64_per_var": (diff / total).tolist()}


def error_vs(x, ref):
    """Relative L2 difference of x from ref (coefficient arrays (E, 5, N_p); the mesh's
    elements have equal volumes, so this is the function-space norm): over all variables, and
    per variable against that variable's own reference norm (None where the reference
    variable's norm is below 1e-3 of the largest one: the w-momentum of the z-invariant vortex,
    whose increment and residual are quadrature round-off, not flow)."""
    d = (x - ref).pow(2).sum(dim=(0, 2)).sqrt()
    n = ref.pow(2).sum(dim=(0, 2)).sqrt()
    big = float(n.max())
    per = [float(d[v] / n[v]) if float(n[v]) > 1e-3 * big else None for v in range(d.numel())]
    return {"all": float(d.pow(2).sum().sqrt() / n.pow(2).sum().sqrt()), "per_var": per}


def run_p4(args):
    """P4 (35 modes) vortex on 40^3 x 6 tets: mixed vs fp32 GDOF/s per stage and error vs fp64."""
    from paper_2209_01877_amd import Solver

    mesh = kuhn_cube(40, length=10.0, shuffle_seed=2209, vid_seed=2210)
    p = 4
    dt = 0.2 * 0.41 * (10.0 / 40) / ((2 * p + 1) * 3.1)
    vortex = lambda x: fields.isentropic_vortex(x, length=10.0, beta=5.0, mach=0.5)  # noqa: E731
    out, states = {}, {}
    for prec in ["bf16", "fp32", "fp64"]:
        s = Solver(p, prec)
        s.upload(mesh, renumber=args.renumber)
        U = s.project_fn(vortex)
        work = s.new_work()
        U0 = U.clone()
        s.rk_step(U, dt, args.warmup, work)
        t = timed(lambda: s.rk_step(U, dt, args.steps, work), 1, 0)
        U.copy_(U0)
        s.rk_step(U, dt, args.steps, work)
        states[prec] = s.get_state(U)
        s.sync()
        out[prec] = {"gdof_per_s_per_stage": mesh.n_elem * s.n_modes * 5 * 3 * args.steps / t / 1e9,
                     "ms_per_step": 1e3 * t / args.steps}
        del s, U, U0, work
        torch.cuda.empty_cache()
    for prec in out:
        out[prec].update(l2_errors(states[prec], states["fp64"]))
    out["workload"] = f"isentropic vortex, P4, periodic 40^3 x 6 ({mesh.n_elem} tets), {args.steps} SSP-RK3 steps"
    return out


def run_roe(args):
    """The paper's own interface flux (Roe) on the main workload (P3 vortex, 64^3 x 6): GDOF/s
    per stage in bf16, fp32 and fp64, and the bf16/fp32 states after the timed steps against
    the fp64 Roe state."""
    from paper_2209_01877_amd import Solver

    mesh = kuhn_cube(args.n, length=10.0, shuffle_seed=2209, vid_seed=2210)
    p = args.p
    dt = 0.2 * 0.41 * (10.0 / args.n) / ((2 * p + 1) * 3.1)
    vortex = lambda x: fields.isentropic_vortex(x, length=10.0, beta=5.0, mach=0.5)  # noqa: E731
    out, states = {}, {}
    for prec in ["bf16", "fp32", "fp64"]:
        s = Solver(p, prec)
        s.upload(mesh, renumber=args.renumber)
        s.set_flux("roe")
        U = s.project_fn(vortex)
        work = s.new_work()
        U0 = U.clone()
        s.rk_step(U, dt, args.warmup, work)
        t = timed(lambda: s.rk_step(U, dt, args.steps, work), 1, 0)
        U.copy_(U0)
        s.rk_step(U, dt, args.steps, work)
        states[prec] = s.get_state(U)
        s.sync()
        out[prec] = {"gdof_per_s_per_stage": mesh.n_elem * s.n_modes * 5 * 3 * args.steps / t / 1e9}
        del s, U, U0, work
        torch.cuda.empty_cache()
    for prec in out:
        out[prec].update(l2_errors(states[prec], states["fp64"]))
    out["workload"] = (f"isentropic vortex, P{p}, periodic {args.n}^3 x 6 ({mesh.n_elem} tets), Roe flux, "
                       f"{args.steps} SSP-RK3 steps")
    return out


def run_temporal_mixed(args):
    """The paper's temporal mixed precision (Sec. III.B, Table 2) on the main workload: of
    `steps` SSP-RK3 steps the first N run in a low precision and the rest in FP64 (state
    handed over through the caller layout).  Time per step and the final state's difference
    from the all-FP64 run, for N = 0, steps/2 and steps with bf16 and fp32."""
    from paper_2209_01877_amd.schedule import TemporalMixed

    mesh = kuhn_cube(args.n, length=10.0, shuffle_seed=2209, vid_seed=2210)
    p = args.p
    n = args.steps
    dt = 0.2 * 0.41 * (10.0 / args.n) / ((2 * p + 1) * 3.1)
    vortex = lambda x: fields.isentropic_vortex(x, length=10.0, beta=5.0, mach=0.5)  # noqa: E731
    out = {}
    ref = None
    for low in ["bf16", "fp32"]:
        tm = TemporalMixed(p, mesh, low=low, renumber=args.renumber)
        U0 = tm.high.get_state(tm.high.project_fn(vortex))
        tm.run(U0, dt, 1, 2)  # warm-up of both contexts
        for n_low in (0, n // 2, n):
            if low == "fp32" and n_low == 0:
                continue  # the all-FP64 run does not depend on the low precision
            start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            start.record()
            U = tm.run(U0, dt, n_low, n)
            stop.record()
            torch.cuda.synchronize()
            t = start.elapsed_time(stop) / 1e3
            if n_low == 0:
                ref = U
            key = "fp64" if n_low == 0 else f"{low}_first_{n_low}"
            out[key] = {"ms_per_step": 1e3 * t / n, **l2_errors(U, ref)}
        del tm, U0, U
        torch.cuda.empty_cache()
    out["workload"] = (f"isentropic vortex, P{p}, periodic {args.n}^3 x 6 ({mesh.n_elem} tets), {n} SSP-RK3 "
                       "steps, the first N in a low precision (includes the hand-over)")
    return out


def run_small_graph(args):
    """Launch-bound case: P1 density wave on the 4^3 x 6 = 384-tet cube (the smallest
    configuration), 100 SSP-RK3 steps per call, FP64 and bf16: eager launches against a
    replay of the same 100 steps captured in a HIP graph (best of 5 each)."""
    from paper_2209_01877_amd import Solver

    mesh = kuhn_cube(4)
    out = {}
    n = 100
    for prec in ["fp64", "bf16"]:
        s = Solver(1, prec)
        s.upload(mesh, renumber=args.renumber)
        U0 = s.project_fn(lambda x: fields.sine_wave(x))
        dt = 2.26e-3
        work = s.new_work()
        U = U0.clone()
        s.rk_step(U, dt, n, work)
        t_eager = min(timed(lambda: s.rk_step(U, dt, n, work), 1, 0) for _ in range(5))
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            s.rk_step(U, dt, n, work)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            s.rk_step(U, dt, n, work)
        g.replay()
        t_graph = min(timed(g.replay, 1, 0) for _ in range(5))
        out[prec] = {"eager_us_per_step": 1e6 * t_eager / n, "graph_us_per_step": 1e6 * t_graph / n,
                     "graph_speedup": t_eager / t_graph}
        del g, s, U, U0, work
        torch.cuda.empty_cache()
    out["workload"] = f"density wave, P1, periodic 4^3 x 6 ({mesh.n_elem} tets), {n} SSP-RK3 steps per call"
    return out


def run_navier_stokes(args):
    """Viscous (BR1) form: P3 vortex on 48^3 x 6 with mu = 1e-3, FP64 and FP32: GDOF/s per
    SSP-RK3 stage with the viscous terms, beside the same workload without them."""
    from paper_2209_01877_amd import Solver

    mesh = kuhn_cube(48, length=10.0, shuffle_seed=2209, vid_seed=2210)
    p = 3
    dt = 0.2 * 0.41 * (10.0 / 48) / ((2 * p + 1) * 3.1)
    vortex = lambda x: fields.isentropic_vortex(x, length=10.0, beta=5.0, mach=0.5)  # noqa: E731
    out = {}
    for prec in ["fp64", "fp32"]:
        row = {}
        for mu in (1e-3, 0.0):
            s = Solver(p, prec)
            if mu > 0.0:
                s.set_viscosity(mu, 0.72)
            s.upload(mesh, renumber=args.renumber)
            U = s.project_fn(vortex)
            work = s.new_work()
            s.rk_step(U, dt, 1, work)
            steps = max(2, args.steps // 4)
            t = timed(lambda: s.rk_step(U, dt, steps, work), 1, 0)
            s.sync()
            key = "navier_stokes" if mu > 0.0 else "euler"
            row[key + "_gdof_per_s_per_stage"] = mesh.n_elem * s.n_modes * 5 * 3 * steps / t / 1e9
            del s, U, work
            torch.cuda.empty_cache()
        out[prec] = row
    out["workload"] = f"isentropic vortex, P3, 48^3 x 6 ({mesh.n_elem} tets), mu = 1e-3, Pr = 0.72"
    return out


def run_renumbering(args):
    """Grid renumbering (the paper's Sec. III.B: RCMK, +20-30 % overall on its grids, Table 1)
    on the C2 workload: the P3 vortex on 48^3 x 6 = 663,552 tets, element order shuffled from
    seed 2209, then kept (none) or renumbered by RCM, Morton or Hilbert; GDOF/s per SSP-RK3
    stage in FP64 and mixed bf16, with the bandwidth (max |i - j| over face neighbours) and the
    share of neighbour pairs closer than 64 in the new order."""
    from paper_2209_01877_amd import Solver

    n, p = 48, 3
    mesh = kuhn_cube(n, length=10.0, shuffle_seed=2209, vid_seed=2210)
    dt = 0.2 * 0.41 * (10.0 / n) / ((2 * p + 1) * 3.1)
    vortex = lambda x: fields.isentropic_vortex(x, length=10.0, beta=5.0, mach=0.5)  # noqa: E731
    steps = max(2, args.steps // 2)
    out = {}
    for order in ("none", "rcm", "morton", "hilbert"):
        row = {}
        for prec in ("fp64", "bf16"):
            s = Solver(p, prec)
            s.upload(mesh, renumber=order)
            st = s.mesh_stats()
            U = s.project_fn(vortex)
            work = s.new_work()
            s.rk_step(U, dt, 1, work)
            t = timed(lambda: s.rk_step(U, dt, steps, work), 1, 0)
            s.sync()
            row[prec + "_gdof_per_s_per_stage"] = mesh.n_elem * s.n_modes * 5 * 3 * steps / t / 1e9
            row["bandwidth"] = st["bandwidth"]
            row["near64_frac"] = st["near64"] / max(1, 2 * st["interior_faces"])
            del s, U, work
            torch.cuda.empty_cache()
        out[order] = row
    for prec in ("fp64", "bf16"):
        base = out["none"][prec + "_gdof_per_s_per_stage"]
        for order in ("rcm", "morton", "hilbert"):
            out[order][prec + "_gain_vs_none"] = out[order][prec + "_gdof_per_s_per_stage"] / base - 1.0
    out["workload"] = (f"isentropic vortex, P{p}, periodic {n}^3 x 6 ({mesh.n_elem} tets), shuffled element order, "
                       f"{steps} SSP-RK3 steps per timing")
    out["paper"] = "RCMK renumbering: +20-30 % overall runtime on the paper's 2-D grids (Sec. III.B, Table 1)"
    return out


def run_adjoint(args):
    """Differentiation form: P2 on the jittered 40^3 x 6 cube; time of the residual VJP over
    the time of the residual (fp64 and fp32)."""
    from paper_2209_01877_amd import Solver

    mesh = kuhn_cube(40, jitter=0.2, jitter_seed=1877, shuffle_seed=2209)
    out = {}
    for prec in ["fp64", "fp32"]:
        s = Solver(2, prec)
        s.upload(mesh, renumber=args.renumber)
        U = s.project_fn(fields.RandomSmooth(42))
        W = torch.randn(U.shape, dtype=U.dtype, device=U.device, generator=torch.Generator(device="cuda").manual_seed(43))
        R = s.new_state()
        Ub = s.new_state()
        tf = timed(lambda: s.residual(U, R), args.steps, args.warmup)
        tb = timed(lambda: s.residual_vjp(U, W, Ub), args.steps, args.warmup)
        s.sync()
        out[prec] = {"residual_ms": 1e3 * tf / args.steps, "vjp_ms": 1e3 * tb / args.steps,
                     "adjoint_over_forward": tb / tf}
        del s, U, W, R, Ub
        torch.cuda.empty_cache()
    out["workload"] = f"P2, jittered 40^3 x 6 ({mesh.n_elem} tets), RandomSmooth(42) state, Gaussian cotangent"
    return out


def cpu_model() -> str:
    """The host CPU's model string as lscpu prints it (Model name, plus BIOS Model name when
    present), else /proc/cpuinfo's."""
    import subprocess

    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        fields = {}
        for ln in txt.splitlines():
            if ":" in ln:
                k, v = ln.split(":", 1)
                fields.setdefault(k.strip(), v.strip())
        names = [fields[k] for k in ("Model name", "BIOS Model name") if fields.get(k)]
        if names:
            # the family / model / stepping numbers identify the part where a virtualised
            # host reports only a generic model name
            ids = ", ".join(f"{k.lower()} {fields[k]}" for k in ("CPU family", "Model", "Stepping") if fields.get(k))
            extra = [fields[k] + " " + k.lower() for k in ("Socket(s)",) if fields.get(k)]
            return " / ".join(dict.fromkeys(names)) + (f" ({ids})" if ids else "") + (f", {extra[0]}" if extra else "")
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as fh:
            return next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        return ""


def cpu_baseline(p: int, n_cpu: int, steps: int):
    """The FP64 oracle (torch-CPU, face-centric, untuned) on the host's cores, as planned for
    the C2 size: the P3 vortex on 48^3 x 6 = 663,552 tets.  One residual by dual-phase timing
    (two evaluations minus one, the paper's measurement) and one SSP-RK3 step; `value` is the
    step's rate per stage.  A one-thread run of one step on a 14^3 x 6 sample mirrors the
    paper's serial baseline.  (n_cpu / steps: a smaller multi-thread sample instead of C2
    when n_cpu is not 48.)"""
    from oracle.dg import DG

    torch.set_num_threads(max(1, len(os.sched_getaffinity(0))))
    mesh = kuhn_cube(n_cpu, length=10.0, shuffle_seed=2209, vid_seed=2210)
    t_setup = time.time()
    dg = DG(p, mesh.elem_vid, mesh.elem_xyz)
    U = dg.project(lambda x: fields.isentropic_vortex(x, length=10.0))
    t_setup = time.time() - t_setup
    dt = 0.2 * 0.41 * (10.0 / n_cpu) / ((2 * p + 1) * 3.1)
    t0 = time.time()
    dg.residual(U)
    t1 = time.time()
    dg.residual(U)
    dg.residual(U)
    t2 = time.time()
    t_res = (t2 - t1) - (t1 - t0)  # dual phase: T(2) - T(1)
    t0 = time.time()
    for _ in range(steps):
        U = dg.rk3_step(U, dt)
    t_step = (time.time() - t0) / steps
    dof = mesh.n_elem * dg.Np * 5
    cores = torch.get_num_threads()
    # the same oracle on one thread (the paper's serial baseline), on a smaller sample
    n1 = 14
    torch.set_num_threads(1)
    mesh1 = kuhn_cube(n1, length=10.0, shuffle_seed=2209, vid_seed=2210)
    dg1 = DG(p, mesh1.elem_vid, mesh1.elem_xyz)
    U1 = dg1.project(lambda x: fields.isentropic_vortex(x, length=10.0))
    dt1 = 0.2 * 0.41 * (10.0 / n1) / ((2 * p + 1) * 3.1)
    t1 = time.time()
    U1 = dg1.rk3_step(U1, dt1)
    t1 = time.time() - t1
    torch.set_num_threads(cores)
    return {
        "value": dof * 3 / t_step / 1e9,
        "unit": "GDOF/s per RK stage",
        "cores": cores,
        "kind": "oracle",
        "sample": f"P3 vortex on {n_cpu}^3 x 6 = {mesh.n_elem} tets, fp64 torch-CPU, face-centric, untuned: "
                  f"{steps} SSP-RK3 step(s) ({t_step:.1f} s per step), one residual by dual-phase timing "
                  f"({t_res:.2f} s), setup {t_setup:.1f} s",
        "residual_dual_phase_s": t_res,
        "residual_gdof_per_s": dof / t_res / 1e9 if t_res > 0 else None,
        "step_s": t_step,
        "cpu_model": cpu_model(),
        "single_thread": {"value": mesh1.n_elem * dg1.Np * 5 * 3 / t1 / 1e9, "unit": "GDOF/s per RK stage",
                          "sample": f"P3 vortex on {n1}^3 x 6 = {mesh1.n_elem} tets, 1 SSP-RK3 step ({t1:.1f} s)"},
    }


def stream_ceiling(nbytes: int = 1 << 30, reps: int = 5) -> dict:
    """Practical HBM bandwidth: the library's streaming probe (16-byte non-temporal accesses)
    over two device buffers of nbytes, timed with HIP events on the launch stream; best of reps
    after one untimed pass per kind.  Copy moves 2 x nbytes, read and write nbytes."""
    from paper_2209_01877_amd import stream_probe

    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    out = {}
    for kind, moved in (("copy", 2 * nbytes), ("read", nbytes), ("write", nbytes)):
        stream_probe(kind, src, dst)
        best = math.inf
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            stream_probe(kind, src, dst)
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1) / 1e3)
        out[kind] = moved / best / 1e9
        if kind == "copy" and not torch.equal(dst, src):
            raise RuntimeError("stream probe: the copy differs from its source")
    if torch.count_nonzero(dst).item() != 0:  # the last pass was the zero fill
        raise RuntimeError("stream probe: the zero fill left non-zero data")
    # last-level cache (256 MB MALL): cached reads of a 128 MiB buffer, larger than the 8 x 4 MB
    # of L2, after one pass that brings it in; 10 back-to-back launches between the events,
    # so the launch gaps count against it (a lower bound)
    mall_bytes = 128 << 20
    msrc = src[: mall_bytes // 4]
    stream_probe("read_cached", msrc, dst)
    best = math.inf
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            stream_probe("read_cached", msrc, dst)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    out["mall_read"] = 10 * mall_bytes / best / 1e9
    del src, dst, msrc
    torch.cuda.empty_cache()
    return {"copy": out["copy"], "read": out["read"], "write": out["write"], "mall_read": out["mall_read"],
            "unit": "GB/s", "buffer_bytes": nbytes, "mall_buffer_bytes": mall_bytes,
            "method": f"best of {reps}, 16-byte accesses (non-temporal except mall_read)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=64, help="hexahedra per cube edge")
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--renumber", default="hilbert")
    ap.add_argument("--precisions", default="fp16,fp32,bf16,fp64",
                    help="the first is the headline (the mixed mode with fp16 operands: as fast as bf16 and "
                         "eight times more accurate on this path)")
    ap.add_argument("--cpu-n", type=int, default=48, help="oracle sample: hexahedra per edge (48: the C2 size)")
    ap.add_argument("--cpu-steps", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the extra workloads (--extras)")
    ap.add_argument("--extras", default="p4,adjoint,navier_stokes,roe,temporal_mixed,small_graph,renumbering",
                    help="which of those to run")
    ap.add_argument("--copy-calibration", action="store_true", help="run a 1 GiB device copy first")
    args = ap.parse_args()
    args.precisions = args.precisions.split(",")
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU design is "
              "documented but not built", file=sys.stderr)
        sys.exit(2)
    if "RANK" in os.environ and int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py is single-GPU; launch it without torch.distributed", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        # a plain device copy of known size, for scaling FETCH_SIZE / WRITE_SIZE counters
        n = 256 * 1024 * 1024
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"copy calibration: {4 * n} bytes read and written", file=sys.stderr)
        del src, dst
    ceiling = stream_ceiling()
    mesh, dt, res = run_gpu(args)
    head = args.precisions[0]
    r = res[head]
    st_bytes = 4 if head == "fp32" else 8
    n_modes = (args.p + 1) * (args.p + 2) * (args.p + 3) // 6
    achieved = stage_bytes(mesh.n_elem, n_modes, st_bytes) / 3.0 / (r["ms_per_step"] / 3.0 / 1e3) / 1e9
    line = {
        "metric": "GDOF/s per RK stage (P3 Euler), mixed vs FP32 at stated err; adjoint/fwd time",
        "value": r["gdof_per_s_per_stage"],
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "data": "synthetic",
        "config": {
            "workload": f"isentropic vortex, P{args.p}, periodic {args.n}^3 x 6 Kuhn tets "
                        f"({mesh.n_elem} elements), shuffled + {args.renumber} renumbering, SSP-RK3, dt {dt:.3e}",
            "n_elem": mesh.n_elem,
            "order": args.p,
            "dof": mesh.n_elem * n_modes * 5,
            "precision": head,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(head),
        },
        "per_precision": res,
        "error_normalisation": (
            "per precision, against the GPU FP64 run of the same workload (which matches the FP64 oracle to "
            "1e-12): rel_l2_vs_fp64 = |U - U_fp64| / |U_fp64| after the timed steps (whole-state norm, the "
            "smallest figure); increment_rel_l2_vs_fp64 = |U - U_fp64| / |U_fp64 - U_initial| (what the steps "
            "changed); residual_rel_l2_vs_fp64 = |R - R_fp64| / |R_fp64| for one residual of the initial state, "
            "per variable against that variable's norm"),
    }
    if head in ("bf16", "fp16") and args.p <= 3:
        # the mixed path's own algorithmic bytes (regrouped SSP-RK3), which the standard
        # per-element figure used in "roofline" does not credit
        own = stage_bytes_split(mesh.n_elem, n_modes, st_bytes) / 3.0 / (r["ms_per_step"] / 3.0 / 1e3) / 1e9
        line["roofline_regrouped_rk3"] = {
            "bytes_per_element_stage": stage_bytes_split(1, n_modes, st_bytes) / 3.0,
            "standard_bytes_per_element_stage": stage_bytes(1, n_modes, st_bytes) / 3.0,
            "achieved": own, "unit": "GB/s", "frac": own / HBM_PEAK_GBS}
    line["counters"] = measured_counters()
    # the same stage against the box's practical bandwidth (a tuned streaming copy)
    stage_s = r["ms_per_step"] / 3.0 / 1e3
    traffic = line["roofline"]["traffic"]
    ceiling["stage_algorithmic_frac_of_copy"] = achieved / ceiling["copy"]
    ceiling["stage_traffic_GBps"] = None if traffic is None else traffic / stage_s / 1e9
    ceiling["stage_traffic_frac_of_copy"] = None if traffic is None else traffic / stage_s / 1e9 / ceiling["copy"]
    line["stream_ceiling"] = ceiling
    if "fp32" in res and head != "fp32":
        line["speedup_vs_fp32"] = r["gdof_per_s_per_stage"] / res["fp32"]["gdof_per_s_per_stage"]
    extras = [] if args.no_extra else args.extras.split(",")
    runs = [("p4", "p4_precision_form", run_p4), ("adjoint", "adjoint", run_adjoint),
            ("navier_stokes", "navier_stokes", run_navier_stokes), ("roe", "roe_flux", run_roe),
            ("temporal_mixed", "temporal_mixed_precision", run_temporal_mixed),
            ("small_graph", "small_mesh_graph", run_small_graph), ("renumbering", "renumbering", run_renumbering)]
    for name, key, fn in runs:
        if name in extras:
            line[key] = fn(args)
            progress(f"{name} done")
    if "adjoint" in line:
        line["adjoint_over_forward_fp64"] = line["adjoint"]["fp64"]["adjoint_over_forward"]
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.p, args.cpu_n, args.cpu_steps)
        progress("cpu baseline done")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
