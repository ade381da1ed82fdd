"""Benchmark of the pressure-correction step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 512] [--no-cpu]

Workload: the 512^3 wall-bounded channel with 512 bubbles (density ratio
1000, tanh-stretched z, x/y periodic), seeded synthetic inputs resident in
HBM.  A step is one whole pressure-correction step: RHS assembly, forward
transforms, tridiagonal z solves, inverse transforms, velocity correction and
divergence check.  `value` is the plain FP64 form's throughput in Mpts/s
(grid points per second / 1e6); the same line carries the FP32 +
FP64-refinement form on the same inputs, the batched form, the dominant
kernel's roofline, and the CPU oracle timed on the host.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def spectral_bytes(gs, csz):
    return (gs.nx // 2 + 1) * gs.ny * gs.nz * csz


# Algorithmic HBM bytes per cell of each pass, from the step's byte model:
# every separable pass reads its compulsory inputs once and writes its
# compulsory outputs once.  The model fuses the RHS into the forward x
# transform (P1: 40 read + the spectral write) and the correction into the
# inverse x transform (P5: spectral read + 40 read + 32 write), so where a
# pass is split in two here, each kernel is charged its own share and the
# round trip between them (f written and read back, p read back by the
# correction) is reported as overhead, not as algorithmic bytes.
def kernel_bytes(name, gs, csz):
    """(algorithmic bytes, overhead bytes) of one launch of a pass."""
    n = gs.cells
    sp = spectral_bytes(gs, csz)
    table = {
        "rhs_stencil": (5 * 8 * n, 8 * n),           # rho, p*, u*, v*, w* in; f stored (overhead)
        "rhs_fftx": (5 * 8 * n + sp, 0),             # fused: rho, p*, u*, v*, w* -> spectral
        "resid_stencil": (2 * 8 * n, 8 * n),         # f, p in; r stored (overhead)
        "resid_fftx": (2 * 8 * n + sp, 0),           # fused: f, p -> spectral
        "x_fft_fwd": (sp, 8 * n),                    # spectral out; f read back (overhead)
        "x_fft_fwd_resid": (sp, 8 * n),              # spectral out; r read back (overhead)
        "y_fft_fwd": (2 * sp, 0), "z_solve": (2 * sp, 0), "y_fft_inv": (2 * sp, 0),
        "x_fft_inv_store_p": (sp + 8 * n, 0),        # spectral in, p out
        "x_fft_inv_accum_p": (sp + 16 * n, 0),       # spectral in, p in and out
        "p_mean": (0, 0), "x_max": (0, 0),
        "correct_div": (5 * 8 * n + 3 * 8 * n, 8 * n),  # u*, v*, w*, rho, p* in, u, v, w out; p read back
        "div_check": (0, 3 * 8 * n),
    }
    return table.get(name, (0, 0))


def time_plan(plan, case_dev, dt, rho0, steps, warmup, outs, pass_steps=None):
    """ms per step over the timed loop, with the library's HIP events around
    the velocity correction only (two per step, recorded on the step's
    stream), then the per-pass table from a second loop that records events
    between all passes (about 2 us more per pass, outside the timed loop).
    Returns (ms, wall s, correction events of the timed loop, all-pass events,
    steps of the all-pass loop)."""
    import torch
    rho, ps, u, v, w = case_dev
    uo, vo, wo, po = outs
    for _ in range(warmup):
        plan.step(dt, rho0, rho, ps, u, v, w, uo, vo, wo, po, report=False)
    torch.cuda.synchronize()
    plan.set_timing(True, correction_only=True)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(st)
    for _ in range(steps):
        plan.step(dt, rho0, rho, ps, u, v, w, uo, vo, wo, po, report=False)
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / steps
    timed = plan.pass_times()
    nps = pass_steps or min(steps, 10)
    plan.set_timing(True)
    for _ in range(nps):
        plan.step(dt, rho0, rho, ps, u, v, w, uo, vo, wo, po, report=False)
    passes = plan.pass_times()
    plan.set_timing(False)
    return ms, wall, timed, passes, nps


def summarize_passes(passes, steps):
    agg = {}
    for name, t in passes:
        a = agg.setdefault(name, [0.0, 0])
        a[0] += t
        a[1] += 1
    return {k: {"ms_avg": v[0] / v[1], "launches_per_step": v[1] / steps} for k, v in agg.items()}


def src_hash():
    """Hash of the step's HIP sources (csrc/pcx_*), as in the profile summaries."""
    from paper_2502_04189_amd.profsum import src_hash as h
    return h("pcx_")


# pass name -> kernel-name prefix in the rocprofv3 summaries
KERNEL_OF_PASS = {"correct_div": "void pcx::k_corr<", "rhs_stencil": "void pcx::k_rhs<", "x_fft_fwd": "void pcx::k_xfwd<double, 0",
                  "y_fft_fwd": "void pcx::k_y<double, false", "y_fft_inv": "void pcx::k_y<double, true",
                  "z_solve": "void pcx::k_z<double", "x_fft_inv_store_p": "void pcx::k_xinv<double, 0"}


def _profile(profile="fp64_512cube_step"):
    fn = os.path.join(ROOT, "profiles", profile + "_traffic.json")
    if not os.path.exists(fn):
        return None
    d = json.load(open(fn))
    return d if d.get("src_hash") == src_hash() else None


def _profile_kernel(pass_name, prof):
    pre = KERNEL_OF_PASS.get(pass_name)
    if not prof or not pre:
        return None
    for k, v in prof["kernels"].items():
        if k.startswith(pre):
            return v
    return None


def roofline(pass_summary, gs, csz, timed_summary=None):
    """Roofline of the dominant kernel (largest time per step in the per-pass
    table): algorithmic bytes per launch over its average launch duration,
    timed with HIP events the library records on the step's stream around
    that kernel inside the timed loop (timed_summary; else the per-pass
    table).  The committed rocprofv3 summary of the same kernel gives its
    kernel-trace average and the HBM bytes the counters saw (null once the
    sources have changed)."""
    best = max(pass_summary.items(), key=lambda kv: kv[1]["ms_avg"] * kv[1]["launches_per_step"])
    name, s = best
    if timed_summary and name in timed_summary:
        s = timed_summary[name]
    alg, ovh = kernel_bytes(name, gs, csz)
    gbs = alg / (s["ms_avg"] * 1e-3) / 1e9
    pk = _profile_kernel(name, _profile()) if csz == 16 else None
    out = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbs / HBM_PEAK_GBS, 4),
           "traffic": int(pk["fetch_bytes"] + pk["write_bytes"]) if pk else None,
           "kernel": name, "bytes_per_launch": alg, "overhead_bytes_per_launch": ovh,
           "bytes_per_cell": alg / gs.cells, "cells_per_launch": gs.cells,
           "ms_per_launch": round(s["ms_avg"], 4)}
    if pk:
        out["ms_per_launch_rocprof"] = round(pk["ms"], 4)
        out["frac_rocprof"] = round(alg / (pk["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    return name, out


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(case):
    """The oracle as it stands (single-threaded C, FP64) on one whole step of
    the benchmarked case's own inputs, pinned to one host core."""
    import oracle
    g = oracle.Grid.from_workload(case.grid)
    fields = case.fields()
    old = os.sched_getaffinity(0)
    core = min(old)
    os.sched_setaffinity(0, {core})
    try:
        t0 = time.perf_counter()
        oracle.step(g, case.dt, case.rho0, *fields)
        t = time.perf_counter() - t0
    finally:
        os.sched_setaffinity(0, old)
    return {"value": round(case.grid.cells / t / 1e6, 3), "unit": "Mpts/s", "cores": 1, "kind": "oracle",
            "sample": f"one whole oracle step (FP64, single thread pinned to core {core}) on the benchmarked "
                      f"inputs ({case.name}, {case.grid.cells} cells) in {t:.1f} s",
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(), "seconds": round(t, 2)}


def reference_bandwidth():
    """Achievable-bandwidth reference points measured in the same run: a
    1 GiB device-to-device copy and a 1 GiB streaming elementwise kernel
    (read + write), each timed with events over 10 repetitions."""
    import torch
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    out = {}
    for name, fn in (("copy_1GiB", lambda: dst.copy_(src)), ("scale_1GiB", lambda: torch.mul(src, 2.0, out=dst))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 10
        out[name] = {"ms": round(ms, 4), "GB/s": round(2 * src.numel() * 8 / (ms * 1e-3) / 1e9, 1)}
    del src, dst
    torch.cuda.empty_cache()
    return out


def run_batch(steps, warmup, ndom):
    """192 domains of uneven size (refined form) in one persistent graph
    launch, against the same domains run one after another with plain FP64
    plans on the same GPU."""
    import torch
    from paper_2502_04189_amd import pcx
    from paper_2502_04189_amd import workloads as W
    t0 = time.perf_counter()
    cases = W.config4(ndom=ndom)
    log(f"generated {len(cases)} batch domains in {time.perf_counter() - t0:.1f} s")
    cells = sum(c.grid.cells for c in cases)
    doms = []
    for c in cases:
        f = [torch.from_numpy(a).to("cuda") for a in c.fields()]
        o = [torch.empty(c.grid.shape, dtype=torch.float64, device="cuda") for _ in range(4)]
        doms.append({"grid": c.grid, "dt": c.dt, "rho0": c.rho0, "rho": f[0], "pstar": f[1], "u": f[2],
                     "v": f[3], "w": f[4], "u_out": o[0], "v_out": o[1], "w_out": o[2], "p_out": o[3]})
    # the tuned shapes of the batch's size classes, kept between runs on one machine
    cache = pcx.batch_tune_cache_path()
    t0 = time.perf_counter()
    b = pcx.Batch(doms, "fp32_refined", autotune=True, tune_cache=cache)
    t_create = time.perf_counter() - t0
    for _ in range(warmup):
        b.launch()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(steps):
        b.launch()
    e1.record(st)
    torch.cuda.synchronize()
    bms = e0.elapsed_time(e1) / steps
    reps, status = b.reports()
    worst = max(r["rel_residual"] for r in reps)
    nconv = sum(r["converged"] for r in reps)
    # sequential plain FP64 plans
    plans = [pcx.Plan(d["grid"], "fp64") for d in doms]
    def seq():
        for p, d in zip(plans, doms):
            p.step(d["dt"], d["rho0"], d["rho"], d["pstar"], d["u"], d["v"], d["w"], d["u_out"], d["v_out"],
                   d["w_out"], d["p_out"], report=False)
    for _ in range(warmup):
        seq()
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(steps):
        seq()
    e1.record(st)
    torch.cuda.synchronize()
    sms = e0.elapsed_time(e1) / steps
    # the same domains batched in FP64 (one solve each): the batching gain at
    # equal arithmetic
    def timed(batch):
        for _ in range(warmup):
            batch.launch()
        torch.cuda.synchronize()
        e0.record(st)
        for _ in range(steps):
            batch.launch()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    b64 = pcx.Batch(doms, "fp64", autotune=True, tune_cache=cache)
    b64ms = timed(b64)
    _, st64 = b64.reports()
    b64.close()
    # both forms on the default (untuned) shapes: what the tuning buys
    bdef = pcx.Batch(doms, "fp32_refined")
    bdefms = timed(bdef)
    bdef.close()
    bdef = pcx.Batch(doms, "fp64")
    bdef64ms = timed(bdef)
    bdef.close()
    solves = reps[0]["solves"]
    log(f"batch: {bms:.3f} ms per launch ({cells} cells), default shapes {bdefms:.3f} ms, fp64 batch {b64ms:.3f} ms "
        f"(default shapes {bdef64ms:.3f} ms), "
        f"sequential fp64 {sms:.3f} ms, create {t_create:.1f} s")
    return {"domains": len(doms), "cells": cells, "ms_per_launch": round(bms, 4),
            "value": round(cells / (bms * 1e-3) / 1e6, 1), "unit": "Mpts/s",
            "solves_per_domain": reps[0]["solves"], "worst_rel_residual": worst,
            "domains_converged": nconv, "status": status,
            "sequential_fp64_ms": round(sms, 4), "speedup_vs_sequential_fp64": round(sms / bms, 3),
            "fp64_batch_ms": round(b64ms, 4), "fp64_batch_status": st64,
            "fp64_batch_speedup_vs_sequential_fp64": round(sms / b64ms, 3),
            "refined_default_shapes_ms": round(bdefms, 4),
            "fp64_default_shapes_ms": round(bdef64ms, 4),
            # HBM fraction of the per-domain byte model: 176 B/cell for one
            # FP64 solve, 176 + 64 (s - 1) for s FP32 solves
            "fp64_batch_hbm_frac_model": round(cells * 176.0 / (b64ms * 1e-3) / 8e12, 4),
            "refined_batch_hbm_frac_model": round(cells * (176.0 + 64.0 * (solves - 1)) / (bms * 1e-3) / 8e12, 4),
            "create_s_incl_autotune": round(t_create, 2)}


def prof_batch(steps, warmup, ndom):
    """The batch alone, for a kernel trace: FP64 then refined launches."""
    import torch
    from paper_2502_04189_amd import pcx
    from paper_2502_04189_amd import workloads as W
    cases = W.config4(ndom=ndom)
    doms = []
    for c in cases:
        f = [torch.from_numpy(a).to("cuda") for a in c.fields()]
        o = [torch.empty(c.grid.shape, dtype=torch.float64, device="cuda") for _ in range(4)]
        doms.append({"grid": c.grid, "dt": c.dt, "rho0": c.rho0, "rho": f[0], "pstar": f[1], "u": f[2],
                     "v": f[3], "w": f[4], "u_out": o[0], "v_out": o[1], "w_out": o[2], "p_out": o[3]})
    cache = pcx.batch_tune_cache_path()
    for prec in ("fp64", "fp32_refined"):
        b = pcx.Batch(doms, prec, autotune=True, tune_cache=cache)
        for _ in range(warmup + steps):
            b.launch()
        torch.cuda.synchronize()
        b.close()
        log(f"prof batch {prec}: {warmup + steps} launches of {len(doms)} domains")


# Algorithmic HBM bytes per cell of the substep kernels around the
# projection: every field a kernel reads or writes, once (neighbours re-read
# through the caches are overhead).
FLOW_BYTES = {"psi": 8 + 8,               # phi -> psi
              "flux": 16 + 32,            # phi, psi -> a (3 faces), kappa (normals evaluated in the kernel)
              # phi, u, v, w, kappa, a (3), h (3), h_phi, p1, p2 -> u* (3), h (3), p*, phi', rho', h_phi
              "momentum_phase": 112 + 80}


def flow_setup(case):
    """The two-phase state of a bubble channel: phi from its density
    (phase 1 = gas, rho = 1000 - 999 phi), the velocity its pressure step
    corrects (discretely solenoidal), zero pressures; gas/liquid
    viscosities 1e-5 / 1e-3, sigma = 0.07, gravity -9.81 in z,
    Gamma = 2 max |u|, eps = 0.51 dx."""
    import torch
    from paper_2502_04189_amd import pcx
    gs = case.grid
    dev = [torch.from_numpy(a).to("cuda") for a in case.fields()]
    plan = pcx.Plan(gs, "fp64")
    u, v, w, _, _ = plan.step(case.dt, case.rho0, *dev, report=False)
    torch.cuda.synchronize()
    plan.close()
    phi = (1000.0 - dev[0]) / 999.0
    del dev
    st = [phi.contiguous(), u, v, w]
    umax = float(max(u.abs().max(), v.abs().max(), w.abs().max()))
    prm = dict(rho1=1.0, rho2=1000.0, mu1=1e-5, mu2=1e-3, sigma=0.07, g=(0.0, 0.0, -9.81), gamma=2.0 * umax,
               eps=0.51 * gs.lx / gs.nx)
    return st, prm, umax


def run_poisson(gs, steps, warmup):
    """pcx_poisson_solve (FP64) on a random right-hand side: the benchmark's
    own boundaries (x, y periodic, walls in z) and Dirichlet x and y (sine
    transforms); spectral bytes per cell of the five passes: x 8 + sp,
    y 2 sp, z 2 sp, y 2 sp, x sp + 8 (sp = 16 B of a complex mode per cell
    pair, about 8 B per cell)."""
    import torch
    from paper_2502_04189_amd import pcx
    from paper_2502_04189_amd import workloads as W
    out = {}
    f = torch.randn(gs.shape, dtype=torch.float64, device="cuda")
    p = torch.empty_like(f)
    for name, bc in (("periodic_x_y_wall_z", (gs.bcx, gs.bcy, gs.bcz)), ("dirichlet_x_y_wall_z", (2, 2, gs.bcz))):
        g2 = W.GridSpec(gs.nx, gs.ny, gs.nz, gs.lx, gs.ly, gs.zf, *bc)
        plan = pcx.Plan(g2, "fp64")
        for _ in range(warmup):
            plan.poisson_solve(f, p)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            plan.poisson_solve(f, p)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        sp = spectral_bytes(g2, 16) if bc[0] == 0 else gs.nx * gs.ny * gs.nz * 16
        alg = 8 * gs.cells + sp + 6 * sp + sp + 8 * gs.cells
        out[name] = {"ms": round(ms, 4), "alg_bytes": alg, "hbm_frac": round(alg / (ms * 1e-3) / 8e12, 4)}
        plan.close()
        log(f"poisson solve {name}: {ms:.3f} ms")
    return out


def run_varcoef(case, dev, split_ms, tol=1e-10, maxit=4000):
    """The variable-coefficient projection D((1/rho_f) G p) = D u*/dt that the
    splitting replaces, by conjugate gradients preconditioned with the FP64
    constant-coefficient solve, on the benchmark's own inputs: its time and
    iterations against the split step's, and the split step's velocity
    error relative to it with the workload's p* and with p* = its pressure
    (where the splitting is exact).  One timed run (it takes seconds)."""
    import torch
    from paper_2502_04189_amd import pcx
    gs = case.grid
    rho, ps, u, v, w = dev
    vc = pcx.VarCoef(gs)
    outs = [torch.empty(gs.shape, dtype=torch.float64, device="cuda") for _ in range(4)]
    vc.project(case.dt, case.rho0, rho, u, v, w, tol=tol, maxit=2, outs=outs)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    uo, vo, wo, p, it, rr, st = vc.project(case.dt, case.rho0, rho, u, v, w, tol=tol, maxit=maxit, outs=outs)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    vc.close()
    plan = pcx.Plan(gs, "fp64")
    so = [torch.empty_like(uo) for _ in range(4)]
    err = {}
    for name, pst in (("workload_pstar", ps), ("exact_pstar", p)):
        plan.step(case.dt, case.rho0, rho, pst, u, v, w, *so, report=False)
        torch.cuda.synchronize()
        err[name] = max(float((a - b).abs().max() / b.abs().max()) for a, b in zip(so[:3], (uo, vo, wo)))
    plan.close()
    del so, outs
    log(f"varcoef projection: {it} iterations, residual {rr:.2e}, {ms:.1f} ms; split errors {err}")
    return {"tol": tol, "iterations": it, "rel_residual": rr, "converged": st == pcx.PCX_OK,
            "ms": round(ms, 2), "ms_per_iteration": round(ms / max(it, 1), 3),
            "split_step_ms": round(split_ms, 4), "cost_vs_split_step": round(ms / split_ms, 1),
            "split_velocity_rel_error": err}


def flow_dt(gs, prm, umax):
    """Step of the explicit substeps: the advective limit 0.5 h_min / max|u|
    and the diffusive one of the ACDI term (diffusivity Gamma eps) and the
    viscous term (max mu/rho): RK3 is stable on the negative real axis up to
    about 2.5, the discrete Laplacian's largest eigenvalue is
    sum_d 4/h_d^2, and half of that limit is taken."""
    import numpy as np
    hz = float(np.min(np.diff(gs.zf)))
    hx, hy = gs.lx / gs.nx, gs.ly / gs.ny
    nu = max(prm["mu1"] / prm["rho1"], prm["mu2"] / prm["rho2"])
    lam = 4.0 / hx ** 2 + 4.0 / hy ** 2 + 4.0 / hz ** 2
    return min(0.5 * min(hx, hy, hz) / umax, 1.25 / ((prm["gamma"] * prm["eps"] + nu) * lam))


def run_flow(case, steps, warmup, split_check=True):
    """Whole Runge-Kutta steps (three substeps: phase field, momentum
    predictor, pressure-correction step) of the bubble channel."""
    import torch
    from paper_2502_04189_amd import pcx
    gs = case.grid
    st, prm, umax = flow_setup(case)
    F = pcx.Flow(gs, **prm)
    z = lambda: torch.zeros(gs.shape, dtype=torch.float64, device="cuda")
    h = [z() for _ in range(4)]
    Dt = flow_dt(gs, prm, umax)
    dtprev, cur = None, 0

    # ping-pong without allocation: state A -> B -> A ...
    bufs = [st + [z()], [z() for _ in range(5)]]
    pres = [z(), z(), z()]

    def step_all(n):
        nonlocal dtprev, cur
        for _ in range(n):
            for s in (1, 2, 3):
                al = (8 / 15, 2 / 15, 1 / 3)[s - 1]
                r = 0.0 if dtprev is None else al * Dt / dtprev
                src, dst = bufs[cur], bufs[1 - cur]
                # pressures: pres[0] newest, pres[1] previous; output into pres[2]
                F.substep(s, Dt, *src[:4], pres[0], pres[1], r, h, dst[:4] + [pres[2]], report=False)
                pres[:] = [pres[2], pres[0], pres[1]]
                cur = 1 - cur
                dtprev = al * Dt
        return bufs[cur]

    step_all(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    fin = step_all(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    phi = fin[0]
    ok = bool(torch.isfinite(fin[1]).all()) and float(phi.min()) > -1e-6 and float(phi.max()) < 1 + 1e-6
    log(f"rk3 steps: {ms:.3f} ms per step of three substeps, phi in [{float(phi.min()):.3e}, {float(phi.max()):.6f}]")
    split = None
    if split_check:
        # the splitting error on a settled state: the run starts from zero
        # pressures, and an extrapolated p* is only as good as the pressures
        # of the last substeps
        fin = step_all(30)
        split = splitting_error(F, gs, Dt, fin, pres, dtprev)
        split["after_rk3_steps"] = warmup + steps + 30
    F.close()
    cells = gs.cells
    out = {"ms_per_rk3_step": round(ms, 4), "ms_per_substep": round(ms / 3, 4),
           "value": round(cells / (ms * 1e-3) / 1e6, 1), "unit": "Mpts/s (whole RK3 steps)",
           "steps": steps, "Dt": Dt, "finite_and_bounded": ok,
           "substep_kernel_bytes_per_cell": FLOW_BYTES}
    if split is not None:
        out["splitting_error_vs_varcoef"] = split
    return out


def splitting_error(F, gs, Dt, state, pres, dtprev, tol=1e-11):
    """The splitting error on the flow's own state: the next substep's
    predictor (pcx_flow_predict: u*, the new density, p* extrapolated from
    the last two pressures) corrected by the split step and by the
    variable-coefficient projection (tol 1e-11), and by the split step with
    p* = 0 (no extrapolation) for comparison; max-norm differences relative
    to the projection's velocity and pressure."""
    import torch
    from paper_2502_04189_amd import pcx
    r = (8 / 15) * Dt / dtprev
    h = [torch.zeros_like(state[0]) for _ in range(4)]
    phi_o = torch.empty_like(state[0])
    us, vs, ws, rho, ps, rho0, dt = F.predict(1, Dt, *state[:4], pres[0], pres[1], r, h, phi_o)
    vc = pcx.VarCoef(gs)
    uv, vv, wv, pv, it, rr, st = vc.project(dt, rho0, rho, us, vs, ws, tol=tol, maxit=4000)
    vc.close()
    plan = pcx.Plan(gs, "fp64")
    out = {"varcoef_iterations": it, "varcoef_rel_residual": rr, "tol": tol}
    for name, pst in (("pstar_extrapolated", ps), ("pstar_zero", torch.zeros_like(ps))):
        su, sv, sw, sp, _ = plan.step(dt, rho0, rho, pst, us, vs, ws, report=False)
        torch.cuda.synchronize()
        eu = max(float((a - b).abs().max() / b.abs().max()) for a, b in zip((su, sv, sw), (uv, vv, wv)))
        ep = float((sp - pv).abs().max() / pv.abs().max())
        out[name] = {"u_rel": eu, "p_rel": ep}
        del su, sv, sw, sp
    plan.close()
    log(f"splitting error on the flow state: {out}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512, help="grid size n^3 of the channel workload")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-refined", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--ndom", type=int, default=192)
    ap.add_argument("--prof", action="store_true",
                    help="profiling mode: a few FP64 (or --prof-refined) steps plus a 1 GiB torch copy "
                         "that calibrates the HBM byte counters; prints no JSON")
    ap.add_argument("--prof-refined", action="store_true")
    ap.add_argument("--no-flow", action="store_true")
    ap.add_argument("--no-varcoef", action="store_true")
    ap.add_argument("--prof-varcoef", action="store_true",
                    help="profiling mode: one variable-coefficient projection of the workload; no JSON")
    ap.add_argument("--prof-flow", action="store_true",
                    help="profiling mode: a few Runge-Kutta steps of the substep around the projection; no JSON")
    ap.add_argument("--prof-batch", action="store_true",
                    help="profiling mode: only the 192-domain batch, FP64 then refined (tuned shapes); "
                         "prints no JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU decomposition is "
              f"a design, not a build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2502_04189_amd import pcx
    from paper_2502_04189_amd import workloads as W
    pcx.lib()

    if args.prof_batch:
        prof_batch(args.steps, args.warmup, args.ndom)
        log("prof mode done")
        return

    t0 = time.perf_counter()
    nb = 512 if args.n == 512 else max(1, (args.n // 64) ** 3)
    case = W.config3() if args.n == 512 else W.channel_bubbles(args.n, nb, 1003, f"channel_{args.n}^3")
    log(f"generated {case.name} in {time.perf_counter() - t0:.1f} s")
    gs = case.grid
    dev = [torch.from_numpy(a).to("cuda") for a in case.fields()]
    rho0 = pcx.rho_min(dev[0])
    assert rho0 == case.rho0
    outs = [torch.empty(gs.shape, dtype=torch.float64, device="cuda") for _ in range(4)]
    cells = gs.cells

    if args.prof_varcoef:
        plan = pcx.Plan(gs, "fp64")
        ms = time_plan(plan, dev, case.dt, rho0, 2, 1, outs)[0]
        plan.close()
        run_varcoef(case, dev, ms)
        log("prof mode done")
        return

    if args.prof_flow:
        del dev, outs
        torch.cuda.empty_cache()
        run_flow(case, args.steps, args.warmup, split_check=False)
        log("prof mode done")
        return

    if args.prof:
        plan = pcx.Plan(gs, "fp32_refined" if args.prof_refined else "fp64", fixed_iters=3)
        for _ in range(args.warmup + args.steps):
            plan.step(case.dt, rho0, *dev, *outs, report=False)
        torch.cuda.synchronize()
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("prof mode done: steps", args.warmup + args.steps, "copy bytes", 2 * src.numel() * 8)
        return

    # ---- FP64
    plan = pcx.Plan(gs, "fp64")
    ms, wall, timed, passes, nps = time_plan(plan, dev, case.dt, rho0, args.steps, args.warmup, outs)
    summ = summarize_passes(passes, nps)
    kname, roof = roofline(summ, gs, 16, summarize_passes(timed, args.steps))
    _, _, _, _, rep = plan.step(case.dt, rho0, *dev, *outs, report=True)
    p64 = outs[3].clone()
    log(f"fp64: {ms:.3f} ms/step, passes {json.dumps(summ)}")
    log(f"fp64 report {rep}")
    bytes_model = 176 * cells
    res = {
        "metric": "Mpts/s and Poisson steps/s at 512^3: FP64 vs FP32+refine at 1e-10, HBM %",
        "value": round(cells / (ms * 1e-3) / 1e6, 1),
        "unit": "Mpts/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"wall-channel {args.n}^3, {nb} bubbles, density ratio 1000, tanh z (a=1.8), "
                               f"x/y periodic; plain FP64 pressure-correction step",
                   "nx": gs.nx, "ny": gs.ny, "nz": gs.nz},
        "steps_per_s": round(1000.0 / ms, 2),
        "hbm_frac_step_model": round(bytes_model / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "fp64_rel_residual": rep["rel_residual"],
        "passes_fp64": summ,
        "roofline": roof,
    }
    del plan

    # ---- the variable-coefficient projection the splitting replaces
    if not args.no_varcoef:
        res["varcoef_projection"] = run_varcoef(case, dev, ms)
        torch.cuda.empty_cache()

    # ---- FP32 + FP64 refinement on the same inputs
    if not args.no_refined:
        rplan = pcx.Plan(gs, "fp32_refined")
        _, _, _, _, rrep = rplan.step(case.dt, rho0, *dev, *outs, report=True, raise_on_status=False)
        solves = rrep["solves"]
        rplan.close()
        rplan = pcx.Plan(gs, "fp32_refined", fixed_iters=solves)
        rms, _, _, rpasses, rnps = time_plan(rplan, dev, case.dt, rho0, args.steps, args.warmup, outs)
        _, _, _, _, rrep = rplan.step(case.dt, rho0, *dev, *outs, report=True, raise_on_status=False)
        dp = float((outs[3] - p64).abs().max() / p64.abs().max())
        log(f"refined: {rms:.3f} ms/step solves {solves} report {rrep} |p - p64|/|p64| {dp:.3e}")
        res["refined"] = {"ms_per_step": round(rms, 4), "value": round(cells / (rms * 1e-3) / 1e6, 1),
                          "unit": "Mpts/s", "solves": rrep["solves"], "rel_residual": rrep["rel_residual"],
                          "converged": bool(rrep["converged"]), "p_rel_diff_vs_fp64_gpu": dp,
                          "speedup_vs_fp64": round(ms / rms, 3),
                          "passes": summarize_passes(rpasses, rnps)}
        del rplan

    del dev, outs, p64
    torch.cuda.empty_cache()

    # ---- batched form
    if not args.no_batch:
        res["batched"] = run_batch(args.steps, args.warmup, args.ndom)

    # ---- the plan's Poisson solve alone at 512^3, with the benchmark's
    # boundaries and with Dirichlet (sine-transform) x and y
    res["poisson_solve"] = run_poisson(gs, args.steps, args.warmup)
    torch.cuda.empty_cache()

    # ---- whole Runge-Kutta steps around the projection (same workload)
    if not args.no_flow:
        res["rk3_substeps"] = run_flow(case, min(args.steps, 5), min(args.warmup, 1))
        torch.cuda.empty_cache()

    res["reference_bandwidth"] = reference_bandwidth()
    if not args.no_cpu:
        cb = cpu_baseline(case)
        res["cpu_baseline"] = cb
        res["speedup_vs_cpu_oracle"] = round(res["value"] / cb["value"], 1)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
