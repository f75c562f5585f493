#!/usr/bin/env python3
"""Benchmark: cell-stage updates/s of the entropy-stable moving-mesh step on
the 3D two-species 256^3 shock-bubble workload (water/air, stiffened gas).

One step = mesh redistribution (monitor, 3 filter passes, 5 Jacobi sweeps,
limiter) + GCL metrics + CFL step + three fused SSP-RK3 stages (ES flux:
2w = 6 EC flux + MR-WENO dissipation) + ghost layers + the FP64 total
entropy.  value = 256^3 * 3 / (seconds per step).

Prints one JSON line.  --gpus N > 1 is refused: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E, GB/s
PEAK_FP64_TFLOPS = 78.6        # MI355X FP64 vector (FMA = 2 flops)
PEAK_FP32_TFLOPS = 157.3       # MI355X FP32 vector (packed)

# Algorithmic work of one cell-stage of the fused RK stage, 3D, N = 2 (the
# counts are derived in the design notes): flops with add/mul/div/sqrt/log = 1
# and FMA = 2; bytes = JU (6) + J + 9 spatial + 3 time metrics + JU_n (6) + J_n
# read, JU_out (6) + J_out written, FP64.
FLOPS_PER_CELL_STAGE = {(3, 2): 7337, (3, 1): 5804, (2, 2): 4040, (2, 1): 3029}
BYTES_PER_CELL_STAGE = {(3, 2): 33 * 8, (3, 1): 29 * 8, (2, 2): 23 * 8, (2, 1): 19 * 8}


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in ("es_rhs.hip", "es_flux.hpp", "es_device.hpp"):
        with open(os.path.join(ROOT, "paper_2202_07989_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_counters():
    """What rocprofv3 counters measured on the fused stage, if taken on the
    current kernel source: HBM bytes per stage (FETCH_SIZE + WRITE_SIZE,
    calibrated on a copy kernel) and executed FP64 flops per cell-stage."""
    p = os.path.join(ROOT, "profiles", "rk_stage_c3_256_traffic.json")
    if not os.path.exists(p):
        return {}
    with open(p) as fh:
        t = json.load(fh)
    if t.get("kernel_hash") != kernel_hash():
        return {}
    return t


def host_cpu():
    """Host CPU model and the cores this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, avail


def oracle_stage_rate(m, seconds, max_reps):
    """Cell-stage rate of the oracle's fused RK stage on an m^3 box of the
    shock-bubble data (threads as OMP_NUM_THREADS says); returns (rate,
    reps, elapsed)."""
    import oracle
    from paper_2202_07989_amd import inputs as I
    sps = I.spec_c3(m)
    o = oracle.Oracle(sps)
    JUs, Js, xs = I.init_shock_bubble(sps)
    o.fill_ghosts(JUs, o.nc)
    o.fill_ghosts(Js, 1)
    o.fill_ghosts_x(xs)
    jx, jt = o.metrics(xs)
    _, lam, dt = o.max_wavespeed(JUs, Js, jx, 0.3)
    t0 = time.perf_counter()
    reps = 0
    while True:
        o.rk_stage(1, dt, JUs, Js, JUs, Js, jx, jt)
        reps += 1
        el = time.perf_counter() - t0
        if el > seconds or reps >= max_reps:
            break
    return m ** 3 * reps / el, reps, el


def cpu_baseline(sp, JU, J, x, n):
    """The CPU oracle (never tuned) on a bounded sample of the same workload:
    fused RK stages on a 64^3 box of the same shock-bubble data, with all the
    host cores given to this process (OpenMP), then with one thread (a
    child process with OMP_NUM_THREADS=1)."""
    import subprocess
    m = 64 if n >= 64 else n
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rate, reps, el = oracle_stage_rate(m, 10.0, 20)
    model, avail = host_cpu()
    one = None
    try:
        env = dict(os.environ, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--mode", "oracle-rate", "--n", str(m)],
                           env=env, capture_output=True, text=True, timeout=120)
        one = json.loads(r.stdout.strip().splitlines()[-1]) if r.returncode == 0 else None
    except (subprocess.TimeoutExpired, ValueError, IndexError):
        one = None
    out = {"value": rate, "unit": "cell-stage updates/s", "cores": threads, "kind": "oracle",
           "host_cpu": model, "host_cores_available": avail,
           "sample": f"{reps} fused RK stage(s) of the oracle on a {m}^3 box of the same "
                     f"3D two-species shock-bubble data ({el:.1f} s, {threads} threads)"}
    if one:
        out["value_1_thread"] = one["value"]
        out["sample_1_thread"] = one["sample"]
    return out


def stage_inputs(ctx, mon, cfl, gU, gJ, gx, dt_dev):
    """Moving-mesh metrics, dt and stage buffers of the current state."""
    import torch
    d = 3
    jx = torch.empty((d * d,) + tuple(gJ.shape[1:]), dtype=torch.float64, device="cuda")
    jt = torch.empty((d,) + tuple(gJ.shape[1:]), dtype=torch.float64, device="cuda")
    disp = torch.empty_like(gx)
    ctx.mesh_redistribute(mon, gU, gJ, gx, disp)
    ctx.es_metrics(gx, None, 0.0, None, jx, None)
    ctx.max_wavespeed(gU, gJ, jx, cfl, None, dt_dev)
    ctx.es_metrics(gx, disp, 0.5, dt_dev, jx, jt)
    JUo, Jo = torch.empty_like(gU), torch.empty_like(gJ)
    JUn, Jn = gU.clone(), gJ.clone()
    return jx, jt, JUo, Jo, JUn, Jn


def run_stage_only(ctx, mon, cfl, gU, gJ, gx, dt_dev, reps):
    import torch
    jx, jt, JUo, Jo, JUn, Jn = stage_inputs(ctx, mon, cfl, gU, gJ, gx, dt_dev)
    for _ in range(reps):
        ctx.es_rk_stage(1, dt_dev, JUn, Jn, gU, gJ, jx, jt, JUo, Jo)
    a = torch.ones(1 << 28, dtype=torch.float64, device="cuda")     # 2 GiB
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "stage", "reps": reps, "copy_bytes_each_way": a.numel() * 8}), flush=True)


def spec_for(args, I, n):
    """The 3D two-species workload; --reconstruction js swaps in the classical
    WENO5 of the comparison variant MM-WENOJS (epsilon 1e-6)."""
    sp = I.spec_c3(n)
    if getattr(args, "reconstruction", "mr") == "js":
        sp["reconstruction"], sp["weno_eps"] = 1, 1e-6
    return sp


def run_precision(args, prec_name, n, steps, warmup, stage_reps):
    """Time whole steps and the fused stage of one precision; returns a dict."""
    import numpy as np
    import torch

    from paper_2202_07989_amd import es
    from paper_2202_07989_amd import inputs as I

    sp = spec_for(args, I, n)
    prec = es.ES_MIXED if prec_name == "mixed" else es.ES_FP64
    JU, J, x = I.init_shock_bubble(sp)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    gU, gJ, gx = dev(JU), dev(J), dev(x)
    ctx = es.Context(sp, precision=prec)
    mon = I.monitor_spec(n_sweeps=5, n_smooth=3, sigma=(0,), alpha=(1200.0,))
    cfl = 0.3
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    tau_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    ent = torch.zeros(1, dtype=torch.float64, device="cuda")

    def step():
        ctx.es_step(gU, gJ, gx, mon=mon, cfl=cfl, move_mesh=True, dt_dev=dt_dev, dtau_dev=tau_dev)
        ctx.es_entropy(gU, gJ, ent)

    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_step = e0.elapsed_time(e1) / steps
    rc, flags = ctx.es_status()
    cells = n ** 3
    value = cells * 3 / (ms_step / 1e3)

    # dominant kernel, timed live: the fused RK stage (x-y launch + z sweep)
    # on the benchmark's own state and moving-mesh metrics
    jx, jt, JUo, Jo, JUn, Jn = stage_inputs(ctx, mon, cfl, gU, gJ, gx, dt_dev)
    ctx.es_rk_stage(1, dt_dev, JUn, Jn, gU, gJ, jx, jt, JUo, Jo)
    torch.cuda.synchronize()
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record(stream)
    for _ in range(stage_reps):
        ctx.es_rk_stage(1, dt_dev, JUn, Jn, gU, gJ, jx, jt, JUo, Jo)
    s1.record(stream)
    torch.cuda.synchronize()
    ms_stage = s0.elapsed_time(s1) / stage_reps
    # es_rhs alone (x-y launch + z sweep writing d(JU)/dt, dJ/dt; no stage
    # combination) on the same state and metrics
    ctx.es_rhs(gU, gJ, jx, jt, JUo, Jo)
    torch.cuda.synchronize()
    s0.record(stream)
    for _ in range(stage_reps):
        ctx.es_rhs(gU, gJ, jx, jt, JUo, Jo)
    s1.record(stream)
    torch.cuda.synchronize()
    ms_rhs = s0.elapsed_time(s1) / stage_reps
    key = (3, 2)
    achieved = FLOPS_PER_CELL_STAGE[key] * cells / (ms_stage / 1e3) / 1e12
    peak = PEAK_FP64_TFLOPS if prec == es.ES_FP64 else PEAK_FP32_TFLOPS
    hbm_gbs = BYTES_PER_CELL_STAGE[key] * cells / (ms_stage / 1e3) / 1e9
    del ctx
    torch.cuda.empty_cache()
    return dict(value=value, ms_step=ms_step, wall=wall, status=rc, ms_stage=ms_stage, ms_rhs=ms_rhs,
                achieved=achieved, peak=peak, hbm_gbs=hbm_gbs, sp=sp, JU=JU, J=J, x=x)


def config_rates(steps=20):
    """Whole-step rates of the 2D configurations, FP64 and mixed:
    64^2 one-species smooth advection on the fixed curvilinear mesh (CFL
    0.5), and the 512^2 two-species shock-bubble on the moving mesh (10
    Jacobi sweeps, 3 filter passes, alpha 1200, CFL 0.4)."""
    import numpy as np
    import torch

    from paper_2202_07989_amd import es
    from paper_2202_07989_amd import inputs as I

    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    stream = torch.cuda.current_stream()
    out = {}
    for name, sp, init, move, cfl in (
            ("2d_1species_64_fixed_curvilinear", I.spec_c1(64), I.init_c1, False, 0.5),
            ("2d_2species_512_moving_shock_bubble", I.spec_c2(512), I.init_shock_bubble, True, 0.4)):
        JU, J, x = init(sp)
        mon = I.monitor_spec(n_sweeps=10, n_smooth=3, sigma=(0,), alpha=(1200.0,)) if move else None
        row = {}
        for prec_name, prec in (("fp64", es.ES_FP64), ("mixed", es.ES_MIXED)):
            ctx = es.Context(sp, precision=prec)
            gU, gJ, gx = dev(JU), dev(J), dev(x)
            dt = torch.zeros(1, dtype=torch.float64, device="cuda")
            for _ in range(3):
                ctx.es_step(gU, gJ, gx, mon=mon, cfl=cfl, move_mesh=move, dt_dev=dt)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                ctx.es_step(gU, gJ, gx, mon=mon, cfl=cfl, move_mesh=move, dt_dev=dt)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            cells = sp["n"][0] * sp["n"][1]
            row[prec_name] = {"ms_per_step": ms, "cell_stage_updates_per_s": 3 * cells / (ms / 1e3),
                              "status": ctx.es_status()[0]}
            del ctx
        row["mixed_speedup"] = row["fp64"]["ms_per_step"] / row["mixed"]["ms_per_step"]
        out[name] = row
    return out


def full_length(args):
    """The 2D 512^2 moving-mesh shock-bubble for its 200 steps and the 3D
    256^3 one for its 50, FP64 and mixed, from the seeded initial data:
    status after every 10 steps (stops at the first non-physical state),
    smallest partial densities and J at the end, time."""
    import numpy as np
    import torch

    from paper_2202_07989_amd import es
    from paper_2202_07989_amd import inputs as I

    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    out = {"mode": "full-length"}
    for name, sp, steps, mon, cfl in (
            ("2d_512_200_steps", I.spec_c2(512), 200,
             I.monitor_spec(n_sweeps=10, n_smooth=3, sigma=(0,), alpha=(1200.0,)), 0.4),
            ("3d_256_50_steps", I.spec_c3(256), 50,
             I.monitor_spec(n_sweeps=5, n_smooth=3, sigma=(0,), alpha=(1200.0,)), 0.3)):
        JU, J, x = I.init_shock_bubble(sp)
        Iin = I.interior(sp)
        for prec_name, prec in (("fp64", es.ES_FP64), ("mixed", es.ES_MIXED)):
            ctx = es.Context(sp, precision=prec)
            gU, gJ, gx = dev(JU), dev(J), dev(x)
            dt = torch.zeros(1, dtype=torch.float64, device="cuda")
            t, done, rc = 0.0, 0, 0
            t0 = time.perf_counter()
            while done < steps:
                for _ in range(10):
                    ctx.es_step(gU, gJ, gx, mon=mon, cfl=cfl, move_mesh=True, dt_dev=dt)
                    t += float(dt.item())
                    done += 1
                rc, flags = ctx.es_status()
                print(json.dumps({"run": name, "precision": prec_name, "step": done, "status": rc}), flush=True)
                if rc != 0:
                    break
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            rho = (gU[Iin][:2] / gJ[Iin]).reshape(2, -1)
            out[f"{name}_{prec_name}"] = {"steps_done": done, "status": rc, "t_end": t, "wall_s": wall,
                                          "min_partial_density": [float(rho[0].min()), float(rho[1].min())],
                                          "min_J": float(gJ[Iin].min())}
            del ctx, gU, gJ, gx
            torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def accuracy_study(args):
    """FP64 and mixed GPU runs of the same workload side by side: per
    component of U = JU/J and for rho and p, l1 = mean|a-b|/mean|b| and
    linf = max|a-b|/max|b| over the interior after --steps steps (mixed vs
    FP64 GPU), and, when --oracle-ref names a file written by the oracle's
    reference script, both GPU runs against the FP64 oracle on its
    subsample of nodes."""
    import numpy as np
    import torch

    from paper_2202_07989_amd import es
    from paper_2202_07989_amd import inputs as I

    n = args.n
    sp = I.spec_c3(n)
    ng = sp["ng"]
    N = sp["nspec"]
    JU, J, x = I.init_shock_bubble(sp)
    mon = I.monitor_spec(n_sweeps=5, n_smooth=3, sigma=(0,), alpha=(1200.0,))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    inner = (slice(None),) + tuple(slice(ng, ng + n) for _ in range(3))
    cv = [float(c) for c in sp["cv"][:N]]
    Rg = [float(c) * (float(g) - 1.0) for c, g in zip(sp["cv"][:N], sp["gamma"][:N])]
    pinf_tot = float(sum(sp["pinf"][:N]))

    def prims(U):
        """rho and p of conserved states U (components first), stiffened EOS."""
        rho = sum(U[l] for l in range(N))
        kin = 0.5 * sum(U[N + j] ** 2 for j in range(3)) / rho
        cvr = sum(cv[l] * U[l] for l in range(N))
        T = (U[N + 3] - kin - pinf_tot) / cvr
        p = sum(Rg[l] * U[l] for l in range(N)) * T - pinf_tot
        return rho, p

    finals, dts = {}, {}
    for prec_name, prec in (("fp64", es.ES_FP64), ("mixed", es.ES_MIXED)):
        ctx = es.Context(sp, precision=prec)
        gU, gJ, gx = dev(JU), dev(J), dev(x)
        dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
        seq = []
        for s in range(args.steps):
            ctx.es_step(gU, gJ, gx, mon=mon, cfl=0.3, move_mesh=True, dt_dev=dt_dev)
            seq.append(dt_dev)
            dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        rc, _ = ctx.es_status()
        print(json.dumps({"accuracy_run": prec_name, "steps": args.steps, "status": rc}), flush=True)
        dts[prec_name] = torch.cat(seq).cpu().numpy()
        finals[prec_name] = (gU[inner].contiguous(), gJ[inner].contiguous())
        del ctx, gx
        torch.cuda.empty_cache()

    def fields(JUi, Ji):
        U = JUi / Ji
        rho, p = prims(U)
        return [U[c] for c in range(U.shape[0])] + [rho, p]

    names = [f"U{c}" for c in range(N + 4)] + ["rho", "p"]
    a = fields(*finals["mixed"])
    b = fields(*finals["fp64"])
    mixed_vs_fp64 = {nm: {"l1": float((x_ - y_).abs().mean() / y_.abs().mean()),
                          "linf": float((x_ - y_).abs().max() / y_.abs().max())}
                     for nm, x_, y_ in zip(names, a, b)}
    out = {"mode": "accuracy", "workload": f"3D two-species shock-bubble {n}^3, {args.steps} moving-mesh "
           "steps (5 Jacobi sweeps, 3 filter passes, alpha 1200), CFL 0.3",
           "mixed_vs_fp64_gpu": mixed_vs_fp64,
           "dt_rel_diff_max": float(np.abs(dts["mixed"] - dts["fp64"]).max() / np.abs(dts["fp64"]).max())}
    if args.oracle_ref:
        ref = np.load(args.oracle_ref)
        assert int(ref["n"]) == n and int(ref["step"]) == args.steps, "reference of another run"
        s0, ss = int(ref["sub0"]), int(ref["substep"])
        sub = (slice(None),) + tuple(slice(s0, None, ss) for _ in range(3))
        rf = fields(torch.from_numpy(ref["JU"]).cuda(), torch.from_numpy(ref["J"]).cuda())
        for prec_name in ("fp64", "mixed"):
            JUi, Ji = finals[prec_name]
            gf = fields(JUi[sub].contiguous(), Ji[sub].contiguous())
            out[f"{prec_name}_gpu_vs_oracle_sampled"] = {
                nm: {"l1": float((x_ - y_).abs().mean() / y_.abs().mean()),
                     "linf": float((x_ - y_).abs().max() / y_.abs().max())}
                for nm, x_, y_ in zip(names, gf, rf)}
        out["oracle_sample"] = (f"every {ss}th interior node per direction from node {s0} "
                                f"({rf[0].numel()} nodes)")
        out["dt_rel_diff_vs_oracle_max"] = float(np.abs(dts["fp64"] - ref["dts"]).max()
                                                 / np.abs(ref["dts"]).max())
    print(json.dumps(out), flush=True)


def adapt_initial_mesh(ctx, sp, mon, x, prims0, max_iter=200, tol=1e-3):
    """Initial adaptive mesh (the vortex examples start from an adapted mesh,
    Figure 5.1 at t = 0): repeat mesh_redistribute on the initial data
    evaluated at the current nodes (J = 1 while adapting) until no node moves
    by more than tol of the computational spacing, then set J to the discrete
    Jacobian of the final mesh and JU = J U.  x: device mesh with ghost
    layers; prims0(list of node coordinate arrays) -> (rho, v list, p).
    Returns (JU, J, iterations) on the device."""
    import numpy as np
    import torch

    from paper_2202_07989_amd import inputs as I

    d = sp["dim"]
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    Iin = I.interior(sp)
    h = min(sp["dxi"][:d])

    def state_at(gx, J=None):
        xi = gx.cpu().numpy()
        pts = [xi[Iin][k] for k in range(d)]
        rho, v, p = prims0(pts)
        U = I.conserved(sp, [rho], v, p)
        Jin = np.ones_like(rho) if J is None else J.cpu().numpy()[Iin][0]
        JU, Jp, _ = I.assemble(sp, U, Jin, pts)
        gU, gJ = dev(JU), dev(Jp)
        ctx.es_fill_ghosts(gU, sp["nspec"] + d + 1)
        ctx.es_fill_ghosts(gJ, 1)
        return gU, gJ

    disp = torch.zeros_like(x)
    tau = torch.zeros(1, dtype=torch.float64, device="cuda")
    it = 0
    for it in range(1, max_iter + 1):
        gU, gJ = state_at(x)
        ctx.mesh_redistribute(mon, gU, gJ, x, disp, tau, None)
        x += disp
        ctx.es_fill_ghosts_x(x)
        if float(disp.abs().max().item()) < tol * h:
            break
    jx = torch.empty((d * d,) + tuple(x.shape[1:]), dtype=torch.float64, device="cuda")
    ctx.es_metrics(x, None, 0.0, None, jx, None)
    J = torch.empty((1,) + tuple(x.shape[1:]), dtype=torch.float64, device="cuda")
    ctx.es_jacobian(x, jx, J)
    gU, gJ = state_at(x, J)
    return gU, gJ, it


def vortex_study(args):
    """The isentropic-vortex workloads (Section 5, Examples 5.1 and 5.5) on a
    moving mesh with the gradient + Laplacian monitor: l1 and linf errors in
    rho against the exact solution at the nodes, and their orders, 2D at
    t = 4 (N = 40..320, moving and fixed mesh) and 3D at t = 0.1 (N =
    20..160), with the time step C_CFL (Delta xi / L)^(5/3); moving-mesh runs
    start from the adapted initial mesh.  Then the total entropy
    sum_i J eta dV of the EC and ES schemes over time at 2D N = 160."""
    import numpy as np
    import torch

    from paper_2202_07989_amd import es
    from paper_2202_07989_amd import inputs as I

    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()

    def run(dim, n, t_end, dissipation=1, n_entropy=0, move=True):
        sp = I.spec_vortex(dim, n)
        sp["dissipation"] = dissipation
        JU, J, x = I.init_vortex(sp)
        ctx = es.Context(sp)
        gU, gJ, gx = dev(JU), dev(J), dev(x)
        ctx.es_fill_ghosts(gU, 2 + dim)
        ctx.es_fill_ghosts(gJ, 1)
        ctx.es_fill_ghosts_x(gx)
        mon = I.vortex_monitor()
        adapt_iters = 0
        if move:
            gU, gJ, adapt_iters = adapt_initial_mesh(ctx, sp, mon, gx,
                                                     lambda pts: I.vortex_prims(dim, pts, 0.0))
        dt0 = (0.4 if dim == 2 else 0.3) * (1.0 / n) ** (5.0 / 3.0)
        ns = int(np.ceil(t_end / dt0))
        dt = t_end / ns
        ent = torch.zeros(1, dtype=torch.float64, device="cuda")
        series = []
        every = max(1, ns // n_entropy) if n_entropy else 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(ns):
            if every and s % every == 0:
                ctx.es_entropy(gU, gJ, ent)
                series.append((s * dt, float(ent.item())))
            ctx.es_step(gU, gJ, gx, mon=mon if move else None, dt_fixed=dt, move_mesh=move)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if every:
            ctx.es_entropy(gU, gJ, ent)
            series.append((ns * dt, float(ent.item())))
        rc, _ = ctx.es_status()
        Iin = I.interior(sp)
        hU, hJ, hx = (a.cpu().numpy() for a in (gU, gJ, gx))
        rho = hU[Iin][0] / hJ[Iin][0]
        ex, _, _ = I.vortex_prims(dim, [hx[Iin][k] for k in range(dim)], t_end)
        err = np.abs(rho - ex)
        print(f"[vortex] {dim}D N={n} {'moving' if move else 'fixed'} steps={ns} l1={err.mean():.3e} "
              f"linf={err.max():.3e} "
              f"{wall:.1f}s status={rc}", file=sys.stderr, flush=True)
        return dict(n=n, steps=ns, l1=float(err.mean()), linf=float(err.max()), ms_per_step=1e3 * wall / ns,
                    status=rc, initial_mesh_iterations=adapt_iters), series

    out = {"mode": "vortex"}
    for dim, t_end, Ns, move in ((2, 4.0, (40, 80, 160, 320), True), (2, 4.0, (40, 80, 160, 320), False),
                                 (3, 0.1, (20, 40, 80, 160), True)):
        rows = [run(dim, n, t_end, move=move)[0] for n in Ns]
        for a, b in zip(rows[:-1], rows[1:]):
            b["order_l1"] = float(np.log2(a["l1"] / b["l1"]))
            b["order_linf"] = float(np.log2(a["linf"] / b["linf"]))
        out[f"{dim}d_{'moving' if move else 'fixed'}"] = {"t": t_end, "rows": rows}
    ent = {}
    for name, diss in (("EC", 0), ("ES", 1)):
        _, series = run(2, 160, 4.0, dissipation=diss, n_entropy=40)
        ent[name] = series
    out["entropy_2d_160"] = {k: {"t": [t for t, _ in v], "total": [e for _, e in v],
                                 "change_end": v[-1][1] - v[0][1],
                                 "nonincreasing": all(b <= a for (_, a), (_, b) in zip(v, v[1:]))}
                             for k, v in ent.items()}
    print(json.dumps(out), flush=True)


def batch_study(args):
    """The batched form: 64 independent 2D two-species instances of uneven
    size (seeded, 128^2..1024^2, 4-quadrant Riemann data, fixed uniform
    mesh, CFL 0.4 per instance).  One step is the per-instance wave speed and
    three stages, one launch each, captured once in a hipGraph and replayed
    --steps times; FP64 and mixed, after the autotuner has picked the region
    size.  The same steps done instance by instance with the single-instance
    calls (64 x (wave speed + 3 x (stage + 2 ghost fills))) are timed as the
    unbatched baseline."""
    import numpy as np
    import torch

    from paper_2202_07989_amd import es
    from paper_2202_07989_amd import inputs as I

    insts = I.init_c5(count=args.count)
    cells = sum(sp["n"][0] * sp["n"][1] for sp, _, _, _ in insts)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    U0 = [dev(JU) for _, JU, _, _ in insts]
    J0 = [dev(J) for _, _, J, _ in insts]
    jx = []
    for (sp, JU, J, x) in insts:
        ctx = es.Context(sp)
        gxm = dev(x)
        ctx.es_fill_ghosts_x(gxm)
        m = torch.empty((4,) + tuple(J.shape[1:]), dtype=torch.float64, device="cuda")
        ctx.es_metrics(gxm, None, 0.0, None, m, None)
        ctx.es_fill_ghosts(U0[len(jx)], sp["nspec"] + 3)
        ctx.es_fill_ghosts(J0[len(jx)], 1)
        jx.append(m)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    out = {"mode": "batch", "instances": len(insts), "cells": cells,
           "sizes_min_max": [min(sp["n"][0] for sp, _, _, _ in insts), max(sp["n"][0] for sp, _, _, _ in insts)],
           "steps": args.steps}

    def timed(fn, reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    for prec_name, prec in (("fp64", es.ES_FP64), ("mixed", es.ES_MIXED)):
        b = es.Batch([sp for sp, _, _, _ in insts], precision=prec)
        gU, gJ = [t.clone() for t in U0], [t.clone() for t in J0]
        tU, tJ, tx = es.PtrTable(gU), es.PtrTable(gJ), es.PtrTable(jx)
        dt = torch.zeros(len(insts), dtype=torch.float64, device="cuda")
        b.max_wavespeed_batched(tU, tJ, tx, 0.4, None, dt)
        region, pers = b.es_batch_autotune(tU, tJ, tx, None, dt, reps=3)
        # one stage alone (the dominant kernel), timed on the stream it runs on
        oU, oJ = es.PtrTable([torch.empty_like(t) for t in gU]), es.PtrTable([torch.empty_like(t) for t in gJ])
        stage = lambda: b.es_rk_stage_batched(1, dt, tU, tJ, tU, tJ, tx, None, oU, oJ)
        stage()
        ms_stage = timed(stage, 10)
        # whole steps through a graph
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            b.es_step_batched(0.4, tU, tJ, tx, None, dt)
        stream.wait_stream(side)
        torch.cuda.synchronize()
        for a, c in zip(gU + gJ, U0 + J0):
            a.copy_(c)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            b.es_step_batched(0.4, tU, tJ, tx, None, dt)
        graph.replay()
        torch.cuda.synchronize()
        for a, c in zip(gU + gJ, U0 + J0):
            a.copy_(c)
        torch.cuda.synchronize()
        ms_step = timed(graph.replay, args.steps)
        rc, _ = b.es_batch_status()
        flops = FLOPS_PER_CELL_STAGE[(2, 2)] * cells / (ms_stage / 1e3) / 1e12
        peak = PEAK_FP64_TFLOPS if prec == es.ES_FP64 else PEAK_FP32_TFLOPS
        out[prec_name] = {"value": cells * 3 / (ms_step / 1e3), "unit": "cell-stage updates/s",
                          "ms_per_step": ms_step, "stage_ms": ms_stage, "region": region,
                          "persistent": pers, "stage_achieved_TFLOPs": flops, "peak_TFLOPs": peak,
                          "stage_frac": flops / peak,
                          "stage_algorithmic_hbm_frac": BYTES_PER_CELL_STAGE[(2, 2)] * cells
                          / (ms_stage / 1e3) / 1e9 / PEAK_HBM_GBS,
                          "status": rc}
        del graph, b
        torch.cuda.empty_cache()

    # unbatched baseline: the same FP64 steps, instance by instance
    ctxs = [es.Context(sp) for sp, _, _, _ in insts]
    gU, gJ = [t.clone() for t in U0], [t.clone() for t in J0]
    bufs = [[torch.empty_like(u), torch.empty_like(j), torch.empty_like(u), torch.empty_like(j)]
            for u, j in zip(gU, gJ)]
    dts = [torch.zeros(1, dtype=torch.float64, device="cuda") for _ in insts]

    def seq_step():
        for k, c in enumerate(ctxs):
            c.max_wavespeed(gU[k], gJ[k], jx[k], 0.4, None, dts[k])
            A, AJ, B, BJ = bufs[k]
            for st, (sU, sJ, oU_, oJ_) in enumerate(((gU[k], gJ[k], A, AJ), (A, AJ, B, BJ), (B, BJ, A, AJ))):
                c.es_rk_stage(st, dts[k], gU[k], gJ[k], sU, sJ, jx[k], None, oU_, oJ_)
                c.es_fill_ghosts(oU_, 5)
                c.es_fill_ghosts(oJ_, 1)
            gU[k].copy_(A)
            gJ[k].copy_(AJ)

    seq_step()
    torch.cuda.synchronize()
    ms_seq = timed(seq_step, max(1, args.steps // 4))
    out["fp64_sequential"] = {"value": cells * 3 / (ms_seq / 1e3), "ms_per_step": ms_seq,
                              "note": "per instance: max_wavespeed, 3 x (es_rk_stage + 2 ghost fills), "
                                      "state copy; not graph-captured"}
    out["batched_speedup_vs_sequential"] = out["fp64"]["value"] / out["fp64_sequential"]["value"]
    out["mixed_speedup_vs_fp64"] = out["mixed"]["value"] / out["fp64"]["value"]
    print(json.dumps(out), flush=True)


# The paper's walled two-species examples, run to their final times: the
# CPU times it reports for them (Tables 5.2 and 5.3, 32 cores of two Xeon
# E5-2697A v4), quoted as context next to the GPU's wall-clock time.
EXAMPLES = {
    # the tri-point filters its monitor 10 times (the top of the paper's
    # 3-10): with 3, the mesh gathers so tightly at the mixing layers that the
    # 1e-5 partial density turns negative near t = 2.8 (the scheme has no
    # positivity limiter)
    "tripoint": dict(t_end=5.0, alpha=1200.0, n_smooth=10, paper_s={"moving": 201.0, "uniform": 49.0},
                     what="Example 5.7 tri-point, 350 x 150, t = 5"),
    "shock-bubble-he": dict(t_end=0.676, alpha=1000.0, paper_s={"moving": 3840.0, "uniform": 552.0},
                            case="he", n=(800, 160),
                            what="Example 5.8 shock / helium bubble, 800 x 160, t = 0.676"),
    # Example 5.9's own monitor: schlieren function, speed, partial
    # densities and pressure
    "shock-bubble-stiff": dict(t_end=0.8, monitor="m7", paper_s={"moving": 568.0, "uniform": 107.0},
                               case="stiff", n=(800, 160),
                               what="Example 5.9 shock / bubble in stiffened gas, 800 x 160, t = 0.8"),
    # 10 filter passes here too: with 3 the mesh gathers around the light
    # bubble until the smallest J is 5e-4 (t = 0.07) and then tangles
    "shock-bubble-he-3d": dict(t_end=0.72, alpha=1200.0, n_smooth=10,
                               paper_s={"moving": 39960.0, "uniform": 9240.0},
                               case="he", n=(400, 80, 80),
                               what="Example 5.10 3D shock / helium bubble, 400 x 80 x 80, t = 0.72"),
    "shock-bubble-stiff-3d": dict(t_end=0.64, sigma=(1, 3), alpha=(500.0, 500.0),
                                  paper_s={"moving": 7740.0, "uniform": 2792.0}, case="stiff", n=(400, 80, 80),
                                  what="Example 5.11 3D shock / bubble in stiffened gas, 400 x 80 x 80, t = 0.64"),
}


def example_run(args):
    """One of the paper's walled examples (reflecting walls; outflow and
    inflow for the shock-bubble runs) advanced to its final time at CFL 0.4
    (0.3 in 3D) with 10 Jacobi sweeps and 3 filter passes per step (the paper's
    settings; 10 passes for the tri-point and Example 5.10), on the moving mesh or the uniform mesh (--mesh).  Reports the
    wall-clock time from the first step to the last (inputs resident on the
    GPU; blocks of --graph-steps CFL steps replay from a captured HIP graph
    with their dt read back per block, the last steps run eagerly to land on
    the final time), the
    cell-stage rate, the smallest partial density, and for walls on every
    face the drift of species mass and energy."""
    import numpy as np
    import torch

    from paper_2202_07989_amd import es
    from paper_2202_07989_amd import inputs as I

    ex = EXAMPLES[args.example]
    if args.example == "tripoint":
        sp = I.spec_tripoint()
        JU, J, x = I.init_tripoint(sp)
    else:
        sp = I.spec_shock_bubble_walled(ex["case"], ex["n"])
        JU, J, x = I.init_shock_bubble_walled(sp)
    if args.precision == "mixed":
        prec = es.ES_MIXED
    else:
        prec = es.ES_FP64
    if ex.get("monitor") == "m7":
        mon = I.monitor_m7(n_sweeps=10, n_smooth=ex.get("n_smooth", 3))
    else:
        alpha = ex["alpha"] if isinstance(ex["alpha"], tuple) else (ex["alpha"],)
        mon = I.monitor_spec(n_sweeps=10, n_smooth=ex.get("n_smooth", 3), sigma=ex.get("sigma", (0,)),
                             alpha=alpha)
    cfl = 0.4 if sp["dim"] == 2 else 0.3
    move = args.mesh == "moving"
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    ctx = es.Context(sp, precision=prec)
    gU, gJ, gx = dev(JU), dev(J), dev(x)
    Iin = I.interior(sp)
    m0 = gU[Iin].sum(dim=(1, 2, 3)).cpu().numpy()
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    t, steps, dt_prev = 0.0, 0, None
    t_end = ex["t_end"]
    K = args.graph_steps
    graph = None
    dts = torch.zeros(K, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last_print = t0
    while t < t_end * (1 - 1e-14):
        rem = t_end - t
        if graph is not None and rem > 1.5 * K * dt_prev:
            # K CFL steps replayed from the graph, their dt read back at once
            graph.replay()
            block = dts.cpu().numpy()
            t += float(block.sum())
            dt_prev = float(block[-1])
            steps += K
            dt = dt_prev
        else:
            fixed = 0.0
            if dt_prev is not None and rem <= dt_prev:
                fixed = rem
            elif dt_prev is not None and rem < 2.0 * dt_prev:
                fixed = 0.5 * rem
            ctx.es_step(gU, gJ, gx, mon=mon, cfl=cfl, dt_fixed=fixed, move_mesh=move, dt_dev=dt_dev)
            dt = float(dt_dev.item())
            t += dt
            dt_prev = dt
            steps += 1
            if graph is None and K > 1 and steps == 1:
                # every workspace exists after the first step: capture K steps
                graph = torch.cuda.CUDAGraph()
                with torch.cuda.graph(graph):
                    for k in range(K):
                        ctx.es_step(gU, gJ, gx, mon=mon, cfl=cfl, move_mesh=move, dt_dev=dts[k:k + 1])
                # capture recorded the steps without running them
        if steps % 200 < max(K, 1) and (ctx.es_status()[0] != es.ES_OK or not math.isfinite(dt)
                                        or steps > 400000):
            break
        now = time.perf_counter()
        if now - last_print > 30.0:
            print(json.dumps({"example": args.example, "step": steps, "t": t, "dt": dt}), flush=True)
            last_print = now
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rc, flags = ctx.es_status()
    hU, hJ, hx = gU.cpu().numpy(), gJ.cpu().numpy(), gx.cpu().numpy()
    rho = hU[Iin][:2] / hJ[Iin]
    cells = int(np.prod(sp["n"][:sp["dim"]]))
    out = {"mode": "example", "example": ex["what"], "mesh": args.mesh, "precision": args.precision,
           "status": rc, "steps": steps, "t_end": t, "wall_s": wall, "ms_per_step": 1e3 * wall / steps,
           "cell_stage_updates_per_s": 3.0 * cells * steps / wall,
           "min_partial_density": [float(rho[0].min()), float(rho[1].min())],
           "min_J": float(hJ[Iin].min()),
           "paper_cpu_s_32_cores": ex["paper_s"][args.mesh],
           "data": "the paper's initial data, region boundaries spread over one cell"}
    if args.example == "tripoint":
        m1 = hU[Iin].sum(axis=(1, 2, 3))
        out["mass_energy_rel_drift"] = [float(abs(m1[c] - m0[c]) / abs(m0[c])) for c in (0, 1, 4)]
    if args.save:
        np.savez_compressed(args.save, JU=hU[Iin], J=hJ[Iin], x=hx[Iin], t=t, steps=steps)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--precision", choices=["fp64", "mixed", "both"], default="both",
                    help="both: FP64 gives the reported value, the mixed form is timed beside it")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stage-reps", type=int, default=10)
    ap.add_argument("--mode", choices=["step", "stage", "accuracy", "batch", "vortex", "example", "full-length",
                                       "oracle-rate"],
                    default="step",
                    help="stage: only the fused-RK-stage loop and a 2 GiB device copy (for "
                         "rocprofv3 counter runs; the copy calibrates FETCH_SIZE/WRITE_SIZE); "
                         "accuracy: FP64 vs mixed (and vs an oracle reference file) after --steps steps; "
                         "batch: the 64-instance batched 2D form, FP64 and mixed, vs sequential launches; "
                         "vortex: the isentropic-vortex convergence and entropy studies; "
                         "example: one of the paper's walled examples to its final time; "
                         "full-length: the 512^2 (200 steps) and 256^3 (50 steps) shock-bubble runs "
                         "with their status; oracle-rate: the CPU oracle's stage rate alone (no GPU)")
    ap.add_argument("--example", choices=sorted(EXAMPLES), default="shock-bubble-he")
    ap.add_argument("--mesh", choices=["moving", "uniform"], default="moving",
                    help="example mode: MM (moving mesh) or UM (uniform mesh) runs")
    ap.add_argument("--save", default=None, help="example mode: .npz of the final interior state")
    ap.add_argument("--graph-steps", type=int, default=16,
                    help="example mode: CFL steps per captured HIP graph (1: every step eager)")
    ap.add_argument("--count", type=int, default=64, help="batch mode: number of instances")
    ap.add_argument("--reconstruction", choices=["mr", "js"], default="mr",
                    help="step/stage modes: multi-resolution WENO (the method) or the classical "
                         "WENO5 of the comparison variant MM-WENOJS")
    ap.add_argument("--no-configs", action="store_true", help="step mode: skip the 2D configuration rates")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="step mode: end with a 2 GiB device-to-device copy (calibrates the FETCH_SIZE and "
                         "WRITE_SIZE counters of rocprofv3 runs)")
    ap.add_argument("--oracle-ref", default=None,
                    help="accuracy mode: .npz written by the oracle's reference script")
    args = ap.parse_args()
    if args.reconstruction == "js" and args.precision != "fp64":
        ap.error("--reconstruction js runs in FP64 only (add --precision fp64)")
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    if args.mode == "oracle-rate":
        rate, reps, el = oracle_stage_rate(args.n, 10.0, 20)
        th = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
        print(json.dumps({"value": rate, "sample": f"{reps} fused RK stage(s) of the oracle on a {args.n}^3 "
                          f"box of the same data ({el:.1f} s, {th} thread(s))"}), flush=True)
        return

    import numpy as np
    import torch

    from paper_2202_07989_amd import es
    from paper_2202_07989_amd import inputs as I

    torch.cuda.set_device(0)
    n = args.n
    if args.mode == "accuracy":
        accuracy_study(args)
        return
    if args.mode == "batch":
        batch_study(args)
        return
    if args.mode == "vortex":
        vortex_study(args)
        return
    if args.mode == "example":
        example_run(args)
        return
    if args.mode == "full-length":
        full_length(args)
        return
    if args.mode == "stage":
        sp = spec_for(args, I, n)
        prec = es.ES_MIXED if args.precision == "mixed" else es.ES_FP64
        JU, J, x = I.init_shock_bubble(sp)
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        gU, gJ, gx = dev(JU), dev(J), dev(x)
        ctx = es.Context(sp, precision=prec)
        ctx.es_fill_ghosts(gU, sp["nspec"] + 4)
        ctx.es_fill_ghosts(gJ, 1)
        ctx.es_fill_ghosts_x(gx)
        mon = I.monitor_spec(n_sweeps=5, n_smooth=3, sigma=(0,), alpha=(1200.0,))
        dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
        run_stage_only(ctx, mon, 0.3, gU, gJ, gx, dt_dev, args.stage_reps)
        rc, _ = ctx.es_status()
        print(json.dumps({"mode": "stage", "status": rc}), flush=True)
        return

    main_prec = "mixed" if args.precision == "mixed" else "fp64"
    r = run_precision(args, main_prec, n, args.steps, args.warmup, args.stage_reps)
    counters = load_counters() if main_prec == "fp64" else {}
    traffic = counters.get("bytes_per_stage")
    executed = counters.get("executed_fp64_flops_per_cell_stage")
    cells = n ** 3
    key = (3, 2)
    out = {
        "metric": "cell-stage updates/s, 3D 256^3 two-species, FP64 vs mixed FP32; % HBM peak",
        "value": r["value"],
        "unit": "cell-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"3D two-species stiffened-gas shock-bubble {n}^3, moving mesh "
                               "(5 Jacobi sweeps, 3 filter passes, alpha 1200), CFL 0.3, "
                               f"6th-order EC + {'MR-WENO5' if args.reconstruction == 'mr' else 'WENO5-JS'} "
                               "ES flux, SSP-RK3",
                   "grid": [n, n, n], "species": 2, "precision": main_prec,
                   "reconstruction": args.reconstruction},
        "hbm_frac_of_peak_step": BYTES_PER_CELL_STAGE[key] * r["value"] / 1e9 / PEAK_HBM_GBS,
        "roofline": {"bound": "alu", "achieved": r["achieved"], "peak": r["peak"], "unit": "TFLOP/s",
                     "frac": r["achieved"] / r["peak"], "traffic": traffic,
                     "kernel": "es_rk_stage (k_rhs_xy for x and y, k_rhs_dir along z with the stage epilogue)",
                     "ms_per_launch": r["ms_stage"], "algorithmic_hbm_GBs": r["hbm_gbs"],
                     "algorithmic_hbm_frac": r["hbm_gbs"] / PEAK_HBM_GBS,
                     "flops_per_cell_stage": FLOPS_PER_CELL_STAGE[key],
                     "executed_flops_per_cell_stage": executed,
                     "executed_frac": (executed * cells / (r["ms_stage"] / 1e3) / 1e12 / r["peak"]) if executed else None},
        "status": r["status"],
        "wall_s": r["wall"],
        "es_rhs_alone": {"ms_per_call": r["ms_rhs"], "cell_updates_per_s": cells / (r["ms_rhs"] / 1e3),
                         "note": "x-y launch and z sweep writing d(JU)/dt and dJ/dt, same state and metrics"},
        "es_rk_stage": {"ms_per_call": r["ms_stage"], "cell_stage_updates_per_s": cells / (r["ms_stage"] / 1e3)},
    }
    if args.precision == "both":
        m = run_precision(args, "mixed", n, args.steps, args.warmup, args.stage_reps)
        out["mixed"] = {"dtype": "f32+f64", "value": m["value"], "ms_per_step": m["ms_step"],
                        "speedup_vs_fp64": m["value"] / r["value"],
                        "stage_ms_per_launch": m["ms_stage"],
                        "stage_achieved_TFLOPs": m["achieved"], "peak_fp32_TFLOPs": m["peak"],
                        "stage_frac": m["achieved"] / m["peak"], "status": m["status"],
                        "es_rhs_alone_ms": m["ms_rhs"]}
    if not args.no_configs:
        out["configs_2d"] = config_rates()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(r["sp"], r["JU"], r["J"], r["x"], n)
    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float64, device="cuda")     # 2 GiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration_bytes_each_way"] = a.numel() * 8
        del a, b
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
