"""Benchmark of the ParaDIAG hot path on one MI355X.

One step = one ParaDIAG application of eq. (1) to a batch of time slices:
G = (V^{-1} kron I) F on the FP64 matrix cores, the n shifted systems
(A + lambda_j I) z_j = g_j solved to 1e-10 relative residual by V(2,2) Vanka
multigrid, and U = (V kron I) Z.

Headline workload (the precision workload): the 2047 x 2047 unit-square grid
with the 32 alpha-circulant shifts (alpha = 0.01, tau = 1/32); F is chosen as
(V kron I) b with b_j ~ U(-1, 1) + i U(-1, 1), so the shifted systems see
exactly those right-hand sides.  `value` is the FP64 step's systems/s; the
same step with complex64 V-cycles inside FP64 refinement and with FP64
V-cycles whose coarse-grid correction runs in complex64 are reported beside
it, with their speedups and each result's error against the FP64 oracle on
a sample of systems.  Side legs: the same step on 1023 x 1023 with 64
shifts, the 63 x 63 latency case (microseconds per solve), the uneven batch,
the paper's protocol and the heat (differentiation) workload.

Prints one JSON line.  Inputs are resident in HBM before the timed region.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "shifted systems solved/s to 1e-10 rel. residual, FP32+IR vs FP64; HBM GB/s"
HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6

# HBM bytes per launch of the dominant kernel measured with rocprofv3
# FETCH_SIZE and WRITE_SIZE on each workload, each scaled by its reading for a
# plain 1 GiB copy (profiles/), for its plain-block (plan 1) and paced-block
# (plan 2) form (the autotuned run's form, and the other one with
# VMG_EDGE_PACE set).  Valid
# only for the kernel source it was measured on: reported as null once that
# file changes.
MEASURED_TRAFFIC = {"source": "vmg_stream.hip", "source_sha256_16": "3b90151f9b194231",
                    "bytes_per_launch": {"precision_2047": {1: 8127.1e6, 2: 7725.7e6},
                                         "plain_1023": {1: 4047.8e6, 2: 3886.6e6}}}
# finest level across the boundary of two V-cycles: correction + 2 sweeps +
# stopping-test norm, then the next cycle's 2 sweeps + residual + restriction
# (template arguments: precision, sweeps after and before the boundary, the
# coarse level's precision, damped Jacobi instead of Vanka, waves a block:
# 12 in the paced blocks the autotuner may choose, else 4)
def dominant_kernel(plan_edge):
    return "k_edge<double, 2, 2, double, false, %d>" % (12 if plan_edge == 2 else 4)
# systems of the headline workload the oracle solves (the cpu baseline and
# the per-result errors): the smallest and the largest |lambda_j|
ORACLE_SAMPLE = (0, 16)


def progress(msg):
    """One line on stderr per finished part of the run (stdout carries only
    the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash(name):
    import hashlib
    path = os.path.join(ROOT, "paper_2203_11154_amd", "csrc", name)
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--tol", type=float, default=1e-10)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample", type=int, default=len(ORACLE_SAMPLE),
                   help="systems of the headline workload the oracle solves (cpu baseline, per-result errors)")
    p.add_argument("--no-autotune", action="store_true", help="keep the size heuristic kernel schedule")
    p.add_argument("--legs", default="all",
                   help="comma list of parts to run: headline (2047^2 x 32), plain (1023^2 x 64), small (63^2 x 8), "
                        "batched, paper, heat; default all")
    p.add_argument("--copy-calibration", action="store_true",
                   help="run one plain 1 GiB device copy first (reference for hardware byte counters)")
    return p.parse_args()


def host_info():
    """The host the CPU baseline ran on: logical CPUs, those this process may
    use, CPU model and RAM."""
    info = {"nproc": os.cpu_count()}
    try:
        info["affinity_cpus"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    info["ram_GiB"] = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    return info


def cpu_baseline(b, lam, h, tol, sample, gpu_solutions):
    """The FP64 oracle on a bounded sample of the headline workload: the
    systems `sample` solved to `tol` (transforms excluded), BLAS limited to
    one thread so the core count is exact.  Also each GPU result's relative
    error against the oracle's solution of the same system."""
    from threadpoolctl import threadpool_limits
    from oracle import multigrid as omg
    idx = list(sample)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        z_or, iters, relres, _ = omg.solve(b[idx], lam[idx], h, tol=tol)
        dt = time.perf_counter() - t0
    errors = {}
    for name, zs in gpu_solutions.items():
        errors[name] = {str(j): float(np.linalg.norm((zs[k] - z_or[k]).ravel()) / np.linalg.norm(z_or[k].ravel()))
                        for k, j in enumerate(idx)}
    return {"value": len(idx) / dt, "unit": "systems/s", "cores": 1, "kind": "oracle",
            "sample": f"systems {idx} of the {len(lam)} shifted systems at {b.shape[-1]}^2, V(2,2) to {tol:g} "
                      f"({int(iters.sum())} cycles, {dt:.1f} s; transforms excluded)",
            "oracle_cycles": iters.tolist(), "oracle_relres": relres.tolist(), "host": host_info(),
            "gpu_error_vs_oracle": errors}


def run_steps(solver, V, Vinv, F, U, steps, tol, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    status = 0
    for _ in range(steps):
        _, status = solver.paradiag_apply(V, Vinv, F, tol=tol, out=U)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, status


def kernel_breakdown(solver, Vd, Vinvd, Fd, Ud, steps, tol, S, n, torch):
    """Per kernel class and per level: a separate pass with every kernel class
    timed by HIP events (its events perturb the step, so it is not timed as a
    whole)."""
    solver.set_timing(True, reset=True)
    run_steps(solver, Vd, Vinvd, Fd, Ud, steps, tol, torch)
    stats = solver.kernel_stats()
    solver.set_timing(False, reset=False)
    levels = {}
    for k in ("down", "up", "edge"):
        levels[k] = [{"level": l, "launches": a, "avg_ms": round(m / max(a, 1), 4),
                      "GB/s": round(b_ / (m * 1e-3) / 1e9, 1) if m > 0 else None}
                     for l, a, m, b_ in solver.level_stats(k)]
    kernels = {k: {"launches": v[0], "ms": round(v[1], 3),
                   "GB/s": round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[1] > 0 else None,
                   "hbm_frac": round(v[2] / (v[1] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if v[1] > 0 else None}
               for k, v in stats.items() if v[0] > 0}
    tl, tms, _ = stats["transform"]
    if tl and tms > 0:
        flops = 8.0 * S * S * n * n * tl
        kernels["transform"]["TFLOP/s"] = round(flops / (tms * 1e-3) / 1e12, 2)
        kernels["transform"]["mfma_frac"] = round(flops / (tms * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFLOPS, 4)
    return kernels, levels


def edge_kernel_rate(edge_levels):
    """Level-0 cycle-edge launches of a timed pass: launches, average ms,
    algorithmic bytes per launch and GB/s."""
    for lvl, la, ms, by in edge_levels:
        if lvl == 0 and la > 0 and ms > 0:
            return {"launches": la, "avg_ms": round(ms / la, 5), "algorithmic_bytes_per_launch": round(by / la),
                    "GB/s": round(by / (ms * 1e-3) / 1e9, 1),
                    "hbm_frac": round(by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    return None


PRECISIONS = (("fp64", {}, "c128"),
              ("fp32_ir", {"precision": "c64_ir", "ir_inner": 2}, "c64 cycles + c128 refinement"),
              ("fp32_coarse", {"precision": "c128_c64"},
               "c128 finest level and stopping test, c64 coarse-grid correction"))


def paradiag_leg(name, n, S, seed, args, torch, sample=(), breakdown=True, dft=True):
    """One ParaDIAG step workload (n x n grid, S alpha-circulant shifts,
    right-hand sides from `seed`) in the three precisions: FP64 V-cycles,
    complex64 V-cycles inside FP64 refinement, FP64 V-cycles with a complex64
    coarse-grid correction.  Timed steps record HIP events around the
    finest-level cycle-edge kernel only.  Returns the leg's results and, for
    the systems in `sample`, each precision's solution (host arrays)."""
    from paper_2203_11154_amd import Grid, VankaMG, inputs
    tol = args.tol
    lam = inputs.alpha_circulant_shifts(S, 0.01)
    V, Vinv = inputs.alpha_circulant_vectors(S, 0.01)
    b = inputs.rhs(S, n, n, seed=seed)
    dev = torch.device("cuda:0")
    Fd = torch.from_numpy(np.ascontiguousarray(V @ b.reshape(S, -1)).ravel()).to(dev)
    Vd = torch.from_numpy(V).to(dev).contiguous()
    Vinvd = torch.from_numpy(Vinv).to(dev).contiguous()
    Ud = torch.empty_like(Fd)
    bd = torch.from_numpy(b.reshape(-1)).to(dev) if len(sample) else None
    out = {"workload": f"{name}: {S} alpha-circulant shifts (alpha=0.01, tau=1/{S}) on the {n}x{n} unit-square "
                       f"grid, ParaDIAG step (transform, V(2,2) Vanka multigrid to {tol:g}, inverse transform)",
           "grid": n, "systems": S}
    solutions = {}
    m = n * n
    for pname, kw, dtype in PRECISIONS:
        s = VankaMG([Grid(n, num_systems=S)], lam, **kw)
        schedule = s.autotune() if not args.no_autotune else [s.schedule(0)]
        for _ in range(args.warmup):
            s.paradiag_apply(Vd, Vinvd, Fd, tol=tol, out=Ud)
        s.set_timing(True, reset=True, classes=["edge"])
        dt, st = run_steps(s, Vd, Vinvd, Fd, Ud, args.steps, tol, torch)
        edge = edge_kernel_rate(s.level_stats("edge"))
        s.set_timing(False, reset=False)
        it, rr = s.last_stats()
        r = {"value": round(S * args.steps / dt, 2), "unit": "systems/s",
             "ms_per_step": round(1e3 * dt / args.steps, 3), "dtype": dtype,
             ("cycles" if pname != "fp32_ir" else "refinement_steps"): {"min": int(it.min()), "max": int(it.max())},
             "max_relres": float(rr.max()), "converged": st == 0 and bool(np.all(rr <= tol)),
             "levels": len(s.levels()), "schedule": schedule[0], "edge_kernel": edge, "edge_plan": s.plan(0)[0]}
        if pname == "fp64":
            # the same steps without any event (cycles replayed as graphs);
            # the host window (CLOCK_MONOTONIC) locates them in a kernel trace
            w0 = time.monotonic_ns()
            dtg, _ = run_steps(s, Vd, Vinvd, Fd, Ud, args.steps, tol, torch)
            w1 = time.monotonic_ns()
            r["uninstrumented"] = {"ms_per_step": round(1e3 * dtg / args.steps, 3),
                                   "value": round(S * args.steps / dtg, 2),
                                   "timed_window_monotonic_ns": [w0, w1]}
            if dft:
                # the alpha-circulant transforms as scaled DFTs instead of the
                # MFMA GEMMs
                for _ in range(args.warmup):
                    s.paradiag_apply_circulant(0.01, Fd, tol=tol, out=Ud)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    _, st_c = s.paradiag_apply_circulant(0.01, Fd, tol=tol, out=Ud)
                torch.cuda.synchronize()
                dtc = time.perf_counter() - t0
                _, rr_c = s.last_stats()
                r["circulant_dft_step"] = {"ms_per_step": round(1e3 * dtc / args.steps, 3),
                                           "value": round(S * args.steps / dtc, 2),
                                           "converged": st_c == 0 and bool(np.all(rr_c <= tol)),
                                           "note": f"transforms as scaled length-{S} DFTs, uninstrumented"}
        if breakdown:
            r["kernels"], r["fused_by_level"] = kernel_breakdown(s, Vd, Vinvd, Fd, Ud, min(args.steps, 3), tol, S, n,
                                                                 torch)
        if len(sample):
            # the shifted solves on their own (right-hand sides b), for the
            # per-result error against the oracle
            Z, _, rr_s, _ = s.solve(bd, tol=tol)
            torch.cuda.synchronize()
            solutions[pname] = np.stack([Z[j * m:(j + 1) * m].cpu().numpy().reshape(n, n) for j in sample])
            del Z
        out[pname] = r
        progress(f"{name} {pname}: {r['ms_per_step']} ms/step, max relres {r['max_relres']:.3e}")
        del s
        torch.cuda.empty_cache()
    f64 = out["fp64"]["ms_per_step"]
    for pname in ("fp32_ir", "fp32_coarse"):
        out[pname]["speedup_vs_fp64"] = round(f64 / out[pname]["ms_per_step"], 3)
    del Fd, Ud, bd
    torch.cuda.empty_cache()
    return out, solutions, (b, lam, 1.0 / (n + 1))


def small_leg(args, torch):
    """The latency case: 8 alpha-circulant shifts (tau = 1/8) on 63 x 63, V(2,2)
    with 5 levels to 1e-10, one batched solve (graph replay): microseconds
    per solve of all 8 systems."""
    from paper_2203_11154_amd import Grid, VankaMG, inputs
    n, S = 63, 8
    lam = inputs.alpha_circulant_shifts(S)
    bd = torch.from_numpy(inputs.rhs(S, n, n).ravel()).cuda()
    s = VankaMG([Grid(n, num_systems=S, levels=5)], lam)
    Z, _, _, _ = s.solve(bd, tol=args.tol)
    for _ in range(max(args.warmup, 3)):
        s.solve(bd, tol=args.tol, out=Z)
    reps = max(20, args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        _, it, rr, st = s.solve(bd, tol=args.tol, out=Z)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    return {"workload": "8 alpha-circulant shifts on 63x63, V(2,2), 5 levels, to 1e-10 (cache-resident, latency bound)",
            "us_per_solve": round(1e6 * dt, 1), "us_per_system": round(1e6 * dt / S, 1),
            "value": round(S / dt, 1), "unit": "systems/s", "cycles": {"min": int(it.min()), "max": int(it.max())},
            "max_relres": float(rr.max()), "converged": st == 0 and bool(np.all(rr <= args.tol)),
            "note": "host-timed solves (enqueue, device stopping test, host read of the counts) averaged over "
                    f"{reps} calls"}


def batched_leg(args, torch):
    """384 systems on uneven grids (256 x 127^2, 96 x 255^2, 32 x 511^2) with
    shifts Re ~ U(1, 1e4), Im ~ U(-1e4, 1e4), solved to 1e-10 in one batched,
    graph-replayed solve per step."""
    from paper_2203_11154_amd import Grid, VankaMG, inputs
    groups = [(127, 256), (255, 96), (511, 32)]
    S = sum(c for _, c in groups)
    lam = inputs.uniform_shifts(S)
    b = np.concatenate([inputs.rhs(c, n, n, seed=60 + k).ravel() for k, (n, c) in enumerate(groups)])
    bd = torch.from_numpy(b).cuda()
    solver = VankaMG([Grid(n, num_systems=c) for n, c in groups], lam)
    if not args.no_autotune:
        solver.autotune()
    Z, _, _, _ = solver.solve(bd, tol=args.tol)
    for _ in range(args.warmup):
        solver.solve(bd, tol=args.tol, out=Z)
    torch.cuda.synchronize()
    w0 = time.monotonic_ns()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, iters, relres, status = solver.solve(bd, tol=args.tol, out=Z)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    w1 = time.monotonic_ns()
    out = {"value": round(S / dt, 1), "unit": "systems/s", "ms_per_step": round(1e3 * dt, 3),
           "workload": "256x127^2 + 96x255^2 + 32x511^2, uniform shifts, V(2,2) to 1e-10, one batched solve",
           "iterations": {"min": int(iters.min()), "max": int(iters.max())}, "max_relres": float(relres.max()),
           "converged": bool(status == 0 and np.all(relres <= args.tol)),
           "timed_window_monotonic_ns": [w0, w1]}
    del solver
    # the 32 x 511^2 group on its own (its finest level, 267 MB a vector,
    # is the batch's only one well above the 256 MB cache): GB/s of its
    # finest-level kernels by algorithmic bytes, every kernel class timed
    g511 = VankaMG([Grid(511, num_systems=32)], lam[-32:])
    if not args.no_autotune:
        g511.autotune()
    b511 = bd[-32 * 511 * 511:].contiguous()
    Z511, _, _, _ = g511.solve(b511, tol=args.tol)
    g511.set_timing(True, reset=True)
    for _ in range(max(1, min(args.steps, 3))):
        g511.solve(b511, tol=args.tol, out=Z511)
    g511.set_timing(False, reset=False)
    fine = {}
    for k in ("down", "up", "edge"):
        for lvl, la, ms, by in g511.level_stats(k):
            if lvl == 0 and la > 0 and ms > 0:
                fine[k] = {"launches": la, "avg_ms": round(ms / la, 4), "GB/s": round(by / (ms * 1e-3) / 1e9, 1),
                           "hbm_frac": round(by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    out["group_511_alone"] = {"finest_level_kernels": fine, "plan": list(g511.plan(0))}
    del g511, Z511, b511
    # the same batch with the complex64 coarse-grid correction
    mx = VankaMG([Grid(n, num_systems=c) for n, c in groups], lam, precision="c128_c64")
    if not args.no_autotune:
        mx.autotune()
    mx.solve(bd, tol=args.tol, out=Z)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, it_m, rr_m, st_m = mx.solve(bd, tol=args.tol, out=Z)
    torch.cuda.synchronize()
    dtm = (time.perf_counter() - t0) / args.steps
    out["c64_coarse"] = {"value": round(S / dtm, 1), "ms_per_step": round(1e3 * dtm, 3),
                         "iterations": {"min": int(it_m.min()), "max": int(it_m.max())},
                         "max_relres": float(rr_m.max()), "converged": bool(st_m == 0 and np.all(rr_m <= args.tol)),
                         "speedup_vs_fp64": round(dt / dtm, 3)}
    return out


def paper_protocol_leg(args, torch):
    """The paper's Sec. 3 protocol on Example 1 (eq. (9) shifts, n = 256,
    h = tau = 1/256): W(1,0) cycles from h0 = 1/8 to a 1e-8 reduction, the
    additive Vanka smoother (omega = 24/25) against damped Jacobi (4/5)."""
    from paper_2203_11154_amd import Grid, VankaMG, inputs
    n, nt = 255, 256
    lam = inputs.example1_shifts(nt)
    bd = torch.from_numpy(inputs.rhs(nt, n, n).ravel()).cuda()
    out = {"workload": "Example 1: 256 BVM shifts on 255^2, W(1,0), tol 1e-8"}
    for name, kw in (("vanka", dict(omega=0.96)), ("jacobi", dict(omega=0.8, smoother="jacobi", max_iter=200))):
        s = VankaMG([Grid(n, num_systems=nt)], lam, nu1=1, nu2=0, gamma=2, **kw)
        s.solve(bd, tol=1e-8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, it, rr, st = s.solve(bd, tol=1e-8)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        out[name] = {"cycles": int(np.max(it)), "rate": round(float(np.median(rr ** (1.0 / it))), 4),
                     "ms_per_solve": round(1e3 * dt, 3), "systems_per_s": round(nt / dt, 1)}
        del s
    out["vanka_speedup_over_jacobi"] = round(out["jacobi"]["ms_per_solve"] / out["vanka"]["ms_per_solve"], 3)
    # Example 3 (Helmholtz shifts, h = 1/128, j = 8, 16, ..., 128): the real
    # 24/25 against the library's LFA-optimal complex weights (per shift, and
    # per shift and level)
    n3 = 127
    j = np.arange(8, 129, 8)
    lam3 = inputs.example3_shifts(128)[j - 1]
    b3 = torch.from_numpy(inputs.rhs(len(j), n3, n3, seed=9).ravel()).cuda()
    s = VankaMG([Grid(n3, num_systems=len(j))], lam3, nu1=1, nu2=0, gamma=2)
    ex3 = {"workload": "Example 3: 16 Helmholtz shifts (j = 8..128) on 127^2, W(1,0), tol 1e-8"}
    for name, per_level in (("real_24_25", None), ("complex_per_shift", False), ("complex_per_level", True)):
        if per_level is not None:
            s.optimize_omega(per_level=per_level)
        s.solve(b3, tol=1e-8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, it, rr, st = s.solve(b3, tol=1e-8)
        torch.cuda.synchronize()
        ex3[name] = {"cycles": it.tolist(), "ms_per_solve": round(1e3 * (time.perf_counter() - t0), 3),
                     "converged": st == 0 and bool(np.all(rr <= 1e-8))}
    del s
    out["example3_complex_omega"] = ex3
    return out


def heat_leg(args, torch):
    """Differentiation workload: backward-Euler heat all-at-once system on
    511^2 with n = 128 steps, alpha-circulant ParaDIAG preconditioner
    (alpha = 0.01), source sum_k theta_k sin(k pi x) sin(k pi y) e^{-t} with 16
    parameters.  Times the forward solve by the stationary iteration and by
    flexible GMRES, and one loss gradient (forward + adjoint solve)."""
    from paper_2203_11154_amd import inputs
    from paper_2203_11154_amd.autograd import HeatProblem, HeatSolve
    nx, n, K = 511, 128, 16
    tau = 1.0 / n
    lam = inputs.alpha_circulant_shifts(n, 0.01)
    V, Vinv = inputs.alpha_circulant_vectors(n, 0.01)
    prob = HeatProblem(nx, n, tau, lam, V, Vinv, tol=args.tol, inner_tol=1e-11)
    xs = np.arange(1, nx + 1) / (nx + 1)
    basis = torch.from_numpy(np.stack([np.outer(np.sin(k * np.pi * xs), np.sin(k * np.pi * xs))
                                       for k in range(1, K + 1)])).cuda()
    tdecay = torch.from_numpy(np.exp(-tau * np.arange(1, n + 1))).cuda()

    def source(theta):
        return (tdecay[:, None, None] * torch.tensordot(theta, basis, dims=1)[None]).to(torch.complex128).reshape(-1)

    theta = torch.from_numpy(inputs.heat_parameters(K)).cuda()
    theta_star = torch.from_numpy(inputs.heat_parameters(K, seed=inputs.SEED_THETA_STAR)).cuda()
    f = source(theta)
    out = {"workload": "heat 511^2 x 128 steps, alpha-circulant ParaDIAG preconditioner, 16 source parameters"}
    for name, run in (("stationary", lambda: prob.solve(f)), ("fgmres", lambda: prob.solve_gmres(f))):
        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            run()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        out[name] = {"ms_per_solve": round(1e3 * dt, 3), "preconditioned_steps": prob.last["outer"],
                     "relres": prob.last["relres"]}
    ustar = HeatSolve.apply(source(theta_star), prob).real.detach()

    def gradient():
        th = theta.clone().requires_grad_(True)
        loss = ((HeatSolve.apply(source(th), prob).real - ustar) ** 2).sum()
        loss.backward()
        return th.grad

    gradient()  # first adjoint solves capture their cycle graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        grad = gradient()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    out["gradient"] = {"ms_forward_adjoint": round(1e3 * dt, 3), "adjoint_relres": prob.last["relres"],
                       "grad_norm": float(grad.norm())}
    # central differences (step 1e-6) with the iteration counts of the last
    # forward solve frozen (the solve is then one fixed linear map of f and
    # the quadratic loss has no truncation error) against the adjoint gradient
    g = grad.cpu().numpy()
    th0 = theta.clone()
    fd_err = {}
    for k in (0, 5, 15):
        e = torch.zeros(K, dtype=torch.float64, device="cuda")
        e[k] = 1e-6
        lp = float(((HeatSolve.apply(source(th0 + e), prob, True).real - ustar) ** 2).sum())
        lm = float(((HeatSolve.apply(source(th0 - e), prob, True).real - ustar) ** 2).sum())
        fd = (lp - lm) / 2e-6
        fd_err[f"theta_{k}"] = {"adjoint": float(g[k]), "fd": fd, "rel_diff": abs(fd - g[k]) / abs(g[k])}
    out["gradient"]["fd_check"] = fd_err
    del prob
    # the stationary solve with the shifted solves' coarse-grid corrections in
    # complex64 (same tolerances)
    pm = HeatProblem(nx, n, tau, lam, V, Vinv, tol=args.tol, inner_tol=1e-11, precision="c128_c64")
    pm.solve(f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pm.solve(f)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    out["stationary_c64_coarse"] = {"ms_per_solve": round(1e3 * dt, 3), "preconditioned_steps": pm.last["outer"],
                                    "relres": pm.last["relres"],
                                    "speedup_vs_fp64": round(out["stationary"]["ms_per_solve"] / (1e3 * dt), 3)}
    return out


def copy_rate(torch):
    """The same GPU's device-to-device copy rate (2 GiB read, 2 GiB written)."""
    src = torch.empty(1 << 28, dtype=torch.float64, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 5 * 2 * src.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def roofline_of(leg, traffic_key, copy_gbs):
    """Roofline object of the dominant kernel (the FP64 cycle-edge kernel) from
    the HIP events of the leg's timed steps."""
    e = leg["fp64"]["edge_kernel"]
    gbs = e["GB/s"]
    traffic = None
    if MEASURED_TRAFFIC["source_sha256_16"] == kernel_source_hash(MEASURED_TRAFFIC["source"]):
        traffic = MEASURED_TRAFFIC["bytes_per_launch"].get(traffic_key, {}).get(leg["fp64"]["edge_plan"])
    n, S = leg["grid"], leg["systems"]
    r = {"bound": "hbm", "kernel": dominant_kernel(leg["fp64"]["edge_plan"]), "achieved": gbs, "peak": HBM_PEAK_GBS,
         "unit": "GB/s",
         "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "launches": e["launches"], "avg_ms": e["avg_ms"],
         "algorithmic_bytes_per_launch": e["algorithmic_bytes_per_launch"],
         "bytes_per_node": f"56 (read x, b, e/4; write x_(k+1) pre-smoothed, coarse rhs/4) x {n}^2 x {S}",
         "context": {"copy_GB/s": round(copy_gbs, 1)}}
    if traffic:
        tr = traffic / (e["avg_ms"] * 1e-3) / 1e9
        r["context"].update({"traffic_GB/s": round(tr, 1), "traffic_frac_of_copy": round(tr / copy_gbs, 3),
                             "traffic_over_algorithmic": round(traffic / e["algorithmic_bytes_per_launch"], 4)})
    return r


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only (the library has no multi-GPU path); --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import torch

    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    legs = {"headline", "plain", "small", "batched", "paper", "heat"} if args.legs == "all" else \
        set(x.strip() for x in args.legs.split(","))
    out = {"metric": METRIC}
    copy_gbs = copy_rate(torch)
    sample = ORACLE_SAMPLE[:max(0, args.cpu_sample)] if not args.no_cpu_baseline else ()
    if "headline" in legs:
        head, solutions, (b, lam, h) = paradiag_leg("precision_2047", 2047, 32, 4, args, torch, sample=sample)
        f64 = head["fp64"]
        if not f64["converged"]:
            raise SystemExit(f"FP64 ParaDIAG step did not converge: max relres {f64['max_relres']:.3e}")
        out.update({"value": f64["value"], "unit": "systems/s", "n_gpus": 1, "steps": args.steps,
                    "warmup": args.warmup, "ms_per_step": f64["ms_per_step"], "higher_is_better": True,
                    "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
                    "config": {"workload": head["workload"], "grid": 2047, "systems": 32, "cycle": "V(2,2)",
                               "levels": f64["levels"], "omega": 0.96, "precision": "FP64",
                               "schedule": f64["schedule"]},
                    "iterations": f64["cycles"], "max_relres": f64["max_relres"],
                    "roofline": roofline_of(head, "precision_2047", copy_gbs),
                    "fp32_ir": head["fp32_ir"], "fp32_coarse": head["fp32_coarse"],
                    "fp64_detail": {k: v for k, v in f64.items() if k not in ("value", "ms_per_step")},
                    "kernels_note": "kernels and fused_by_level: a separate pass with every kernel class timed by "
                                    "HIP events; the timed steps time the dominant kernel only"})
    if "plain" in legs:
        plain, _, _ = paradiag_leg("plain_1023", 1023, 64, 0, args, torch)
        plain["roofline"] = roofline_of(plain, "plain_1023", copy_gbs)
        out["plain_1023"] = plain
    if "small" in legs:
        out["plain_63"] = small_leg(args, torch)
        progress("plain_63 done")
    if "batched" in legs:
        out["batched_uneven"] = batched_leg(args, torch)
        progress("batched_uneven done")
    if "paper" in legs:
        out["paper_protocol"] = paper_protocol_leg(args, torch)
        progress("paper_protocol done")
    if "heat" in legs:
        out["heat"] = heat_leg(args, torch)
        progress("heat done")
    if "headline" in legs and len(sample):
        out["cpu_baseline"] = cpu_baseline(b, lam, h, args.tol, sample, solutions)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
