"""Benchmark of the ParaDIAG hot path on one MI355X.

One step = one ParaDIAG application of eq. (1) to a batch of time slices:
G = (V^{-1} kron I) F on the FP64 matrix cores, the 64 shifted systems
(A + lambda_j I) z_j = g_j solved to 1e-10 relative residual by V(2,2) Vanka
multigrid, and U = (V kron I) Z.  The workload is the 1023 x 1023 unit-square
grid with the 64 alpha-circulant shifts (alpha = 0.01, tau = 1/64); F is
chosen as (V kron I) b with b_j ~ U(-1, 1) + i U(-1, 1), so the shifted
systems see exactly those right-hand sides.

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
# FETCH_SIZE and WRITE_SIZE on this workload, each scaled by its reading for a
# plain 1 GiB copy (profiles/).  Valid only for the kernel source it was
# measured on: reported as null once that file changes.
MEASURED_TRAFFIC = {"source": "vmg_stream.hip", "source_sha256_16": "55aa523806855e73", "bytes_per_launch": 4065.1e6}
# finest level across the boundary of two V-cycles: correction + 2 sweeps +
# stopping-test norm, then the next cycle's 2 sweeps + residual + restriction
DOMINANT = "k_edge<double, 2, 2, double>"


def kernel_source_hash(name):
    import hashlib
    path = os.path.join(ROOT, "paper_2203_11154_amd", "csrc", name)
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--n", type=int, default=1023, help="interior grid size")
    p.add_argument("--systems", type=int, default=64, help="time slices = shifted systems")
    p.add_argument("--tol", type=float, default=1e-10)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-ir", action="store_true")
    p.add_argument("--cpu-sample", type=int, default=8, help="systems the oracle solves for the CPU baseline")
    p.add_argument("--no-autotune", action="store_true", help="keep the size heuristic kernel schedule")
    p.add_argument("--no-batched", action="store_true", help="skip the uneven-grid batched leg")
    p.add_argument("--no-paper", action="store_true", help="skip the paper-protocol leg")
    p.add_argument("--no-heat", action="store_true", help="skip the heat (differentiation) leg")
    p.add_argument("--copy-calibration", action="store_true",
                   help="run one plain 1 GiB device copy first (reference for hardware byte counters)")
    return p.parse_args()


def cpu_baseline(b, lam, h, tol, count):
    """The FP64 oracle on a bounded sample of the same workload: `count` of
    the shifted systems solved to `tol` (transforms excluded), BLAS limited to
    one thread so the core count is exact."""
    from threadpoolctl import threadpool_limits
    from oracle import multigrid as omg
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        _, iters, relres, _ = omg.solve(b[:count], lam[:count], h, tol=tol)
        dt = time.perf_counter() - t0
    return {"value": count / dt, "unit": "systems/s", "cores": 1, "kind": "oracle",
            "sample": f"{count} of the {len(lam)} shifted systems at {b.shape[-1]}^2, V(2,2) to {tol:g} "
                      f"({int(iters.sum())} cycles, {dt:.1f} s; transforms excluded)"}


def precision_leg(args, torch):
    """The precision workload: 32 alpha-circulant shifts (alpha = 0.01,
    tau = 1/32) on 2047^2, the ParaDIAG step to 1e-10 with complex64 V-cycles
    inside FP64 refinement, and FP64 V-cycles with a complex64 coarse-grid
    correction, against FP64 V-cycles (all uninstrumented, cycles replayed as
    graphs, autotuned; refinement with 2 inner cycles a step)."""
    from paper_2203_11154_amd import Grid, VankaMG, inputs
    n, S, tol = 2047, 32, args.tol
    lam = inputs.alpha_circulant_shifts(S, 0.01)
    V, Vinv = inputs.alpha_circulant_vectors(S, 0.01)
    b = inputs.rhs(S, n, n, seed=4)
    Fd = torch.from_numpy(np.ascontiguousarray(V @ b.reshape(S, -1)).ravel()).cuda()
    del b
    Vd, Vinvd = torch.from_numpy(V).cuda(), torch.from_numpy(Vinv).cuda()
    Ud = torch.empty_like(Fd)
    res = {"workload": "precision_2047: 32 alpha-circulant shifts on 2047x2047, ParaDIAG step to 1e-10"}
    for name, kw in (("fp64", {}), ("fp32_ir", {"precision": "c64_ir", "ir_inner": 2}),
                     ("fp32_coarse", {"precision": "c128_c64"})):
        s = VankaMG([Grid(n, num_systems=S)], lam, **kw)
        if not args.no_autotune:
            s.autotune()
        for _ in range(args.warmup):
            s.paradiag_apply(Vd, Vinvd, Fd, tol=tol, out=Ud)
        dt, st = run_steps(s, Vd, Vinvd, Fd, Ud, args.steps, tol, torch)
        it, rr = s.last_stats()
        res[name] = {"ms_per_step": round(1e3 * dt / args.steps, 3), "value": round(S * args.steps / dt, 2),
                     "cycles_or_steps": {"min": int(it.min()), "max": int(it.max())}, "max_relres": float(rr.max()),
                     "converged": st == 0 and bool(np.all(rr <= tol))}
        del s
    res["speedup_vs_fp64"] = round(res["fp64"]["ms_per_step"] / res["fp32_ir"]["ms_per_step"], 3)
    res["fp32_coarse_speedup_vs_fp64"] = round(res["fp64"]["ms_per_step"] / res["fp32_coarse"]["ms_per_step"], 3)
    del Fd, Ud
    torch.cuda.empty_cache()
    return res


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
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, iters, relres, status = solver.solve(bd, tol=args.tol, out=Z)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    out = {"value": round(S / dt, 1), "unit": "systems/s", "ms_per_step": round(1e3 * dt, 3),
           "workload": "256x127^2 + 96x255^2 + 32x511^2, uniform shifts, V(2,2) to 1e-10, one batched solve",
           "iterations": {"min": int(iters.min()), "max": int(iters.max())}, "max_relres": float(relres.max()),
           "converged": bool(status == 0 and np.all(relres <= args.tol))}
    del solver
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


def run_steps(solver, V, Vinv, F, U, steps, tol, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    status = 0
    for _ in range(steps):
        _, status = solver.paradiag_apply(V, Vinv, F, tol=tol, out=U)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, status


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only (the library has no multi-GPU path); --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import torch
    from paper_2203_11154_amd import Grid, VankaMG, inputs

    n, S, tol = args.n, args.systems, args.tol
    h = 1.0 / (n + 1)
    lam = inputs.alpha_circulant_shifts(S, 0.01)
    V, Vinv = inputs.alpha_circulant_vectors(S, 0.01)
    b = inputs.rhs(S, n, n)
    F_host = (V @ b.reshape(S, -1)).reshape(S, n, n)
    dev = torch.device("cuda:0")
    Vd = torch.from_numpy(V).to(dev).contiguous()
    Vinvd = torch.from_numpy(Vinv).to(dev).contiguous()
    Fd = torch.from_numpy(np.ascontiguousarray(F_host).ravel()).to(dev)
    Ud = torch.empty_like(Fd)
    del F_host

    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    solver = VankaMG([Grid(n, num_systems=S)], lam)
    schedule = solver.autotune() if not args.no_autotune else [solver.schedule(0)]
    for _ in range(args.warmup):
        solver.paradiag_apply(Vd, Vinvd, Fd, tol=tol, out=Ud)
    # the timed steps record HIP events around the dominant kernel only (the
    # roofline's durations), leaving the rest of the step unperturbed
    solver.set_timing(True, reset=True, classes=["edge"])
    dt, status = run_steps(solver, Vd, Vinvd, Fd, Ud, args.steps, tol, torch)
    edge_levels = solver.level_stats("edge")
    solver.set_timing(False, reset=False)
    iters, relres = solver.last_stats()
    if status != 0 or not np.all(relres <= tol):
        raise SystemExit(f"FP64 ParaDIAG step did not converge: status {status}, max relres {relres.max():.3e}")
    ms_per_step = 1e3 * dt / args.steps
    value = S * args.steps / dt

    # dominant kernel: the finest-level cycle-edge kernel (HBM bound); it is
    # the only launch of its instantiation, so HIP-event and rocprofv3
    # averages cover the same launches
    _, la, ms, by = edge_levels[0]
    gbs = by / (ms * 1e-3) / 1e9
    traffic = None
    if MEASURED_TRAFFIC["source_sha256_16"] == kernel_source_hash(MEASURED_TRAFFIC["source"]):
        traffic = MEASURED_TRAFFIC["bytes_per_launch"]
    roofline = {"bound": "hbm", "kernel": DOMINANT, "achieved": round(gbs, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                "traffic": traffic, "launches": la, "avg_ms": round(ms / max(la, 1), 5),
                "algorithmic_bytes_per_launch": round(by / max(la, 1)),
                "bytes_per_node": "56 (read x, b, e/4; write x_(k+1) pre-smoothed, coarse rhs/4)"}
    # context: the same GPU's device-to-device copy rate (2 GiB read, 2 GiB
    # written), and the kernel's measured traffic against it
    src = torch.empty(1 << 28, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * src.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    roofline["context"] = {"copy_GB/s": round(copy_gbs, 1)}
    if traffic:
        tr_gbs = traffic / (ms / max(la, 1) * 1e-3) / 1e9
        roofline["context"].update({"traffic_GB/s": round(tr_gbs, 1),
                                    "traffic_frac_of_copy": round(tr_gbs / copy_gbs, 3)})
    # per-kernel breakdown: a separate pass with every kernel class timed
    # (untimed as a whole; its events perturb the step)
    solver.set_timing(True, reset=True)
    run_steps(solver, Vd, Vinvd, Fd, Ud, min(args.steps, 3), tol, torch)
    stats = solver.kernel_stats()
    solver.set_timing(False, reset=False)
    levels = {}
    for k in ("down", "up", "edge"):
        levels[k] = [{"level": l, "launches": a, "avg_ms": round(m / max(a, 1), 4),
                      "GB/s": round(b_ / (m * 1e-3) / 1e9, 1) if m > 0 else None}
                     for l, a, m, b_ in solver.level_stats(k)]
    tl, tms, tby = stats["transform"]
    flops = 8.0 * S * S * n * n * tl
    kernels = {k: {"launches": v[0], "ms": round(v[1], 3),
                   "GB/s": round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[1] > 0 else None,
                   "hbm_frac": round(v[2] / (v[1] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if v[1] > 0 else None}
               for k, v in stats.items() if v[0] > 0}
    kernels["transform"]["TFLOP/s"] = round(flops / (tms * 1e-3) / 1e12, 2) if tms > 0 else None
    kernels["transform"]["mfma_frac"] = round(flops / (tms * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFLOPS, 4) if tms else None

    out = {"metric": METRIC, "value": round(value, 2), "unit": "systems/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
           "config": {"workload": f"plain_{n}: {S} alpha-circulant shifts (alpha=0.01, tau=1/{S}) on the "
                                  f"{n}x{n} unit-square grid, ParaDIAG step (transform, V(2,2) Vanka multigrid "
                                  f"to {tol:g}, inverse transform)",
                      "grid": n, "systems": S, "cycle": "V(2,2)", "levels": len(solver.levels()),
                      "omega": 0.96, "precision": "FP64", "schedule": schedule[0]},
           "iterations": {"min": int(iters.min()), "max": int(iters.max())},
           "max_relres": float(relres.max()),
           "roofline": roofline, "kernels": kernels, "fused_by_level": levels,
           "kernels_note": "kernels and fused_by_level: a separate pass with every kernel class timed by HIP "
                           "events; the timed steps time the dominant kernel only"}
    # context: the same steps without per-kernel events (cycles replayed as
    # captured graphs), and with the alpha-circulant transforms done as scaled
    # DFTs (paradiag_apply_circulant) instead of the MFMA GEMMs
    dtg, _ = run_steps(solver, Vd, Vinvd, Fd, Ud, args.steps, tol, torch)
    for _ in range(args.warmup):
        solver.paradiag_apply_circulant(0.01, Fd, tol=tol, out=Ud)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, st_c = solver.paradiag_apply_circulant(0.01, Fd, tol=tol, out=Ud)
    torch.cuda.synchronize()
    dtc = time.perf_counter() - t0
    _, rr_c = solver.last_stats()
    out["uninstrumented"] = {"ms_per_step": round(1e3 * dtg / args.steps, 3),
                             "value": round(S * args.steps / dtg, 2),
                             "note": "same steps, cycles replayed as graphs, no per-kernel events"}
    out["circulant_dft_step"] = {"ms_per_step": round(1e3 * dtc / args.steps, 3),
                                 "value": round(S * args.steps / dtc, 2),
                                 "converged": st_c == 0 and bool(np.all(rr_c <= tol)),
                                 "note": "transforms as scaled length-64 DFTs, uninstrumented"}
    del solver
    torch.cuda.empty_cache()

    if not args.no_ir:
        ir = VankaMG([Grid(n, num_systems=S)], lam, precision="c64_ir")
        if not args.no_autotune:
            ir.autotune()
        for _ in range(args.warmup):
            ir.paradiag_apply(Vd, Vinvd, Fd, tol=tol, out=Ud)
        ir.set_timing(True, reset=True, classes=["edge"])
        dti, st_ir = run_steps(ir, Vd, Vinvd, Fd, Ud, args.steps, tol, torch)
        ir.set_timing(False, reset=False)
        it_ir, rr_ir = ir.last_stats()
        ok = st_ir == 0 and bool(np.all(rr_ir <= tol))
        out["fp32_ir"] = {"value": round(S * args.steps / dti, 2), "unit": "systems/s",
                          "ms_per_step": round(1e3 * dti / args.steps, 3),
                          "speedup_vs_fp64": round(ms_per_step / (1e3 * dti / args.steps), 3),
                          "refinement_steps": {"min": int(it_ir.min()), "max": int(it_ir.max())},
                          "max_relres": float(rr_ir.max()), "converged": ok, "dtype": "c64 cycles + c128 refinement"}
        del ir
        # FP64 V-cycles whose coarse-grid correction runs in complex64: the
        # finest level, the stopping test and the result in FP64
        mx = VankaMG([Grid(n, num_systems=S)], lam, precision="c128_c64")
        if not args.no_autotune:
            mx.autotune()
        for _ in range(args.warmup):
            mx.paradiag_apply(Vd, Vinvd, Fd, tol=tol, out=Ud)
        mx.set_timing(True, reset=True, classes=["edge"])
        dtm, st_m = run_steps(mx, Vd, Vinvd, Fd, Ud, args.steps, tol, torch)
        mx.set_timing(False, reset=False)
        it_m, rr_m = mx.last_stats()
        dtmg, _ = run_steps(mx, Vd, Vinvd, Fd, Ud, args.steps, tol, torch)
        out["fp32_coarse"] = {"value": round(S * args.steps / dtm, 2), "unit": "systems/s",
                              "ms_per_step": round(1e3 * dtm / args.steps, 3),
                              "speedup_vs_fp64": round(ms_per_step / (1e3 * dtm / args.steps), 3),
                              "uninstrumented_ms_per_step": round(1e3 * dtmg / args.steps, 3),
                              "uninstrumented_speedup_vs_fp64": round(dtg / dtmg, 3),
                              "cycles": {"min": int(it_m.min()), "max": int(it_m.max())},
                              "max_relres": float(rr_m.max()), "converged": st_m == 0 and bool(np.all(rr_m <= tol)),
                              "dtype": "c128 finest level and stopping test, c64 coarse-grid correction"}
        del mx

    if not args.no_ir:
        out["fp32_ir_2047"] = precision_leg(args, torch)

    if not args.no_batched:
        out["batched_uneven"] = batched_leg(args, torch)
    if not args.no_paper:
        out["paper_protocol"] = paper_protocol_leg(args, torch)
    if not args.no_heat:
        out["heat"] = heat_leg(args, torch)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(b, lam, h, tol, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
