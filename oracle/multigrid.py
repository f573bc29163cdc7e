"""Geometric multigrid for the shifted systems of eq. (2), FP64 (test
infrastructure only).

Components as Sec. 3 lists them: re-discretised coarse operators with 2h,
full-weighting restriction, linear interpolation, the additive Vanka smoother
with omega = 24/25 (Sec. 2.1, after Theorem 2.1), a direct solve on the
coarsest grid, and a stopping test on the reduction of the relative residual
norm.  The cycle type (gamma = 1: V, gamma = 2: W) and the numbers of pre- and
post-smoothing steps are parameters; Sec. 3 uses W(1,0), the benchmark
workloads V(2,2).
"""
import numpy as np

from . import operators as ops
from . import exact

OMEGA_VANKA = 24.0 / 25.0     # Sec. 2.1, after Theorem 2.1; Table 1
OMEGA_JACOBI = 4.0 / 5.0      # Sec. 3; Table 1


def coarse_direct_solve(b, lam, h):
    """Coarsest grid: "solved" directly (Sec. 3), here by dense LU of the
    assembled A_H + lambda_j I."""
    return exact.dense_solve(b, lam, h)


def mg_cycle(level, x, b, lam, shapes, omega=OMEGA_VANKA, nu1=2, nu2=2, gamma=1,
             smoother="vanka"):
    """One multigrid cycle MG(level, x, b) for all systems at once.

    1. nu1 smoothing steps;
    2. restrict the residual with full weighting;
    3. start the coarse correction at zero and apply gamma cycles of the
       coarse problem (coarse operator A_{2h} + lambda_j I) to it;
    4. interpolate the correction and add it;
    5. nu2 smoothing steps.
    On the coarsest level the system is solved directly.
    """
    nx, ny, h = shapes[level]
    if level == len(shapes) - 1:
        return coarse_direct_solve(b, lam, h)
    sweep = ops.vanka_sweep if smoother == "vanka" else ops.jacobi_sweep
    for _ in range(nu1):
        x = sweep(x, b, lam, h, omega)
    r_coarse = ops.restrict_full_weighting(ops.residual(x, b, lam, h))
    e_coarse = np.zeros_like(r_coarse)
    for _ in range(gamma):
        e_coarse = mg_cycle(level + 1, e_coarse, r_coarse, lam, shapes, omega, nu1, nu2, gamma, smoother)
    x = x + ops.prolong_bilinear(e_coarse)
    for _ in range(nu2):
        x = sweep(x, b, lam, h, omega)
    return x


def residual_norms(x, b, lam, h):
    """Unweighted 2-norm of b_j - L_j x_j per system."""
    r = ops.residual(x, b, lam, h)
    return np.sqrt(np.sum(np.abs(r) ** 2, axis=(-2, -1)))


def solve(b, lam, h, tol=1e-10, max_iter=100, levels=0, omega=OMEGA_VANKA, nu1=2, nu2=2,
          gamma=1, smoother="vanka", fixed_iters=None, x0=None):
    """Multigrid iteration for every system of eq. (2) from x = 0 (or x0).

    After each complete cycle the relative residual ||b_j - L_j x_j|| / ||b_j||
    is measured; system j stops at the first cycle where it is <= tol, or after
    max_iter cycles.  With ``fixed_iters`` (one count per system) system j runs
    exactly that many cycles instead.  A system with b_j = 0 returns x = 0
    after zero cycles.

    Returns (x, iters, relres, history) where history[j] lists the relative
    residual after each of system j's cycles.
    """
    b = np.asarray(b, dtype=np.complex128)
    lam = np.asarray(lam, dtype=np.complex128)
    S, ny, nx = b.shape
    shapes = ops.level_shapes(nx, ny, h, levels)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    bnorm = np.sqrt(np.sum(np.abs(b) ** 2, axis=(-2, -1)))
    iters = np.zeros(S, dtype=np.int64)
    relres = np.where(bnorm > 0, residual_norms(x, b, lam, h) / np.where(bnorm > 0, bnorm, 1.0), 0.0)
    history = [[] for _ in range(S)]
    if fixed_iters is not None:
        target = np.asarray(fixed_iters, dtype=np.int64)
        active = target > 0
    else:
        target = np.full(S, max_iter, dtype=np.int64)
        active = (bnorm > 0) & (relres > tol)
    om = np.asarray(omega)
    while np.any(active):
        idx = np.nonzero(active)[0]
        om_idx = om[idx] if om.ndim == 1 else omega
        x[idx] = mg_cycle(0, x[idx], b[idx], lam[idx], shapes, om_idx, nu1, nu2, gamma, smoother)
        iters[idx] += 1
        rel = residual_norms(x[idx], b[idx], lam[idx], h) / np.where(bnorm[idx] > 0, bnorm[idx], 1.0)
        for t, j in enumerate(idx):
            relres[j] = rel[t]
            history[j].append(rel[t])
            if iters[j] >= target[j]:
                active[j] = False
            elif fixed_iters is None and rel[t] <= tol:
                active[j] = False
    return x, iters, relres, history


def observed_rate(history_j):
    """Geometric mean of the residual reduction per cycle."""
    h = np.asarray(history_j, dtype=np.float64)
    if len(h) == 0:
        return 0.0
    return float(h[-1] ** (1.0 / len(h)))


def two_grid_error_step(e, lam, h, omega=OMEGA_VANKA, nu1=1, nu2=0, smoother="vanka"):
    """Error propagation of one two-grid cycle with an exact coarse solve:
    e <- S^{nu2} (I - P L_H^{-1} R L_h) S^{nu1} e (b = 0)."""
    S, ny, nx = e.shape
    shapes = ops.level_shapes(nx, ny, h, levels=2)
    zero = np.zeros_like(e)
    return mg_cycle(0, e, zero, lam, shapes, omega, nu1, nu2, 1, smoother)
