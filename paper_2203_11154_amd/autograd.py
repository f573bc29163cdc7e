"""Differentiable shifted solves and ParaDIAG steps (torch.autograd).

The backward pass of z = L_j^{-1} b_j (eq. (2)) is the adjoint solve with the
conjugate shifts, grad_b = (A + conj(lambda_j) I)^{-1} grad_z, reusing the
same kernels, and grad_lambda_j = -sum conj(z_j) grad_b_j (PyTorch's
conjugate-Wirtinger convention for complex tensors).  Every step runs in the
HIP library; this module only wires the calls into autograd.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from .solver import Grid, VankaMG, _ptr, _stream


class ShiftedSolve(torch.autograd.Function):
    """z = ShiftedSolve.apply(b, lam, solver, tol): all systems of `solver`.

    b: complex128 CUDA tensor holding every system (solver layout).
    lam: complex128 tensor of the shifts, one per system; it carries the
    gradient with respect to them.  When it differs from the solver's current
    shifts the solver takes it in place (vanka_mg_set_shifts) before solving.
    """

    @staticmethod
    def forward(ctx, b, lam, solver, tol=1e-10):
        lam_h = lam.detach().cpu().numpy().astype(np.complex128).ravel()
        if not np.array_equal(lam_h, solver.shifts):
            solver.set_shifts(lam_h)
        z, _, _, status = solver.solve(b.detach().contiguous().reshape(-1), tol)
        ctx.solver, ctx.tol, ctx.shape = solver, tol, b.shape
        ctx.save_for_backward(z)
        return z.reshape(b.shape)

    @staticmethod
    def backward(ctx, grad_z):
        (z,) = ctx.saved_tensors
        solver = ctx.solver
        gb, _, _, _ = solver.solve(grad_z.contiguous().reshape(-1), ctx.tol, conj=True)
        grad_lam = solver.shift_gradient(z, gb) if ctx.needs_input_grad[1] else None
        return gb.reshape(ctx.shape), grad_lam, None, None


class ParaDiag(torch.autograd.Function):
    """U = ParaDiag.apply(F, solver, V, Vinv, tol): eq. (1),
    U = (V kron I) blockdiag(L_j^{-1}) (V^{-1} kron I) F; backward applies the
    adjoint (V^{-H} kron I) blockdiag(L_j^{-H}) (V^H kron I)."""

    @staticmethod
    def forward(ctx, F, solver, V, Vinv, tol=1e-10):
        U, _ = solver.paradiag_apply(V, Vinv, F.detach().contiguous().reshape(-1), tol)
        ctx.solver, ctx.V, ctx.Vinv, ctx.tol, ctx.shape = solver, V, Vinv, tol, F.shape
        return U.reshape(F.shape)

    @staticmethod
    def backward(ctx, grad_U):
        gF, _ = ctx.solver.paradiag_apply(ctx.V, ctx.Vinv, grad_U.contiguous().reshape(-1), ctx.tol, conj=True)
        return gF.reshape(ctx.shape), None, None, None, None


class HeatProblem:
    """Backward-Euler all-at-once heat system K u = f on an nx x nx unit-square
    grid with n time steps of size tau, solved by the ParaDIAG-II iteration with
    the alpha-circulant preconditioner whose eigen-decomposition (lam, V, Vinv)
    is supplied by the caller (complex128 numpy arrays)."""

    def __init__(self, nx, n, tau, lam, V, Vinv, tol=1e-10, inner_tol=1e-12, max_outer=50, **solver_opts):
        self.nx, self.n, self.tau = nx, n, tau
        self.tol, self.inner_tol, self.max_outer = tol, inner_tol, max_outer
        self.solver = VankaMG([Grid(nx, num_systems=n)], lam, **solver_opts)
        dev = torch.device("cuda", torch.cuda.current_device())
        self.V = torch.from_numpy(np.ascontiguousarray(V, dtype=np.complex128)).to(dev)
        self.Vinv = torch.from_numpy(np.ascontiguousarray(Vinv, dtype=np.complex128)).to(dev)
        self.last = {}

    def solve(self, f, transpose=False, replay=False):
        """u with K u = f (K^T u = f with transpose); f complex128 CUDA, n*nx*nx."""
        self.solver._check_vec(f, self.solver.total, "f")
        u = torch.empty_like(f)
        outer = ctypes.c_int32(0)
        rel = ctypes.c_double(0.0)
        code = self.solver.lib.paradiag_heat_solve(
            self.solver.handle, _ptr(self.V), _ptr(self.Vinv), float(self.tau), _ptr(f), _ptr(u), float(self.tol),
            float(self.inner_tol), int(bool(transpose)), int(bool(replay)), int(self.max_outer),
            ctypes.byref(outer), ctypes.byref(rel), _stream())
        status = _lib.check(code, "paradiag_heat_solve")
        self.last = {"outer": outer.value, "relres": rel.value, "status": status}
        return u

    def solve_gmres(self, f, transpose=False, restart=10, max_iter=100):
        """u with K u = f (K^T u = f with transpose) by flexible GMRES,
        right-preconditioned by the same ParaDIAG step."""
        self.solver._check_vec(f, self.solver.total, "f")
        u = torch.empty_like(f)
        its = ctypes.c_int32(0)
        rel = ctypes.c_double(0.0)
        code = self.solver.lib.paradiag_heat_gmres(
            self.solver.handle, _ptr(self.V), _ptr(self.Vinv), float(self.tau), _ptr(f), _ptr(u), float(self.tol),
            float(self.inner_tol), int(bool(transpose)), int(restart), int(max_iter), ctypes.byref(its),
            ctypes.byref(rel), _stream())
        status = _lib.check(code, "paradiag_heat_gmres")
        self.last = {"outer": its.value, "relres": rel.value, "status": status}
        return u

    def residual(self, u, f, transpose=False):
        _, nrm = self.solver.heat_residual(self.tau, u, f, transpose=transpose)
        return nrm


class HeatSolve(torch.autograd.Function):
    """u = HeatSolve.apply(f, problem, replay): the ParaDIAG-II heat solve with
    its adjoint (the transposed iteration) as the backward pass."""

    @staticmethod
    def forward(ctx, f, problem, replay=False):
        ctx.problem, ctx.replay, ctx.shape = problem, replay, f.shape
        return problem.solve(f.detach().contiguous().reshape(-1), replay=replay).reshape(f.shape)

    @staticmethod
    def backward(ctx, grad_u):
        g = ctx.problem.solve(grad_u.contiguous().reshape(-1), transpose=True, replay=ctx.replay)
        return g.reshape(ctx.shape), None, None
