"""Python face of the HIP library: torch tensors in, torch tensors out.

Only argument marshalling happens here; every step of the solve runs in the
library's kernels.  torch provides device memory and the current stream.
"""
import ctypes

import numpy as np
import torch

from . import _lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("the Vanka multigrid library needs a ROCm GPU (torch.cuda is unavailable)")


class Grid:
    """One grid and the number of shifted systems solved on it."""

    def __init__(self, nx, ny=None, h=None, num_systems=1, levels=0):
        self.nx = int(nx)
        self.ny = int(nx if ny is None else ny)
        self.h = float(1.0 / (self.nx + 1) if h is None else h)
        self.num_systems = int(num_systems)
        self.levels = int(levels)

    def to_c(self):
        return _lib.VmgGrid(self.nx, self.ny, self.h, self.levels, self.num_systems)


class VankaMG:
    """Setup, solve and ParaDIAG application for batches of shifted systems
    (A + lambda_j I) z_j = b_j on one or more grids.

    precision: "c128" (complex128 cycles), "c64_ir" (complex64 cycles inside
    FP64 iterative refinement) or "c128_c64" (FP64 V-cycles with the
    coarse-grid correction in complex64).  smoother: "vanka" or "jacobi".
    """

    def __init__(self, grids, shifts, omega=24.0 / 25.0, nu1=2, nu2=2, gamma=1, max_iter=100,
                 precision="c128", smoother="vanka", ir_inner=3, check_every=64, graphs=True):
        _require_gpu()
        self.lib = _lib.load()
        if isinstance(grids, Grid):
            grids = [grids]
        self.grids = list(grids)
        shifts = np.ascontiguousarray(np.asarray(shifts, dtype=np.complex128).ravel())
        self.num_systems = sum(g.num_systems for g in self.grids)
        if shifts.size != self.num_systems:
            raise ValueError(f"{shifts.size} shifts for {self.num_systems} systems")
        self.shifts = shifts
        self.device = torch.cuda.current_device()
        opts = _lib.VmgOpts()
        self.lib.vanka_mg_default_opts(ctypes.byref(opts))
        opts.omega = omega
        opts.nu1, opts.nu2, opts.gamma, opts.max_iter = nu1, nu2, gamma, max_iter
        opts.precision = {"c128": 0, "c64_ir": 1, "c128_c64": 2}[precision]
        opts.smoother = {"vanka": 0, "jacobi": 1}[smoother]
        opts.ir_inner, opts.check_every = ir_inner, check_every
        opts.graphs = int(bool(graphs))
        self.opts = opts
        self.precision = precision
        arr = (_lib.VmgGrid * len(self.grids))(*[g.to_c() for g in self.grids])
        handle = ctypes.c_void_p()
        sh = shifts.view(np.float64)
        code = self.lib.vanka_mg_setup(arr, len(self.grids), sh.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       ctypes.byref(opts), _stream(), ctypes.byref(handle))
        _lib.check(code, "vanka_mg_setup")
        self.handle = handle
        self.sizes = [g.nx * g.ny * g.num_systems for g in self.grids]
        self.total = sum(self.sizes)

    def close(self):
        if getattr(self, "handle", None):
            self.lib.vanka_mg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def levels(self, g=0):
        cnt = ctypes.c_int32()
        nx = (ctypes.c_int32 * 32)()
        ny = (ctypes.c_int32 * 32)()
        _lib.check(self.lib.vanka_mg_levels(self.handle, g, ctypes.byref(cnt), nx, ny), "vanka_mg_levels")
        return [(nx[i], ny[i]) for i in range(cnt.value)]

    def set_omega(self, omega=None):
        """Per-system complex relaxation weights (None: back to the scalar
        omega given at construction)."""
        if omega is None:
            _lib.check(self.lib.vanka_mg_set_omega(self.handle, None), "vanka_mg_set_omega")
            return
        om = np.ascontiguousarray(np.broadcast_to(np.asarray(omega, dtype=np.complex128), (self.num_systems,)))
        _lib.check(self.lib.vanka_mg_set_omega(self.handle, om.view(np.float64).ctypes.data_as(
            ctypes.POINTER(ctypes.c_double))), "vanka_mg_set_omega")

    def set_shifts(self, lam):
        """New shifts for the same grids, in place (coefficients and coarsest
        inverses recomputed into the handle's buffers; weights back to the
        constructor's omega)."""
        sh = np.ascontiguousarray(np.asarray(lam, dtype=np.complex128).ravel())
        if sh.size != self.num_systems:
            raise ValueError(f"{sh.size} shifts for {self.num_systems} systems")
        _lib.check(self.lib.vanka_mg_set_shifts(self.handle, sh.view(np.float64).ctypes.data_as(
            ctypes.POINTER(ctypes.c_double))), "vanka_mg_set_shifts")
        self.shifts = sh

    def optimize_omega(self, per_level=False):
        """Per shift (per_level: and level), the complex omega minimising the
        LFA smoothing factor of the handle's smoother (vanka_mg_optimize_omega)."""
        _lib.check(self.lib.vanka_mg_optimize_omega(self.handle, int(bool(per_level))), "vanka_mg_optimize_omega")

    def autotune(self, cache_path=None):
        """Time the kernel schedules of every level and keep the fastest;
        returns the schedule per grid (see schedule())."""
        path = None if cache_path is None else str(cache_path).encode()
        _lib.check(self.lib.vanka_mg_autotune(self.handle, path, _stream()), "vanka_mg_autotune")
        return [self.schedule(g) for g in range(len(self.grids))]

    def schedule(self, g=0):
        """Per level: 0 = LDS-tiled kernels, r > 0 = streaming kernels with r
        rows per block, -1 = coarsest level."""
        n = len(self.levels(g))
        arr = (ctypes.c_int32 * n)()
        _lib.check(self.lib.vanka_mg_schedule(self.handle, g, n, arr), "vanka_mg_schedule")
        return list(arr)

    def _check_vec(self, t, n, name):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()):
            raise TypeError(f"{name} must be a contiguous complex128 CUDA tensor")
        if t.numel() != n:
            raise ValueError(f"{name} has {t.numel()} elements, expected {n}")

    def plan(self, g=0):
        """(edge, tail_level) of grid g: whether the finest level runs across
        the boundary of two V-cycles in one launch (0 no, 1 yes, 2 yes in
        paced blocks), and the first level run in one workgroup per system
        (-1: none)."""
        e, t = ctypes.c_int32(0), ctypes.c_int32(0)
        _lib.check(self.lib.vanka_mg_plan(self.handle, g, ctypes.byref(e), ctypes.byref(t)), "vanka_mg_plan")
        return int(e.value), int(t.value)

    def solve(self, B, tol=1e-10, conj=False, fixed_iters=None, out=None, stats=True):
        """Solve every system; B holds all systems concatenated (any shape with
        the right number of elements).  Returns (Z, iters, relres, status).
        stats=False with fixed_iters: no host outputs, the call only enqueues
        work (iters and relres are None; see last_stats)."""
        self._check_vec(B, self.total, "B")
        Z = torch.empty_like(B) if out is None else out
        self._check_vec(Z, self.total, "out")
        iters = np.zeros(self.num_systems, dtype=np.int32) if stats else None
        relres = np.zeros(self.num_systems, dtype=np.float64) if stats else None
        fx = None
        if fixed_iters is not None:
            fa = np.ascontiguousarray(np.asarray(fixed_iters, dtype=np.int32).ravel())
            if fa.size != self.num_systems:
                raise ValueError("fixed_iters needs one count per system")
            fx = fa.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        code = self.lib.vanka_mg_solve(self.handle, _ptr(B), _ptr(Z), float(tol), int(bool(conj)), fx,
                                       iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if stats else None,
                                       relres.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if stats else None,
                                       _stream())
        if fixed_iters is not None:
            self._keep = fa
        status = _lib.check(code, "vanka_mg_solve")
        return Z, iters, relres, status

    def apply_op(self, op, level, b, x=None, conj=False, out_numel=None):
        """One solver operation (``_lib.OP_*``) on caller data at `level`."""
        out = torch.empty(out_numel if out_numel is not None else b.numel(), dtype=torch.complex128,
                          device=b.device)
        code = self.lib.vanka_mg_apply_op(self.handle, op, level, int(bool(conj)),
                                          _ptr(x) if x is not None else None, _ptr(b), _ptr(out), _stream())
        _lib.check(code, "vanka_mg_apply_op")
        return out

    def _fixed(self, fixed_iters):
        if fixed_iters is None:
            return None, None
        fa = np.ascontiguousarray(np.asarray(fixed_iters, dtype=np.int32).ravel())
        if fa.size != self.num_systems:
            raise ValueError("fixed_iters needs one count per system")
        return fa, fa.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))

    def paradiag_apply(self, V, Vinv, F, tol=1e-10, conj=False, out=None, fixed_iters=None):
        """U = (V kron I) blockdiag(L_j^{-1}) (Vinv kron I) F (eq. (1)); with
        conj the adjoint (V^{-H} kron I) blockdiag(L_j^{-H}) (V^H kron I) F."""
        n = self.num_systems
        for t, nm in ((V, "V"), (Vinv, "Vinv")):
            self._check_vec(t, n * n, nm)
        self._check_vec(F, self.total, "F")
        U = torch.empty_like(F) if out is None else out
        keep, fx = self._fixed(fixed_iters)
        code = self.lib.paradiag_apply(self.handle, _ptr(V), _ptr(Vinv), _ptr(F), _ptr(U), float(tol),
                                       int(bool(conj)), fx, _stream())
        del keep
        status = _lib.check(code, "paradiag_apply")
        return U, status

    def paradiag_apply_circulant(self, alpha, F, tol=1e-10, conj=False, out=None, fixed_iters=None):
        """The same step for the alpha-circulant eigenvector matrix V, whose
        transforms are scaled DFTs along the time index (the handle's shifts
        must be the matching eigenvalues, see inputs.alpha_circulant_shifts)."""
        self._check_vec(F, self.total, "F")
        U = torch.empty_like(F) if out is None else out
        keep, fx = self._fixed(fixed_iters)
        code = self.lib.paradiag_apply_circulant(self.handle, float(alpha), _ptr(F), _ptr(U), float(tol),
                                                 int(bool(conj)), fx, _stream())
        del keep
        status = _lib.check(code, "paradiag_apply_circulant")
        return U, status

    def shift_gradient(self, Z, G):
        """grad_lambda[j] = -sum conj(Z_j) G_j (one complex value per system)."""
        self._check_vec(Z, self.total, "Z")
        self._check_vec(G, self.total, "G")
        out = torch.empty(self.num_systems, dtype=torch.complex128, device=Z.device)
        _lib.check(self.lib.vanka_mg_shift_gradient(self.handle, _ptr(Z), _ptr(G), _ptr(out), _stream()),
                   "vanka_mg_shift_gradient")
        return out

    def heat_residual(self, tau, U, F, out=None, transpose=False, norm=True):
        """R = F - K U for the backward-Euler all-at-once operator K (K^T with
        transpose), or R = K U when F is None; returns (R, ||R||^2 or None)."""
        self._check_vec(U, self.total, "U")
        if F is not None:
            self._check_vec(F, self.total, "F")
        R = torch.empty_like(U) if out is None else out
        nrm = ctypes.c_double(0.0)
        code = self.lib.paradiag_heat_residual(self.handle, float(tau), _ptr(U), None if F is None else _ptr(F), _ptr(R),
                                               int(bool(transpose)), ctypes.byref(nrm) if norm else None, _stream())
        _lib.check(code, "paradiag_heat_residual")
        return R, (nrm.value if norm else None)

    def last_stats(self):
        """(iters, relres) per system of the last solve or ParaDIAG step."""
        iters = np.zeros(self.num_systems, dtype=np.int32)
        relres = np.zeros(self.num_systems, dtype=np.float64)
        _lib.check(self.lib.vanka_mg_last_stats(self.handle, iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                                relres.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream()),
                   "vanka_mg_last_stats")
        return iters, relres

    def set_timing(self, enable=True, reset=True, classes=None):
        """Per-kernel HIP-event timing on (eager launches) or off; classes: the
        kernel classes (names of _lib.KERNEL_CLASSES) to time, None = all."""
        mask = 0 if classes is None else sum(1 << _lib.KERNEL_CLASSES.index(c) for c in classes)
        _lib.check(self.lib.vanka_mg_set_timing_mask(self.handle, mask), "vanka_mg_set_timing_mask")
        _lib.check(self.lib.vanka_mg_set_timing(self.handle, int(enable), int(reset)), "vanka_mg_set_timing")

    def level_stats(self, kclass):
        """[(level, launches, total_ms, total_algorithmic_bytes)] for every level
        on which one class of kernel ran."""
        k = _lib.KERNEL_CLASSES.index(kclass)
        n = 32
        la = (ctypes.c_int64 * n)()
        ms = (ctypes.c_double * n)()
        by = (ctypes.c_double * n)()
        _lib.check(self.lib.vanka_mg_level_stats(self.handle, k, n, la, ms, by), "vanka_mg_level_stats")
        return [(i, la[i], ms[i], by[i]) for i in range(n) if la[i] > 0]

    def kernel_stats(self):
        """{class: (launches, total_ms, total_algorithmic_bytes)}"""
        n = _lib.NUM_KCLASS
        la = (ctypes.c_int64 * n)()
        ms = (ctypes.c_double * n)()
        by = (ctypes.c_double * n)()
        _lib.check(self.lib.vanka_mg_kernel_stats(self.handle, la, ms, by), "vanka_mg_kernel_stats")
        return {k: (la[i], ms[i], by[i]) for i, k in enumerate(_lib.KERNEL_CLASSES)}


def lfa_omega(eta, smoother="vanka"):
    """(omega, mu): for each eta = lambda h^2 the complex relaxation weight
    minimising the LFA smoothing factor, and that factor (host computation,
    vanka_mg_lfa_omega)."""
    lib = _lib.load()
    e = np.ascontiguousarray(np.atleast_1d(np.asarray(eta, dtype=np.complex128)))
    om = np.empty_like(e)
    mu = np.empty(e.shape, dtype=np.float64)
    pd = ctypes.POINTER(ctypes.c_double)
    _lib.check(lib.vanka_mg_lfa_omega(e.view(np.float64).ctypes.data_as(pd), e.size,
                                      {"vanka": 0, "jacobi": 1}[smoother],
                                      om.view(np.float64).ctypes.data_as(pd), mu.ctypes.data_as(pd)),
               "vanka_mg_lfa_omega")
    return om, mu


def transform_circulant(n, alpha, F, inverse=False, conj=False, out=None):
    """out = (V^{-1} kron I) F (inverse: V kron I; conj: V^H, V^{-H}) for the
    alpha-circulant eigenvector matrix V of n time steps, by scaled DFTs."""
    _require_gpu()
    lib = _lib.load()
    m = F.numel() // n
    if not (F.is_cuda and F.dtype == torch.complex128 and F.is_contiguous()) or F.numel() != n * m:
        raise TypeError("transform_circulant needs a contiguous complex128 CUDA tensor of n x m values")
    out = torch.empty_like(F) if out is None else out
    code = lib.paradiag_transform_circulant(int(n), int(m), float(alpha), int(bool(inverse)), int(bool(conj)),
                                            _ptr(F), _ptr(out), _stream())
    _lib.check(code, "paradiag_transform_circulant")
    return out


def transform(M, F, trans_conj=False, out=None):
    """out = (M kron I) F for complex128 CUDA tensors M (n x n) and F (n x m)."""
    _require_gpu()
    lib = _lib.load()
    n = M.shape[0]
    m = F.numel() // n
    for t in (M, F):
        if not (t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()):
            raise TypeError("transform needs contiguous complex128 CUDA tensors")
    out = torch.empty_like(F) if out is None else out
    code = lib.paradiag_transform(n, m, _ptr(M), int(bool(trans_conj)), _ptr(F), _ptr(out), _stream())
    _lib.check(code, "paradiag_transform")
    return out

def transform_noalloc(M, F, trans_conj=False, out=None):
    """transform() through the entry point that allocates no device memory
    (the expanded matrix lives in the library's fixed per-GPU array; n <= 256;
    calls that overlap on one GPU race).  `out` must be given by callers that
    cannot allocate."""
    _require_gpu()
    lib = _lib.load()
    n = M.shape[0]
    m = F.numel() // n
    for t in (M, F):
        if not (t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()):
            raise TypeError("transform_noalloc needs contiguous complex128 CUDA tensors")
    out = torch.empty_like(F) if out is None else out
    code = lib.paradiag_transform_noalloc(n, m, _ptr(M), int(bool(trans_conj)), _ptr(F), _ptr(out), _stream())
    _lib.check(code, "paradiag_transform_noalloc")
    return out
