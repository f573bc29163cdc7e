"""Grid operators of the shifted systems, FP64 (test infrastructure only).

Conventions
-----------
* A grid has ``nx`` x ``ny`` interior nodes with mesh width ``h``; node
  (i, k), i = 1..nx, k = 1..ny, sits at (i h, k h).  Values on the boundary
  ring are zero (homogeneous Dirichlet, Sec. 1 below eq. (2)).
* Arrays hold interior values only, shape ``(S, ny, nx)`` complex128 with x
  fastest; S is the number of systems (one per shift).
* ``lam`` is a length-S complex array of shifts lambda_j.

Reading of the paper at the Dirichlet boundary (the paper does not discuss
patches that touch it): every grid cell is one Vanka patch, cells touching the
boundary use the same 4x4 patch inverse, and only interior unknowns are
updated.  This is the same as applying the interior stencil of eq. (6) at every
interior node with the residual taken as zero off the interior.
"""
import numpy as np


def pad0(x):
    """Surround the last two axes with the zero Dirichlet ring."""
    width = [(0, 0)] * (x.ndim - 2) + [(1, 1), (1, 1)]
    return np.pad(x, width)


def apply_shifted_laplacian(x, lam, h):
    """L_j x = (A + lambda_j I) x for every system j.

    A is the 5-point finite-difference Laplacian (1/h^2)[., -1, .; -1, 4, -1;
    ., -1, .] (Sec. 1, below eq. (2)); the shifted operator is eq. (2).
    """
    lam = np.asarray(lam, dtype=np.complex128)
    xp = pad0(x)
    neighbours = (xp[..., :-2, 1:-1] + xp[..., 2:, 1:-1]
                  + xp[..., 1:-1, :-2] + xp[..., 1:-1, 2:])
    diag = 4.0 + lam[:, None, None] * (h * h)
    return (diag * x - neighbours) / (h * h)


def residual(x, b, lam, h):
    """r = b_j - L_j x_j (eq. (2))."""
    return b - apply_shifted_laplacian(x, lam, h)


def vanka_abc_paper(eta):
    """Coefficients a, b, c of the element-wise Vanka stencil, exactly as
    printed below eq. (6), with eta_j = lambda_j h^2."""
    eta = np.asarray(eta, dtype=np.complex128)
    a = 0.25 * (1.0 / (2.0 + eta) + 2.0 / (4.0 + eta) + 1.0 / (6.0 + eta))
    b = 0.25 * (1.0 / (2.0 + eta) - 1.0 / (6.0 + eta))
    c = 0.25 * (1.0 / (2.0 + eta) - 2.0 / (4.0 + eta) + 1.0 / (6.0 + eta))
    return a, b, c


def vanka_abc(eta):
    """The same a, b, c as ``vanka_abc_paper`` over one common denominator.

    Putting the three fractions of eq. (6) over d = (2+eta)(4+eta)(6+eta)
    gives a = (14 + 8 eta + eta^2)/d, b = 1/((2+eta)(6+eta)), c = 2/d.
    These forms avoid the cancellation of the printed sums when |eta| is
    large (the coarse levels of a strongly shifted system).
    """
    eta = np.asarray(eta, dtype=np.complex128)
    d = (2.0 + eta) * (4.0 + eta) * (6.0 + eta)
    a = (14.0 + 8.0 * eta + eta * eta) / d
    b = 1.0 / ((2.0 + eta) * (6.0 + eta))
    c = 2.0 / d
    return a, b, c


def vanka_smoother_apply(r, lam, h):
    """M_{e,j} r with the explicit stencil of eq. (6):

        M_{e,j} = (h^2/4) [c 2b c; 2b 4a 2b; c 2b c],

    one stencil per system, r taken as zero off the interior."""
    lam = np.asarray(lam, dtype=np.complex128)
    a, b, c = vanka_abc(lam * h * h)
    a = a[:, None, None]
    b = b[:, None, None]
    c = c[:, None, None]
    rp = pad0(r)
    edges = (rp[..., :-2, 1:-1] + rp[..., 2:, 1:-1]
             + rp[..., 1:-1, :-2] + rp[..., 1:-1, 2:])
    corners = (rp[..., :-2, :-2] + rp[..., :-2, 2:]
               + rp[..., 2:, :-2] + rp[..., 2:, 2:])
    return (h * h / 4.0) * (4.0 * a * r + 2.0 * b * edges + c * corners)


def _per_system(omega):
    """A relaxation weight as a scalar or one (possibly complex) value per
    system, shaped to broadcast against (S, ny, nx)."""
    om = np.asarray(omega)
    return om[:, None, None] if om.ndim == 1 else om


def vanka_sweep(x, b, lam, h, omega):
    """One additive Vanka relaxation, x <- x + omega M_{e,j} (b - L_j x).

    Its error propagator is S_j = I - omega M_{e,j} L_j (Sec. 2, after
    eq. (3)).  Every patch correction uses the residual of the same old x
    (the additive, parallel form of eq. (3)).  omega may be one value per
    system and complex (the complex relaxation parameter the paper leaves for
    future work after Example 3)."""
    return x + _per_system(omega) * vanka_smoother_apply(residual(x, b, lam, h), lam, h)


def jacobi_sweep(x, b, lam, h, omega):
    """Damped point Jacobi, x <- x + omega D_j^{-1}(b - L_j x) with
    D_j = (4 + lambda_j h^2)/h^2: the comparison smoother of Sec. 3
    (omega = 4/5 there)."""
    lam = np.asarray(lam, dtype=np.complex128)
    dinv = (h * h) / (4.0 + lam * h * h)
    return x + _per_system(omega) * dinv[:, None, None] * residual(x, b, lam, h)


def coarse_size(n):
    """Interior size after one standard coarsening, (n - 1)/2; the fine
    node 2I carries coarse node I (Sec. 2.1: standard coarsening)."""
    if n < 3 or n % 2 == 0:
        raise ValueError(f"cannot coarsen {n} interior nodes (need odd n >= 3)")
    return (n - 1) // 2


def _fw_1d_last(r):
    """1-D full weighting [1 2 1]/4 along the last axis: the coarse value at
    coarse node I is (r(2I-1) + 2 r(2I) + r(2I+1))/4 (1-based fine nodes)."""
    nc = coarse_size(r.shape[-1])
    # fine nodes 2I-1, 2I, 2I+1 (I = 1..nc) sit at 0-based positions
    # 2I-2, 2I-1, 2I along the axis
    left = r[..., 0:2 * nc - 1:2]
    centre = r[..., 1:2 * nc:2]
    right = r[..., 2:2 * nc + 1:2]
    out = 0.25 * left + 0.5 * centre + 0.25 * right
    return out


def restrict_full_weighting(r):
    """Full-weighting restriction named in Sec. 3 (stencil not printed):
    the textbook 9-point stencil (1/16)[1 2 1; 2 4 2; 1 2 1] centred on fine
    node (2I, 2K), applied as 1-D [1 2 1]/4 along x and then along y."""
    tmp = _fw_1d_last(r)
    tmp = np.swapaxes(_fw_1d_last(np.swapaxes(tmp, -1, -2)), -1, -2)
    return np.ascontiguousarray(tmp)


def _interp_1d_last(e):
    """1-D linear interpolation along the last axis from nc coarse nodes to
    2 nc + 1 fine nodes: fine 2I copies coarse I, fine 2I+1 averages coarse
    I and I+1, coarse values 0 and nc+1 are the zero Dirichlet boundary."""
    nc = e.shape[-1]
    out = np.zeros(e.shape[:-1] + (2 * nc + 1,), dtype=e.dtype)
    ext = np.zeros(e.shape[:-1] + (nc + 2,), dtype=e.dtype)
    ext[..., 1:nc + 1] = e                 # ext[..., I] = coarse node I
    # even fine node 2I (I = 1..nc) is 0-based position 2I-1
    out[..., 1::2] = ext[..., 1:nc + 1]
    # odd fine node 2I+1 (I = 0..nc) is 0-based position 2I
    out[..., 0::2] = 0.5 * (ext[..., 0:nc + 1] + ext[..., 1:nc + 2])
    return out


def prolong_bilinear(e):
    """Linear (bilinear) interpolation named in Sec. 3: the tensor product
    of 1-D linear interpolation in x and in y."""
    tmp = _interp_1d_last(e)
    tmp = np.swapaxes(_interp_1d_last(np.swapaxes(tmp, -1, -2)), -1, -2)
    return np.ascontiguousarray(tmp)


def level_shapes(nx, ny, h, levels=0, coarsest=7):
    """Grid hierarchy (nx, ny, h) from fine to coarse.

    Coarse operators are the re-discretisation with 2h (Sec. 3), so level l
    has mesh width 2^l h.  With ``levels`` > 0 exactly that many levels are
    built; with ``levels`` = 0 coarsening stops once the smaller side has at
    most ``coarsest`` nodes (Sec. 3 uses h0 = 1/8 on the unit square: 7x7).
    """
    shapes = [(nx, ny, h)]
    if levels > 0:
        for _ in range(levels - 1):
            cnx, cny, ch = shapes[-1]
            shapes.append((coarse_size(cnx), coarse_size(cny), 2.0 * ch))
    else:
        while min(shapes[-1][0], shapes[-1][1]) > coarsest:
            cnx, cny, ch = shapes[-1]
            shapes.append((coarse_size(cnx), coarse_size(cny), 2.0 * ch))
    return shapes
