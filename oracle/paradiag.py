"""ParaDIAG around the shifted solves (Sec. 1, eqs. (1)-(2); test
infrastructure only).

The all-at-once system of eq. (1) is (B kron I_h + I_t kron A) u = f with the
n time slices of u stacked as the rows of an (n, ny, nx) array.  With
B = V D V^{-1} it is solved in three steps:
  G = (V^{-1} kron I_h) F,   z_j = (A + lambda_j I)^{-1} g_j,   U = (V kron I_h) Z.
The heat workload uses the alpha-circulant C_alpha as a preconditioner (the
circulant-type preconditioner that Sec. 1 mentions) for K, the
backward-Euler all-at-once operator, inside either the stationary iteration
u <- u + P_alpha^{-1}(f - K u) or a Krylov method (flexible GMRES with right
preconditioning; the paper names the preconditioner, not the outer solver).
"""
import numpy as np

from . import operators as ops
from . import multigrid as mg
from . import exact


def time_transform(M, F):
    """(M kron I_h) F for F of shape (n, ny, nx): out_i = sum_k M_ik F_k."""
    n = F.shape[0]
    return (M @ F.reshape(n, -1)).reshape(F.shape)


def shifted_block_solve(G, lam, h, tol, solver="multigrid", **mg_opts):
    """Step 2 of eq. (1): z_j = (A + lambda_j I)^{-1} g_j for every j, by the
    Vanka multigrid iteration or, with solver="dst", exactly."""
    if solver == "dst":
        return exact.dst_solve(G, lam, h)
    z, _, _, _ = mg.solve(G, lam, h, tol=tol, **mg_opts)
    return z


def paradiag_apply(F, lam, V, Vinv, h, tol=1e-10, solver="multigrid", **mg_opts):
    """(B kron I + I kron A)^{-1} F for B = V diag(lam) V^{-1} (eq. (1))."""
    G = time_transform(Vinv, F.astype(np.complex128))
    Z = shifted_block_solve(G, lam, h, tol, solver, **mg_opts)
    return time_transform(V, Z)


def backward_euler_apply(U, tau, h, u0=None):
    """K u for the backward-Euler all-at-once heat operator:
    (K u)^m = (u^m - u^{m-1})/tau + A u^m, m = 1..n, u^0 = u0 (default 0)."""
    n = U.shape[0]
    prev = np.zeros_like(U)
    prev[1:] = U[:-1]
    if u0 is not None:
        prev[0] = u0
    zero = np.zeros(n, dtype=np.complex128)
    return (U - prev) / tau + ops.apply_shifted_laplacian(U, zero, h)


def backward_euler_apply_transpose(W, tau, h):
    """K^T w: (K^T w)^m = (w^m - w^{m+1})/tau + A w^m (A is symmetric)."""
    nxt = np.zeros_like(W)
    nxt[:-1] = W[1:]
    zero = np.zeros(W.shape[0], dtype=np.complex128)
    return (W - nxt) / tau + ops.apply_shifted_laplacian(W, zero, h)


def heat_source(theta, n, nx, tau):
    """f^m(x, y) = sum_k theta_k sin(k pi x) sin(k pi y) exp(-t_m), t_m = m tau,
    m = 1..n, on the nx x nx interior of the unit square."""
    f = np.zeros((n, nx, nx))
    t = tau * np.arange(1, n + 1)
    for k, th in enumerate(theta, start=1):
        f += th * np.exp(-t)[:, None, None] * exact.sine_mode(k, k, nx, nx)[None]
    return f


def paradiag_heat_solve(f, tau, h, lam, V, Vinv, tol=1e-10, inner_tol=1e-12, max_outer=50,
                        transpose=False, solver="multigrid", **mg_opts):
    """Stationary ParaDIAG iteration u <- u + P_alpha^{-1}(f - K u) from u = 0
    until ||f - K u|| <= tol ||f||.  With transpose=True it solves K^T w = f
    with P_alpha^{-T} = (V^{-T} kron I)(D kron I + I kron A)^{-1}(V^T kron I).
    Returns (u, outer_iterations, relres)."""
    f = f.astype(np.complex128)
    u = np.zeros_like(f)
    fn = np.linalg.norm(f)
    Kop = backward_euler_apply_transpose if transpose else backward_euler_apply
    Vl, Vr = (Vinv.T, V.T) if transpose else (V, Vinv)
    rel = 1.0
    for it in range(1, max_outer + 1):
        r = f - Kop(u, tau, h)
        rel = np.linalg.norm(r) / fn
        if rel <= tol:
            return u, it - 1, rel
        G = time_transform(Vr, r)
        Z = shifted_block_solve(G, lam, h, inner_tol, solver, **mg_opts)
        u = u + time_transform(Vl, Z)
    r = f - Kop(u, tau, h)
    return u, max_outer, np.linalg.norm(r) / fn


def paradiag_heat_fgmres(f, tau, h, lam, V, Vinv, tol=1e-10, inner_tol=1e-12, restart=10, max_iter=100,
                         transpose=False, solver="multigrid", **mg_opts):
    """Restarted flexible GMRES on K u = f (K^T w = f with transpose=True),
    right-preconditioned by the alpha-circulant ParaDIAG step P_alpha^{-1},
    from u = 0.

    Each restart cycle starts from r = f - K u, beta = ||r||, v_1 = r / beta.
    Step j applies the preconditioner z_j = P^{-1} v_j and the operator
    w = K z_j, orthogonalises w against v_1..v_j by modified Gram-Schmidt
    (h_ij = <v_i, w>, w <- w - h_ij v_i), sets h_{j+1,j} = ||w|| and
    v_{j+1} = w / h_{j+1,j}.  The coefficients y minimise
    ||beta e_1 - H_j y|| (a dense least-squares solve); the cycle ends when
    that minimum is at most tol ||f||, after `restart` steps, or at max_iter
    steps in total, and then u <- u + sum_i y_i z_i.  The loop stops when the
    true residual ||f - K u|| <= tol ||f||.
    Returns (u, total_steps, relres, history of the least-squares residuals
    relative to ||f||)."""
    f = f.astype(np.complex128)
    u = np.zeros_like(f)
    fn = np.linalg.norm(f)
    Kop = backward_euler_apply_transpose if transpose else backward_euler_apply
    Vl, Vr = (Vinv.T, V.T) if transpose else (V, Vinv)

    def precond(v):
        G = time_transform(Vr, v)
        return time_transform(Vl, shifted_block_solve(G, lam, h, inner_tol, solver, **mg_opts))

    total, hist = 0, []
    while True:
        r = f - Kop(u, tau, h)
        beta = np.linalg.norm(r)
        if fn == 0.0 or beta <= tol * fn or total >= max_iter:
            return u, total, (beta / fn if fn > 0 else 0.0), hist
        Vb = [r / beta]
        Zb = []
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        y = None
        for j in range(restart):
            Zb.append(precond(Vb[j]))
            w = Kop(Zb[j], tau, h)
            for i in range(j + 1):
                H[i, j] = np.vdot(Vb[i], w)
                w = w - H[i, j] * Vb[i]
            H[j + 1, j] = np.linalg.norm(w)
            Vb.append(w / H[j + 1, j] if H[j + 1, j] != 0 else w)
            total += 1
            e1 = np.zeros(j + 2, dtype=np.complex128)
            e1[0] = beta
            y = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)[0]
            res = np.linalg.norm(e1 - H[:j + 2, :j + 1] @ y) / fn
            hist.append(res)
            if res <= tol or total >= max_iter or H[j + 1, j] == 0:
                break
        for i in range(len(y)):
            u = u + y[i] * Zb[i]


def heat_mode_coefficients(n, nx, tau):
    """Closed form of the heat workload: the response to theta_k = 1 is
    c_k^m phi_kk with (c^m - c^{m-1})/tau + mu_kk c^m = exp(-t_m), c^0 = 0,
    where mu_kk = (8/h^2) sin^2(k pi h/2) is the eigenvalue of A on phi_kk.
    Returns c of shape (K_max=nx, n) for k = 1..nx."""
    h = 1.0 / (nx + 1)
    k = np.arange(1, nx + 1)
    mu = (8.0 / (h * h)) * np.sin(k * np.pi * h / 2) ** 2
    c = np.zeros((nx, n))
    prev = np.zeros(nx)
    for m in range(1, n + 1):
        cur = (prev / tau + np.exp(-m * tau)) / (1.0 / tau + mu)
        c[:, m - 1] = cur
        prev = cur
    return c


def heat_loss_closed_form(theta, theta_star, n, nx, tau):
    """L = sum over slices and nodes of (u - u*)^2 and dL/dtheta in closed
    form: modes phi_kk are orthogonal with ||phi_kk||^2 = ((nx+1)/2)^2."""
    K = len(theta)
    c = heat_mode_coefficients(n, nx, tau)[:K]
    wk = np.sum(c * c, axis=1) * ((nx + 1) / 2.0) ** 2
    d = np.asarray(theta) - np.asarray(theta_star)
    return float(np.sum(d * d * wk)), 2.0 * d * wk
