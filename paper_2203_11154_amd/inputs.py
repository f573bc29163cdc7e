"""Seeded synthetic workloads shared by the tests, the benchmark and the
oracle-side checks.

This module only draws random numbers and evaluates the closed-form
definitions of the workloads (grids, shifts, right-hand sides); it holds none
of the solver's arithmetic and imports nothing else from this package.

Random draws use ``numpy.random.default_rng(seed)`` (PCG64) in FP64, real part
first, then imaginary part, each of the full shape (S, ny, nx).
"""
import numpy as np

SEED_RHS = 0
SEED_THETA = 1
SEED_THETA_STAR = 2
SEED_SHIFTS = 3


def rhs(S, ny, nx, seed=SEED_RHS):
    """b_j with real and imaginary parts i.i.d. U(-1, 1), complex128 (S, ny, nx)."""
    rng = np.random.default_rng(seed)
    re = rng.uniform(-1.0, 1.0, size=(S, ny, nx))
    im = rng.uniform(-1.0, 1.0, size=(S, ny, nx))
    return re + 1j * im


def alpha_circulant_shifts(n, alpha=0.01, tau=None):
    """lambda_j = (1 - alpha^{1/n} exp(2 pi i (j-1)/n))/tau, j = 1..n: the
    eigenvalues of the alpha-circulant backward-Euler matrix
    (1/tau)(I - Z_alpha); tau defaults to 1/n."""
    tau = 1.0 / n if tau is None else tau
    j = np.arange(n)
    return (1.0 - alpha ** (1.0 / n) * np.exp(2j * np.pi * j / n)) / tau


def alpha_circulant_vectors(n, alpha=0.01):
    """Eigenvector matrix V of the alpha-circulant and its inverse, matching
    the order of ``alpha_circulant_shifts``: V = diag(alpha^{-(i-1)/n}) F with
    F_{ik} = exp(-2 pi i (i-1)(k-1)/n), and V^{-1} = F^H diag(alpha^{(i-1)/n})/n.
    Both complex128 (n, n), row-major."""
    i = np.arange(n)
    F = np.exp(-2j * np.pi * np.outer(i, i) / n)
    scale = alpha ** (i / n)
    V = F / scale[:, None]
    Vinv = (F.conj().T * scale[None, :]) / n
    return np.ascontiguousarray(V), np.ascontiguousarray(Vinv)


def uniform_shifts(S, seed=SEED_SHIFTS, re=(1.0, 1e4), im=(-1e4, 1e4)):
    """Shifts with Re ~ U(re) and Im ~ U(im) (the batched uneven-grid workload)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(re[0], re[1], size=S)
    b = rng.uniform(im[0], im[1], size=S)
    return a + 1j * b


def example1_shifts(n):
    """Eigenvalues of the boundary-value-method matrix of Example 1,
    B = (1/tau) tridiag(-1/2, 0, 1/2) with last row (..., -1, 1), tau = 1/n."""
    B = np.zeros((n, n))
    for i in range(n - 1):
        if i > 0:
            B[i, i - 1] = -0.5
        B[i, i + 1] = 0.5
    B[n - 1, n - 2], B[n - 1, n - 1] = -1.0, 1.0
    return np.linalg.eigvals(B * n)


def example2_shifts(n, beta=0.01):
    """Eigenvalues of the (n+1) x (n+1) quasi-boundary-value matrix of
    Example 2: first row (1, 0, ..., 0, 1/beta), then (-1, 1) steps; tau = 1/n."""
    m = n + 1
    B = np.eye(m) - np.eye(m, k=-1)
    B[0, m - 1] = 1.0 / beta
    return np.linalg.eigvals(B * n)


def example3_shifts(count=128):
    """Example 3 (Helmholtz): lambda_j = -j^2 (1 - 0.5 i), j = 1..count."""
    j = np.arange(1, count + 1, dtype=np.float64)
    return -(j ** 2) * (1.0 - 0.5j)


def heat_parameters(K=16, seed=SEED_THETA):
    """theta_k ~ N(0, 1), k = 1..K."""
    return np.random.default_rng(seed).standard_normal(K)


def unit_square_h(nx):
    """Mesh width of an nx x nx interior grid on the unit square."""
    return 1.0 / (nx + 1)


# The five workloads.  Grids are unit squares (h = 1/(n+1)).
WORKLOADS = {
    "plain_63": dict(groups=[(63, 8)], shifts="alpha_circulant", n_time=8, alpha=0.01, levels=5,
                     nu1=2, nu2=2, tol=1e-10, precision="c128"),
    "plain_1023": dict(groups=[(1023, 64)], shifts="alpha_circulant", n_time=64, alpha=0.01, levels=0,
                       nu1=2, nu2=2, tol=1e-10, precision="c128"),
    "batched_uneven": dict(groups=[(127, 256), (255, 96), (511, 32)], shifts="uniform", levels=0,
                           nu1=2, nu2=2, tol=1e-10, precision="c128"),
    "ir_2047": dict(groups=[(2047, 32)], shifts="alpha_circulant", n_time=32, alpha=0.01, levels=0,
                    nu1=2, nu2=2, tol=1e-10, precision="c64_ir"),
    "heat_511": dict(groups=[(511, 128)], shifts="alpha_circulant", n_time=128, alpha=0.01, levels=0,
                     nu1=2, nu2=2, tol=1e-10, precision="c128", n_theta=16),
}


def workload_shifts(name):
    """Shifts of every system of a workload, concatenated over its grids."""
    w = WORKLOADS[name]
    total = sum(s for _, s in w["groups"])
    if w["shifts"] == "alpha_circulant":
        return alpha_circulant_shifts(w["n_time"], w["alpha"])
    return uniform_shifts(total)
