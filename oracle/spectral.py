"""Time-discretisation matrices B and their eigen-decompositions B = V D V^{-1}
(Sec. 1, eq. (1); test infrastructure only).

* ``bvm_matrix``: the boundary-value-method matrix of Example 1, eq. (9).
* ``qbvm_matrix``: the quasi-boundary-value matrix of Example 2, eq. (10).
* ``helmholtz_shifts``: the shifts of Example 3.
* ``alpha_circulant``: the alpha-circulant backward-Euler matrix
  C_alpha = (1/tau)(I - Z_alpha) used as the ParaDIAG preconditioner in the
  heat workloads (Sec. 1 mentions circulant-type approximations as
  preconditioners), with its closed-form eigen-decomposition.
"""
import numpy as np


def bvm_matrix(n):
    """Eq. (9): B = (1/tau) tridiag(-1/2, 0, 1/2) with last row (..., -1, 1),
    tau = 1/n."""
    tau = 1.0 / n
    B = np.zeros((n, n))
    for i in range(n - 1):
        if i > 0:
            B[i, i - 1] = -0.5
        B[i, i + 1] = 0.5
    B[n - 1, n - 2] = -1.0
    B[n - 1, n - 1] = 1.0
    return B / tau


def qbvm_matrix(n, beta=0.01):
    """Eq. (10): (n+1) x (n+1), first row (1, 0, ..., 0, 1/beta), then
    backward differences (-1, 1) on the sub- and main diagonal; tau = 1/n."""
    tau = 1.0 / n
    m = n + 1
    B = np.eye(m) - np.eye(m, k=-1)
    B[0, m - 1] = 1.0 / beta
    return B / tau


def helmholtz_shifts(count=128):
    """Example 3: lambda_j = -j^2 (1 - 0.5 i), j = 1..count."""
    j = np.arange(1, count + 1, dtype=np.float64)
    return -(j ** 2) * (1.0 - 0.5j)


def alpha_circulant(n, alpha, tau):
    """C_alpha = (1/tau)(I - Z_alpha): Z_alpha has ones on the subdiagonal and
    alpha in the top-right corner (backward Euler with an alpha-periodic
    wrap of the initial condition)."""
    Z = np.eye(n, k=-1)
    Z[0, n - 1] = alpha
    return (np.eye(n) - Z) / tau


def alpha_circulant_eig(n, alpha, tau):
    """Closed-form eigen-decomposition C_alpha = V D V^{-1}.

    Z_alpha = alpha^{1/n} G^{-1} Z_1 G with G = diag(alpha^{(i-1)/n}) and Z_1
    the cyclic down-shift, whose eigenvectors are the Fourier columns
    W_{ij} = exp(-2 pi i (i-1)(j-1)/n) with eigenvalues exp(2 pi i (j-1)/n).
    Hence lambda_j = (1 - alpha^{1/n} exp(2 pi i (j-1)/n))/tau,
    V = G^{-1} W and V^{-1} = W^H G / n.
    Returns (lam, V, Vinv).
    """
    idx = np.arange(n)
    W = np.exp(-2j * np.pi * np.outer(idx, idx) / n)
    g = alpha ** (idx / n)
    V = W / g[:, None]
    Vinv = (W.conj().T * g[None, :]) / n
    lam = (1.0 - alpha ** (1.0 / n) * np.exp(2j * np.pi * idx / n)) / tau
    return lam, V, Vinv
