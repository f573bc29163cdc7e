"""Exact references for the shifted systems (test infrastructure only).

These are independent of the multigrid iteration: a dense Kronecker
assembly of A + lambda_j I, its closed-form sine eigenpairs, and the DST-I
diagonalisation that solves every shifted system exactly at any size.
"""
import numpy as np
import scipy.fft


def dense_laplacian(nx, ny, h):
    """Dense 5-point Dirichlet Laplacian of Sec. 1 (below eq. (2)), built as
    (1/h^2)(I_y kron T_x + T_y kron I_x) with T = tridiag(-1, 2, -1), for the
    x-fastest ordering of interior nodes."""
    def tridiag(n):
        return 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    return (np.kron(np.eye(ny), tridiag(nx)) + np.kron(tridiag(ny), np.eye(nx))) / (h * h)


def dense_shifted(nx, ny, h, lam):
    """Dense L_j = A + lambda_j I of eq. (2)."""
    return dense_laplacian(nx, ny, h).astype(np.complex128) + lam * np.eye(nx * ny)


def dense_solve(b, lam, h):
    """Solve every system of eq. (2) with a dense LU; b has shape (S, ny, nx).
    Meant for grids of at most a few thousand unknowns."""
    S, ny, nx = b.shape
    A = dense_laplacian(nx, ny, h)
    out = np.empty_like(b, dtype=np.complex128)
    for j in range(S):
        Lj = A + lam[j] * np.eye(nx * ny)
        out[j] = np.linalg.solve(Lj, b[j].reshape(-1)).reshape(ny, nx)
    return out


def laplacian_eigenvalues(nx, ny, h):
    """Eigenvalues of the 5-point Dirichlet Laplacian, array (ny, nx):
    mu_{kl} = (4/h^2)(sin^2(k pi/(2(nx+1))) + sin^2(l pi/(2(ny+1)))), k = 1..nx,
    l = 1..ny.  On the unit square h = 1/(nx+1) and this is
    (4/h^2)(sin^2(k pi h/2) + sin^2(l pi h/2))."""
    k = np.arange(1, nx + 1)
    l = np.arange(1, ny + 1)
    sx = np.sin(k * np.pi / (2.0 * (nx + 1))) ** 2
    sy = np.sin(l * np.pi / (2.0 * (ny + 1))) ** 2
    return (4.0 / (h * h)) * (sy[:, None] + sx[None, :])


def sine_mode(k, l, nx, ny):
    """Eigenvector phi_{kl}(i, j) = sin(k pi i/(nx+1)) sin(l pi j/(ny+1)) on the
    interior nodes, array (ny, nx)."""
    i = np.arange(1, nx + 1)
    j = np.arange(1, ny + 1)
    return np.outer(np.sin(l * np.pi * j / (ny + 1)), np.sin(k * np.pi * i / (nx + 1)))


def dst_solve(b, lam, h):
    """Exact solution of every system of eq. (2) by sine diagonalisation:
    z_j = DST(DST(b_j) / (mu_kl + lambda_j)) with the orthonormal DST-I,
    which is its own inverse.  b has shape (S, ny, nx)."""
    b = np.asarray(b, dtype=np.complex128)
    S, ny, nx = b.shape
    mu = laplacian_eigenvalues(nx, ny, h)
    lam = np.asarray(lam, dtype=np.complex128)
    out = np.empty_like(b)
    for j in range(S):
        bh = scipy.fft.dstn(b[j].real, type=1, norm="ortho") + 1j * scipy.fft.dstn(b[j].imag, type=1, norm="ortho")
        zh = bh / (mu + lam[j])
        out[j] = scipy.fft.dstn(zh.real, type=1, norm="ortho") + 1j * scipy.fft.dstn(zh.imag, type=1, norm="ortho")
    return out
