"""Pins of the oracle's grid operators against facts independent of its code:
dense Kronecker assembly, closed-form eigenpairs, the paper's printed symbols
and coefficients, brute-force patch inverses and textbook transfer weights."""
import numpy as np
import pytest

from oracle import operators as ops
from oracle import exact, lfa, multigrid as mg

RNG = np.random.default_rng(1234)


def crandn(*shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


def test_shifted_laplacian_matches_dense_kron():
    nx, ny, h = 7, 5, 0.13
    lam = crandn(3) * 40
    x = crandn(3, ny, nx)
    Lx = ops.apply_shifted_laplacian(x, lam, h)
    for j in range(3):
        dense = exact.dense_shifted(nx, ny, h, lam[j])
        np.testing.assert_allclose(Lx[j].ravel(), dense @ x[j].ravel(), rtol=1e-13, atol=1e-10)


def test_laplacian_eigenvalues_match_library_eigensolver():
    nx, ny, h = 9, 5, 0.1
    mu = np.sort(exact.laplacian_eigenvalues(nx, ny, h).ravel())
    ref = np.linalg.eigvalsh(exact.dense_laplacian(nx, ny, h))
    np.testing.assert_allclose(mu, ref, rtol=1e-12)


@pytest.mark.parametrize("k,l", [(1, 1), (2, 5), (7, 3)])
def test_sine_modes_are_eigenvectors(k, l):
    # A phi_kl = mu_kl phi_kl with mu_kl = (4/h^2)(sin^2(k pi h/2) + sin^2(l pi h/2))
    n = 15
    h = 1.0 / (n + 1)
    lam = np.array([3.0 + 7.0j])
    phi = exact.sine_mode(k, l, n, n)[None].astype(np.complex128)
    mu = 4.0 / h ** 2 * (np.sin(k * np.pi * h / 2) ** 2 + np.sin(l * np.pi * h / 2) ** 2)
    np.testing.assert_allclose(ops.apply_shifted_laplacian(phi, lam, h), (mu + lam[0]) * phi, atol=1e-9)


def test_vanka_coefficients_stable_equal_printed():
    eta = np.concatenate([crandn(200) * 3, crandn(50) * 0.01, np.array([0.0, 1e-3j, 2.5 - 1j])])
    a1, b1, c1 = ops.vanka_abc_paper(eta)
    a2, b2, c2 = ops.vanka_abc(eta)
    for u, v in ((a1, a2), (b1, b2), (c1, c2)):
        np.testing.assert_allclose(u, v, rtol=1e-13, atol=1e-15)


def test_vanka_coefficients_at_zero_shift():
    # eta = 0: the Laplacian patch inverse, a, b, c = 7/24, 1/12, 1/24
    a, b, c = ops.vanka_abc(0.0)
    np.testing.assert_allclose([a, b, c], [7 / 24, 1 / 12, 1 / 24], rtol=1e-15)


def cell_matrix(eta, h):
    """4x4 restriction of L_j to the vertices of one cell, ordered
    (0,0), (1,0), (0,1), (1,1): each vertex couples to its two cell neighbours
    along the grid lines but not to the opposite corner."""
    d = 4.0 + eta
    return np.array([[d, -1, -1, 0], [-1, d, 0, -1], [-1, 0, d, -1], [0, -1, -1, d]],
                    dtype=np.complex128) / (h * h)


@pytest.mark.parametrize("eta", [0.0, (3 + 40j) / 64, 2.0 - 5.0j, -0.3 + 0.1j])
def test_patch_inverse_brute_force(eta):
    h = 0.25
    inv = np.linalg.inv(cell_matrix(eta, h))
    a, b, c = ops.vanka_abc(eta)
    expect = h * h * np.array([[a, b, b, c], [b, a, c, b], [b, c, a, b], [c, b, b, a]])
    np.testing.assert_allclose(inv, expect, rtol=1e-12, atol=1e-14)


def test_global_additive_vanka_equals_stencil():
    """Sum over all cells of R_i^T (I/4) L_i^{-1} R_i (eq. (3), weight 1/4 per
    vertex, boundary vertices dropped) equals the stencil matrix of eq. (6)."""
    nx, ny, h = 7, 6, 1.0 / 8
    lam = np.array([300.0 - 2000.0j])
    eta = lam[0] * h * h
    N = nx * ny
    M = np.zeros((N, N), dtype=np.complex128)
    inv = np.linalg.inv(cell_matrix(eta, h))
    for cy in range(0, ny + 1):          # cell with lower-left vertex (cx, cy)
        for cx in range(0, nx + 1):
            verts = [(cx, cy), (cx + 1, cy), (cx, cy + 1), (cx + 1, cy + 1)]
            gidx = [(j - 1) * nx + (i - 1) if 1 <= i <= nx and 1 <= j <= ny else -1 for i, j in verts]
            for p in range(4):
                for q in range(4):
                    if gidx[p] >= 0 and gidx[q] >= 0:
                        M[gidx[p], gidx[q]] += 0.25 * inv[p, q]
    E = np.eye(N, dtype=np.complex128).reshape(N, ny, nx)
    stencil = ops.vanka_smoother_apply(E, np.full(N, lam[0]), h).reshape(N, N).T
    np.testing.assert_allclose(stencil, M, rtol=1e-12, atol=1e-18)


@pytest.mark.parametrize("k,l,lam", [(2, 5, 30 + 100j), (1, 1, 0.5 - 3j), (6, 6, 2000 - 9000j), (7, 1, -50 + 25j)])
def test_sweep_on_sine_mode_is_printed_symbol(k, l, lam):
    """One sweep with b = 0 maps the error phi_kl to S~_j(k pi h, l pi h) phi_kl
    with S~ written out as in eq. (7) (sine modes vanish on the ring)."""
    n = 7
    h = 1.0 / (n + 1)
    omega = 24 / 25
    t1, t2 = k * np.pi * h, l * np.pi * h
    eta = lam * h * h
    a, b, c = ops.vanka_abc_paper(eta)
    s = 1 - omega * (a + b * np.cos(t1) + b * np.cos(t2) + c * np.cos(t1) * np.cos(t2)) * \
        (4 + eta - 2 * np.cos(t1) - 2 * np.cos(t2))
    phi = exact.sine_mode(k, l, n, n)[None].astype(np.complex128)
    out = ops.vanka_sweep(phi, np.zeros_like(phi), np.array([lam]), h, omega)
    np.testing.assert_allclose(out, s * phi, atol=1e-13)
    np.testing.assert_allclose(lfa.symbol_S(t1, t2, eta, omega), s, rtol=1e-13)


def test_jacobi_on_sine_mode():
    n, k, l, lam, omega = 7, 3, 2, 10 + 5j, 0.8
    h = 1.0 / (n + 1)
    eta = lam * h * h
    s = 1 - omega * (4 + eta - 2 * np.cos(k * np.pi * h) - 2 * np.cos(l * np.pi * h)) / (4 + eta)
    phi = exact.sine_mode(k, l, n, n)[None].astype(np.complex128)
    out = ops.jacobi_sweep(phi, np.zeros_like(phi), np.array([lam]), h, omega)
    np.testing.assert_allclose(out, s * phi, atol=1e-13)


def test_full_weighting_stencil_weights():
    """A unit residual at fine node (fi, fk) reaches coarse node (I, K) with
    weight w[fk - 2K][fi - 2I] of (1/16)[1 2 1; 2 4 2; 1 2 1] when both
    offsets are within one node, and nowhere else."""
    nx, ny = 9, 7
    w = np.array([[1, 2, 1], [2, 4, 2], [1, 2, 1]]) / 16.0
    for fk in range(1, ny + 1):
        for fi in range(1, nx + 1):
            r = np.zeros((1, ny, nx))
            r[0, fk - 1, fi - 1] = 1.0
            rc = ops.restrict_full_weighting(r)
            assert rc.shape == (1, 3, 4)
            expect = np.zeros((3, 4))
            for K in range(1, 4):
                for I in range(1, 5):
                    dx, dy = fi - 2 * I, fk - 2 * K
                    if abs(dx) <= 1 and abs(dy) <= 1:
                        expect[K - 1, I - 1] = w[dy + 1, dx + 1]
            np.testing.assert_array_equal(rc[0], expect)


def test_bilinear_interpolation_of_coarse_delta():
    e = np.zeros((1, 3, 4))
    e[0, 1, 2] = 1.0              # coarse node (I, K) = (3, 2) = fine (6, 4)
    f = ops.prolong_bilinear(e)
    assert f.shape == (1, 7, 9)
    expect = np.zeros((7, 9))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            expect[4 + dy - 1, 6 + dx - 1] = (1 - abs(dx) / 2) * (1 - abs(dy) / 2)
    np.testing.assert_array_equal(f[0], expect)


def test_transfers_are_adjoint_up_to_four():
    u = crandn(2, 15, 31)
    v = crandn(2, 7, 15)
    lhs = 4 * np.vdot(ops.restrict_full_weighting(u), v)
    rhs = np.vdot(u, ops.prolong_bilinear(v))
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)


def test_bilinear_reproduces_piecewise_linear_interior():
    # a function linear in each coordinate on the interior of the coarse
    # nodes is reproduced at the fine nodes between them
    e = np.zeros((1, 7, 7))
    cx = np.arange(1, 8) / 8.0
    e[0] = np.outer(2 + cx, 1 - 0.5 * cx)
    f = ops.prolong_bilinear(e)[0]
    fx = np.arange(1, 16) / 16.0
    exact_f = np.outer(2 + fx, 1 - 0.5 * fx)
    # away from the ring the interpolant is exact for a bilinear function
    np.testing.assert_allclose(f[1:-1, 1:-1], exact_f[1:-1, 1:-1], rtol=1e-14)


def test_level_shapes():
    assert [s[0] for s in ops.level_shapes(63, 63, 1 / 64, levels=5)] == [63, 31, 15, 7, 3]
    assert [s[0] for s in ops.level_shapes(1023, 1023, 1 / 1024)] == [1023, 511, 255, 127, 63, 31, 15, 7]
    sh = ops.level_shapes(127, 63, 1 / 128)
    assert sh[-1][:2] == (15, 7) and sh[-1][2] == pytest.approx(1 / 16)
    with pytest.raises(ValueError):
        ops.level_shapes(64, 64, 1 / 65, levels=3)


@pytest.mark.parametrize("lam", [0.5 + 60j, 8 - 3j, 3000 + 5000j])
def test_two_grid_operator_spectrum_matches_rfa(lam):
    """Assemble the oracle's two-grid error operator (1 pre-, 1 post-sweep,
    exact coarse solve) column by column on a 15 x 15 grid and compare its
    whole spectrum with the sine-mode (rigorous Fourier) block analysis.
    This pins sweep, full weighting, interpolation and the coarse operator
    together."""
    n = 15
    h = 1.0 / (n + 1)
    N = n * n
    E = np.eye(N, dtype=np.complex128).reshape(N, n, n)
    cols = mg.two_grid_error_step(E, np.full(N, lam), h, nu1=1, nu2=1)
    T = cols.reshape(N, N).T
    ev = np.linalg.eigvals(T)
    ref = lfa.rfa_two_grid_spectrum(n, lam * h * h, 24 / 25, 1, 1)
    assert len(ref) == N
    key = lambda z: (round(z.real, 9), round(z.imag, 9))
    np.testing.assert_allclose(sorted(ev, key=key), sorted(ref, key=key), atol=1e-9)
