"""Pins of the oracle's multigrid solve: dense direct solves, the DST-I exact
solver, manufactured discrete solutions, and measured two-grid rates against
the Fourier-analysis prediction."""
import numpy as np
import pytest

from oracle import exact, lfa, multigrid as mg, operators as ops
from paper_2203_11154_amd import inputs

RNG = np.random.default_rng(77)


def crandn(*shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


def test_dst_solver_matches_dense_lu():
    nx, ny, h = 15, 7, 1.0 / 16
    lam = np.array([3 + 4j, 100 - 20j, -5 + 80j])
    b = crandn(3, ny, nx)
    np.testing.assert_allclose(exact.dst_solve(b, lam, h), exact.dense_solve(b, lam, h), rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("n,levels", [(15, 0), (31, 0), (31, 4), (15, 3)])
def test_multigrid_reaches_dense_solution(n, levels):
    h = 1.0 / (n + 1)
    lam = inputs.alpha_circulant_shifts(8)
    b = inputs.rhs(8, n, n)
    z, iters, relres, _ = mg.solve(b, lam, h, tol=1e-10, levels=levels)
    zd = exact.dense_solve(b, lam, h)
    assert np.all(relres <= 1e-10)
    err = np.linalg.norm((z - zd).reshape(8, -1), axis=1) / np.linalg.norm(zd.reshape(8, -1), axis=1)
    # ||z - z*|| / ||z*|| <= cond(L_j) * relres; cond ~ 1e3 at n = 31
    assert np.all(err <= 1e-7)
    assert np.all(iters <= 15)


def test_multigrid_rectangle():
    nx, ny, h = 63, 15, 1.0 / 64
    lam = np.array([5 + 5j, 2000 - 3000j])
    b = crandn(2, ny, nx)
    z, iters, relres, _ = mg.solve(b, lam, h, tol=1e-10)
    zd = exact.dst_solve(b, lam, h)
    assert np.all(relres <= 1e-10)
    assert np.linalg.norm(z - zd) <= 1e-7 * np.linalg.norm(zd)


def test_manufactured_discrete_solution():
    n = 31
    h = 1.0 / (n + 1)
    lam = inputs.uniform_shifts(4)
    zstar = crandn(4, n, n)
    b = np.stack([(exact.dense_shifted(n, n, h, lam[j]) @ zstar[j].ravel()).reshape(n, n) for j in range(4)])
    z, iters, relres, _ = mg.solve(b, lam, h, tol=1e-12)
    assert np.linalg.norm(z - zstar) <= 1e-9 * np.linalg.norm(zstar)


def test_plain_small_workload_against_dst():
    """The 63 x 63, 8-shift, 5-level V(2,2) workload converges to 1e-10 and
    agrees with the exact DST solution."""
    n = 63
    h = 1.0 / 64
    lam = inputs.alpha_circulant_shifts(8)
    b = inputs.rhs(8, n, n)
    z, iters, relres, hist = mg.solve(b, lam, h, tol=1e-10, levels=5)
    zx = exact.dst_solve(b, lam, h)
    assert np.all(relres <= 1e-10)
    assert np.all((iters >= 6) & (iters <= 14)), iters
    err = np.linalg.norm((z - zx).reshape(8, -1), axis=1) / np.linalg.norm(zx.reshape(8, -1), axis=1)
    assert np.all(err <= 1e-8)
    # observed V(2,2) rates stay below the two-grid prediction rho(4) ~ 0.064 plus slack
    rates = [mg.observed_rate(hh) for hh in hist]
    assert max(rates) < 0.1


def test_measured_two_grid_rate_matches_rfa():
    """Power iteration on the oracle's two-grid error propagation (1 pre-
    sweep, exact coarse solve) converges to the spectral radius predicted by
    the sine-mode analysis."""
    n = 63
    h = 1.0 / (n + 1)
    lam = np.array([0.8 + 40j])
    e = crandn(1, n, n)
    e /= np.linalg.norm(e)
    ratio = 0.0
    for it in range(60):
        e_new = mg.two_grid_error_step(e, lam, h, nu1=1, nu2=0)
        ratio = np.linalg.norm(e_new) / np.linalg.norm(e)
        e = e_new / np.linalg.norm(e_new)
    rho = np.max(np.abs(lfa.rfa_two_grid_spectrum(n, lam[0] * h * h, 24 / 25, 1, 0)))
    assert ratio == pytest.approx(rho, abs=2e-3)
    # and both are close to the LFA smoothing factor 0.28 (Table 1)
    assert abs(rho - 0.28) < 0.01


def test_w_cycle_and_jacobi_protocol():
    """Sec. 3 protocol: W(1,0) to 1e-8 from h0 = 1/8; Vanka needs far fewer
    cycles than damped Jacobi (rho 0.28 vs 0.6)."""
    n = 63
    h = 1.0 / 64
    lam = np.array([2 + 60j, 30 - 10j])
    b = inputs.rhs(2, n, n)
    _, it_v, rr_v, _ = mg.solve(b, lam, h, tol=1e-8, nu1=1, nu2=0, gamma=2)
    _, it_j, rr_j, _ = mg.solve(b, lam, h, tol=1e-8, nu1=1, nu2=0, gamma=2, smoother="jacobi",
                                omega=mg.OMEGA_JACOBI, max_iter=200)
    assert np.all(rr_v <= 1e-8) and np.all(rr_j <= 1e-8)
    assert np.all(it_j >= 2 * it_v)


def test_zero_rhs_and_fixed_iterations():
    n = 15
    h = 1.0 / 16
    lam = np.array([1 + 1j, 2 + 2j])
    b = inputs.rhs(2, n, n)
    b[1] = 0
    z, iters, relres, _ = mg.solve(b, lam, h)
    assert iters[1] == 0 and np.all(z[1] == 0)
    z2, it2, _, _ = mg.solve(b, lam, h, fixed_iters=[3, 0])
    assert list(it2) == [3, 0]


def test_observed_rate_hand_computed():
    """The observed rate is the geometric mean of the per-cycle reductions of
    the relative residual from r_0/||b|| = 1 (x0 = 0), i.e. the K-th root of
    the last entry of a K-cycle history.  Values worked by hand: an arithmetic
    mean of the ratios, a root of K - 1, or the first entry would each give
    another number."""
    # ratios 0.5, 0.2, 0.2: geometric mean 0.02^(1/3) = 0.271441761659..
    assert mg.observed_rate([0.5, 0.1, 0.02]) == pytest.approx(0.2714417616594907, rel=1e-14)
    # a constant contraction of 0.28 (Table 1's Vanka factor) over 5 cycles
    assert mg.observed_rate([0.28, 0.0784, 0.021952, 0.00614656, 0.0017210368]) == pytest.approx(0.28, rel=1e-13)
    assert mg.observed_rate([0.001]) == pytest.approx(0.001, rel=1e-15)
    assert mg.observed_rate([]) == 0.0
