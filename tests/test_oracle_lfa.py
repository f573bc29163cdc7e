"""Pins of the oracle's Fourier analysis against what the paper prints
(Table 1, the 7/25 optimum, Remark 2.1, Theorem 2.1, the eigenvalue bound of
Example 1) and against closed forms."""
import os

import numpy as np
import pytest

from oracle import lfa, spectral

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1.txt")


def load_table1():
    rows = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        name, *vals = line.split()
        rows[name] = [float(v) for v in vals]
    return rows


@pytest.fixture(scope="module")
def ex1_eta():
    # Example 1: eigenvalues of eq. (9) with n = 256, h = tau = 1/256
    lam = np.linalg.eigvals(spectral.bvm_matrix(256))
    return lam * (1.0 / 256) ** 2


@pytest.mark.parametrize("smoother", ["jacobi", "vanka"])
def test_table1(ex1_eta, smoother):
    omega_p, mu_p, *rho_p = load_table1()[smoother]
    eta = ex1_eta[0]
    w, rho1 = lfa.optimal_omega(eta, smoother)
    assert w == pytest.approx(omega_p, abs=1e-9)
    mu = lfa.smoothing_factor(eta, omega_p, smoother, n=256)
    assert abs(mu - mu_p) <= 6e-4
    for nu, want in enumerate(rho_p, start=1):
        got = lfa.two_grid_factor(eta, omega_p, nu, smoother, n=128)
        assert abs(got - want) <= 6e-4, (smoother, nu, got, want)


def test_closed_form_optimum_zero_shift():
    """eta = 0: M~_0 A~ ranges over [3/4, 4/3] on T^H, so omega = 24/25 gives
    mu = 7/25 (Sec. 2.1 after Theorem 2.1); Jacobi omega = 4/5 gives 3/5."""
    # theta = (pi/2, 0) and (pi, pi) are the extremes; include them exactly
    for t1, t2, val in [(np.pi / 2, 0.0, 3 / 4), (np.pi, np.pi, 4 / 3)]:
        m = lfa.symbol_M_vanka(t1, t2, 0.0) * lfa.symbol_L(t1, t2, 0.0)
        assert m == pytest.approx(val, rel=1e-14)
    t1, t2 = lfa.high_frequency_grid(256)
    prod = (lfa.symbol_M_vanka(t1, t2, 0.0) * lfa.symbol_L(t1, t2, 0.0)).real
    assert prod.min() >= 0.75 - 1e-12 and prod.max() <= 4 / 3 + 1e-12
    assert lfa.smoothing_factor(0.0, 24 / 25, n=256) <= 7 / 25 + 1e-12
    assert abs(1 - 24 / 25 * 0.75) == pytest.approx(7 / 25)
    assert abs(1 - 24 / 25 * 4 / 3) == pytest.approx(7 / 25)
    assert lfa.smoothing_factor(0.0, 4 / 5, "jacobi", n=256) == pytest.approx(3 / 5, abs=1e-3)


def test_remark_uniform_over_eigenvalues(ex1_eta):
    """Remark 2.1: the same omega_opt and factors for every eigenvalue of B."""
    idx = np.linspace(0, len(ex1_eta) - 1, 9).astype(int)
    mus = [lfa.smoothing_factor(e, 24 / 25) for e in ex1_eta[idx]]
    rho4 = [lfa.two_grid_factor(e, 24 / 25, 4) for e in ex1_eta[idx]]
    assert max(mus) - min(mus) < 1e-3 and max(mus) < 0.2805
    assert max(rho4) - min(rho4) < 1e-3


def test_theorem_upper_bound(ex1_eta):
    """Theorem 2.1: mu_loc <= phi_0(omega) + phi_j(omega), here checked on the
    Example 1 shifts (lambda_j = O(1/h))."""
    w = 24 / 25
    t1, t2 = lfa.high_frequency_grid(96)
    phi0 = np.max(np.abs(1 - w * lfa.symbol_M_vanka(t1, t2, 0.0) * lfa.symbol_L(t1, t2, 0.0)))
    for e in ex1_eta[::32]:
        mu = np.max(np.abs(lfa.symbol_S(t1, t2, e, w)))
        phij = np.max(np.abs(w * e * lfa.symbol_M_vanka(t1, t2, e)))
        assert mu <= phi0 + phij + 1e-12


def test_example1_eigenvalue_bound():
    """Example 1: |lambda_j| < n + sqrt(n)/sqrt(2)."""
    for n in (16, 64, 256):
        lam = np.linalg.eigvals(spectral.bvm_matrix(n))
        assert np.max(np.abs(lam)) < n + np.sqrt(n) / np.sqrt(2)


def test_smoothing_factor_close_to_rho1(ex1_eta):
    """Table 1 shows rho(1) = mu_opt; the two analyses agree."""
    e = ex1_eta[5]
    assert lfa.two_grid_factor(e, 0.96, 1) == pytest.approx(lfa.smoothing_factor(e, 0.96), abs=2e-4)


def test_helmholtz_deterioration():
    """Example 3 shifts with negative real part: the smoothing factor grows
    with j (the paper reports a gradual deterioration)."""
    lam = spectral.helmholtz_shifts(128)
    h = 1.0 / 128
    mus = [lfa.smoothing_factor(l * h * h, 24 / 25, n=64) for l in lam[[0, 31, 63, 127]]]
    assert mus[0] < 0.2805
    assert all(b >= a - 1e-9 for a, b in zip(mus, mus[1:]))
    assert mus[-1] > 0.3


def test_complex_omega_optimiser():
    """eta = 0: the best complex omega is the real 24/25 with mu = 7/25
    (Sec. 2.1); for the large Example 3 shifts a complex omega lowers the
    smoothing factor below the real optimum (the paper's future-work
    suggestion after Example 3)."""
    w0, m0 = lfa.optimal_complex_omega(0.0)
    assert abs(w0 - 24 / 25) < 2e-3 and m0 == pytest.approx(7 / 25, abs=2e-3)
    lam = spectral.helmholtz_shifts(128)
    h = 1.0 / 128
    eta = lam[127] * h * h
    w, m = lfa.optimal_complex_omega(eta)
    assert abs(w.imag) > 1e-3
    assert m < lfa.smoothing_factor(eta, 24 / 25, n=64) - 0.02


def test_oracle_sweep_accepts_complex_per_system_omega():
    from oracle import operators as ops
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 7, 7)) + 1j * rng.standard_normal((2, 7, 7))
    b = rng.standard_normal((2, 7, 7)) + 1j * rng.standard_normal((2, 7, 7))
    lam = np.array([3 + 1j, -20 + 9j])
    om = np.array([0.9 + 0.1j, 1.0 - 0.2j])
    out = ops.vanka_sweep(x, b, lam, 0.125, om)
    for j in range(2):
        ref = ops.vanka_sweep(x[j:j + 1], b[j:j + 1], lam[j:j + 1], 0.125, om[j])
        np.testing.assert_allclose(out[j], ref[0], rtol=1e-15)
