"""Differentiation through the HIP path: adjoint (conjugate-shift) solves give
gradients with respect to the right-hand sides, the shifts and the heat
source parameters, checked against the oracle, closed forms and central
finite differences."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import exact, paradiag as opd, spectral
from paper_2203_11154_amd import inputs

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.complex128))).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def test_shifted_solve_gradients():
    from paper_2203_11154_amd import Grid, VankaMG
    from paper_2203_11154_amd.autograd import ShiftedSolve
    n, S = 31, 4
    h = 1.0 / (n + 1)
    lam = inputs.alpha_circulant_shifts(S) + np.array([0, 5j, -3j, 2])
    b = inputs.rhs(S, n, n, seed=31)
    y = inputs.rhs(S, n, n, seed=32)
    solver = VankaMG([Grid(n, num_systems=S)], lam)
    bt = dev(b.ravel()).requires_grad_(True)
    lt = dev(lam).requires_grad_(True)
    z = ShiftedSolve.apply(bt, lt, solver, 1e-13)
    loss = ((z - dev(y.ravel())).abs() ** 2).sum()
    loss.backward()
    # oracle: g = dL/dconj(z) convention -> 2 (z - y); grad_b = L^{-H} g
    zr = exact.dst_solve(b, lam, h)
    g = 2 * (zr - y)
    gb = exact.dst_solve(g, np.conj(lam), h)
    glam = -np.sum(np.conj(zr) * gb, axis=(1, 2))
    np.testing.assert_allclose(host(bt.grad).reshape(S, n, n), gb, rtol=1e-9, atol=1e-12 * np.abs(gb).max())
    np.testing.assert_allclose(host(lt.grad), glam, rtol=1e-8)

    # central differences on Re and Im of one shift: grad = dL/dRe + i dL/dIm
    def loss_at(lmb):
        s = VankaMG([Grid(n, num_systems=S)], lmb)
        zz, _, _, _ = s.solve(dev(b.ravel()), tol=1e-13)
        return float(((zz - dev(y.ravel())).abs() ** 2).sum())
    j, d = 1, 1e-4
    e = np.zeros(S, dtype=complex)
    e[j] = d
    dre = (loss_at(lam + e) - loss_at(lam - e)) / (2 * d)
    dim = (loss_at(lam + 1j * e) - loss_at(lam - 1j * e)) / (2 * d)
    got = host(lt.grad)[j]
    assert abs(got - (dre + 1j * dim)) <= 1e-6 * abs(got)


@pytest.mark.parametrize("precision", ["c128", "c128_c64"])
def test_set_shifts_in_place_equals_fresh_setup(precision):
    """New shifts taken in place (vanka_mg_set_shifts) give bitwise the
    solves of a handle set up with them, free-running and replayed from the
    graphs captured under the old shifts; a shift that makes a coarsest
    matrix singular is refused and the previous shifts stay in force."""
    from paper_2203_11154_amd import Grid, VankaMG, _lib
    n, S = 127, 4
    lam1 = inputs.alpha_circulant_shifts(S)
    lam2 = inputs.uniform_shifts(S, seed=41)
    bd = dev(inputs.rhs(S, n, n, seed=40).ravel())
    s = VankaMG([Grid(n, num_systems=S)], lam1, precision=precision)
    Z1, it1, _, _ = s.solve(bd, tol=1e-10)
    Z1, it1, _, _ = s.solve(bd, tol=1e-10, out=Z1)  # (graphs of the old shifts captured)
    s.set_shifts(lam2)
    fresh = VankaMG([Grid(n, num_systems=S)], lam2, precision=precision)
    for _ in range(2):
        Za, ita, _, _ = s.solve(bd, tol=1e-10)
        Zb, itb, _, _ = fresh.solve(bd, tol=1e-10)
        np.testing.assert_array_equal(ita, itb)
        assert torch.equal(Za, Zb)
        Za, _, _, _ = s.solve(bd, fixed_iters=itb, stats=False)
        Zb, _, _, _ = fresh.solve(bd, fixed_iters=itb, stats=False)
        assert torch.equal(Za, Zb)
    # back to the first shifts: the first solve again
    s.set_shifts(lam1)
    Z3, it3, _, _ = s.solve(bd, tol=1e-10)
    np.testing.assert_array_equal(it3, it1)
    assert torch.equal(Z3, Z1)
    # coarsest grid 1 x 1 with h = 0.5: A_c + lambda = 16 + lambda
    t = VankaMG([Grid(3, h=0.25, num_systems=1, levels=2)], np.array([1.0 + 1j]))
    b3 = dev(inputs.rhs(1, 3, 3, seed=42).ravel())
    Zt, _, _, _ = t.solve(b3, tol=1e-12)
    with pytest.raises(_lib.VankaMGError) as e:
        t.set_shifts(np.array([-16.0 + 0j]))
    assert e.value.code == _lib.VMG_SINGULAR
    Zt2, _, _, _ = t.solve(b3, tol=1e-12)
    assert torch.equal(Zt, Zt2)


def test_shift_gradient_steps_through_new_shifts():
    """ShiftedSolve with shifts that change between calls: the solver takes
    each new lambda in place, and value and gradient equal those of a solver
    set up with that lambda."""
    from paper_2203_11154_amd import Grid, VankaMG
    from paper_2203_11154_amd.autograd import ShiftedSolve
    n, S = 63, 3
    lam = inputs.alpha_circulant_shifts(S)
    b = dev(inputs.rhs(S, n, n, seed=43).ravel())
    y = dev(inputs.rhs(S, n, n, seed=44).ravel())
    solver = VankaMG([Grid(n, num_systems=S)], lam)
    lt = dev(lam)
    for step in range(3):
        lt = lt.detach().requires_grad_(True)
        loss = ((ShiftedSolve.apply(b, lt, solver, 1e-12) - y).abs() ** 2).sum()
        loss.backward()
        ref = VankaMG([Grid(n, num_systems=S)], host(lt))
        lr = lt.detach().clone().requires_grad_(True)
        loss_r = ((ShiftedSolve.apply(b, lr, ref, 1e-12) - y).abs() ** 2).sum()
        loss_r.backward()
        assert float(loss.detach()) == float(loss_r.detach()), step
        assert torch.equal(lt.grad, lr.grad), step
        lt = lt - 0.5 * lt.grad / lt.grad.abs().max()


def test_paradiag_gradient_matches_adjoint():
    from paper_2203_11154_amd import Grid, VankaMG
    from paper_2203_11154_amd.autograd import ParaDiag
    nt, nx = 8, 31
    h = 1.0 / (nx + 1)
    lam = inputs.alpha_circulant_shifts(nt)
    V, Vinv = inputs.alpha_circulant_vectors(nt)
    rng = np.random.default_rng(4)
    F = rng.standard_normal((nt, nx, nx)) + 1j * rng.standard_normal((nt, nx, nx))
    Y = rng.standard_normal((nt, nx, nx)) + 1j * rng.standard_normal((nt, nx, nx))
    solver = VankaMG([Grid(nx, num_systems=nt)], lam)
    Ft = dev(F.ravel()).requires_grad_(True)
    U = ParaDiag.apply(Ft, solver, dev(V), dev(Vinv), 1e-13)
    loss = ((U - dev(Y.ravel())).abs() ** 2).sum()
    loss.backward()
    Ur = opd.paradiag_apply(F, lam, V, Vinv, h, solver="dst")
    g = 2 * (Ur - Y)
    gF = opd.paradiag_apply(g, np.conj(lam), Vinv.conj().T, V.conj().T, h, solver="dst")
    np.testing.assert_allclose(host(Ft.grad).reshape(F.shape), gF, rtol=1e-8, atol=1e-10 * np.abs(gF).max())


def heat_setup(nx, n, K, alpha=0.01):
    from paper_2203_11154_amd.autograd import HeatProblem
    tau = 1.0 / n
    lam = inputs.alpha_circulant_shifts(n, alpha)
    V, Vinv = inputs.alpha_circulant_vectors(n, alpha)
    prob = HeatProblem(nx, n, tau, lam, V, Vinv, tol=1e-10, inner_tol=1e-12)
    xs = np.arange(1, nx + 1) / (nx + 1)
    basis = np.stack([np.outer(np.sin(k * np.pi * xs), np.sin(k * np.pi * xs)) for k in range(1, K + 1)])
    tdecay = np.exp(-tau * np.arange(1, n + 1))
    return prob, torch.from_numpy(basis).cuda(), torch.from_numpy(tdecay).cuda(), tau


def heat_source(theta, basis, tdecay):
    """f^m = sum_k theta_k sin(k pi x) sin(k pi y) exp(-t_m) (real), as complex128."""
    spatial = torch.tensordot(theta, basis, dims=1)
    return (tdecay[:, None, None] * spatial[None]).to(torch.complex128).reshape(-1)


@pytest.mark.parametrize("nx,n", [(63, 16), (511, 128)])
def test_heat_gradient_closed_form(nx, n):
    """Full ParaDIAG-II heat pipeline: u from the preconditioned iteration,
    L = sum (u - u*)^2, dL/dtheta by the adjoint (transposed) iteration; both
    against the closed-form backward-Euler mode recurrence."""
    from paper_2203_11154_amd.autograd import HeatSolve
    K = 16
    prob, basis, tdecay, tau = heat_setup(nx, n, K)
    theta_np = inputs.heat_parameters(K)
    theta_star = inputs.heat_parameters(K, seed=inputs.SEED_THETA_STAR)
    c = opd.heat_mode_coefficients(n, nx, tau)[:K]
    ustar = np.einsum("k,km,kij->mij", theta_star, c, basis.cpu().numpy())
    theta = torch.from_numpy(theta_np).cuda().requires_grad_(True)
    u = HeatSolve.apply(heat_source(theta, basis, tdecay), prob)
    assert prob.last["relres"] <= 1e-10 and prob.last["outer"] <= 8
    loss = ((u.real - torch.from_numpy(ustar.ravel()).cuda()) ** 2).sum()
    loss.backward()
    L_cf, g_cf = opd.heat_loss_closed_form(theta_np, theta_star, n, nx, tau)
    # u meets ||f - K u|| <= 1e-10 ||f||; the error in u, and so in L and its
    # gradient, is that residual times the conditioning of K
    assert float(loss.detach()) == pytest.approx(L_cf, rel=1e-6)
    np.testing.assert_allclose(theta.grad.cpu().numpy(), g_cf, rtol=1e-6)


@pytest.mark.parametrize("nx,n", [(127, 32), (511, 128)])
def test_heat_gradient_finite_differences(nx, n):
    """Central differences with step 1e-6 on frozen iteration counts (the
    solve is then one fixed linear map of f, so the quadratic loss has no
    truncation error) against the adjoint gradient, on a small grid and on
    the differentiation workload's own 511^2 x 128."""
    from paper_2203_11154_amd.autograd import HeatSolve
    K = 16
    prob, basis, tdecay, tau = heat_setup(nx, n, K)
    theta_np = inputs.heat_parameters(K)
    theta_star = inputs.heat_parameters(K, seed=inputs.SEED_THETA_STAR)
    ustar = HeatSolve.apply(heat_source(torch.from_numpy(theta_star).cuda(), basis, tdecay), prob).real.clone()
    theta = torch.from_numpy(theta_np).cuda().requires_grad_(True)
    u = HeatSolve.apply(heat_source(theta, basis, tdecay), prob)   # records the counts
    loss = ((u.real - ustar) ** 2).sum()
    loss.backward()
    grad = theta.grad.cpu().numpy()
    step = 1e-6
    for k in (0, 5, 15):
        e = torch.zeros(K, dtype=torch.float64, device="cuda")
        e[k] = step
        lp = float(((HeatSolve.apply(heat_source(theta.detach() + e, basis, tdecay), prob, True).real - ustar) ** 2).sum())
        lm = float(((HeatSolve.apply(heat_source(theta.detach() - e, basis, tdecay), prob, True).real - ustar) ** 2).sum())
        fd = (lp - lm) / (2 * step)
        print(f"{nx}^2 x {n}: dL/dtheta_{k} adjoint {grad[k]:.10e}, central difference {fd:.10e}, "
              f"rel. diff {abs(fd - grad[k]) / abs(grad[k]):.2e}")
        assert fd == pytest.approx(grad[k], rel=1e-5, abs=1e-9 * np.abs(grad).max())
