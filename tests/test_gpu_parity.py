"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Single operations are compared element by element at sizes that span several
tiles and a ragged tail; full solves at fixed iteration counts must agree to
1e-10 relative (the FP64 bar), free-running solves must reach the tolerance
with the oracle's iteration counts.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import exact, multigrid as omg, operators as ops, paradiag as opd
from paper_2203_11154_amd import inputs

pytestmark = pytest.mark.gpu

OMEGA = 24.0 / 25.0


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.complex128))).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(np.asarray(b).ravel()), 1e-300))


def maxrel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def two_grids():
    """A 95 x 47 rectangle (h = 1/96, 3 systems) and a 63 x 63 square (2
    systems), both with 4 levels: tiles of 64 x 16 leave ragged tails."""
    from paper_2203_11154_amd import Grid, VankaMG
    grids = [Grid(95, 47, h=1.0 / 96, num_systems=3, levels=4), Grid(63, 63, num_systems=2, levels=4)]
    lam = np.concatenate([inputs.alpha_circulant_shifts(3), inputs.uniform_shifts(2)])
    solver = VankaMG(grids, lam)
    return solver, grids, lam


def level_geom(g, level):
    nx, ny, h = g.nx, g.ny, g.h
    for _ in range(level):
        nx, ny, h = (nx - 1) // 2, (ny - 1) // 2, 2 * h
    return nx, ny, h


def split(vec, grids, level, coarse=False):
    out, off = [], 0
    for g in grids:
        nx, ny, _ = level_geom(g, level + (1 if coarse else 0))
        n = nx * ny * g.num_systems
        out.append(vec[off:off + n].reshape(g.num_systems, ny, nx))
        off += n
    return out


def random_level(grids, level, seed, coarse=False):
    rng = np.random.default_rng(seed)
    arrs = []
    for g in grids:
        nx, ny, _ = level_geom(g, level + (1 if coarse else 0))
        arrs.append(rng.uniform(-1, 1, (g.num_systems, ny, nx)) + 1j * rng.uniform(-1, 1, (g.num_systems, ny, nx)))
    return arrs


def group_shifts(grids, lam):
    out, off = [], 0
    for g in grids:
        out.append(lam[off:off + g.num_systems])
        off += g.num_systems
    return out


@pytest.mark.parametrize("level", [0, 1, 2])
@pytest.mark.parametrize("x_zero", [False, True])
@pytest.mark.parametrize("conj", [False, True])
def test_sweep_parity(two_grids, level, x_zero, conj):
    from paper_2203_11154_amd import _lib
    solver, grids, lam = two_grids
    xs = random_level(grids, level, 1)
    bs = random_level(grids, level, 2)
    x = None if x_zero else dev(np.concatenate([a.ravel() for a in xs]))
    out = host(solver.apply_op(_lib.OP_SWEEP, level, dev(np.concatenate([a.ravel() for a in bs])), x, conj=conj))
    for g, lg, xa, ba, got in zip(grids, group_shifts(grids, lam), xs, bs, split(out, grids, level)):
        _, _, h = level_geom(g, level)
        lg = np.conj(lg) if conj else lg
        ref = ops.vanka_sweep(np.zeros_like(xa) if x_zero else xa, ba, lg, h, OMEGA)
        assert maxrel(got, ref) <= 1e-13


@pytest.mark.parametrize("level", [0, 2])
def test_residual_and_restriction_parity(two_grids, level):
    from paper_2203_11154_amd import _lib
    solver, grids, lam = two_grids
    xs = random_level(grids, level, 3)
    bs = random_level(grids, level, 4)
    xd = dev(np.concatenate([a.ravel() for a in xs]))
    bd = dev(np.concatenate([a.ravel() for a in bs]))
    r = host(solver.apply_op(_lib.OP_RESIDUAL, level, bd, xd))
    ncoarse = sum(np.prod(level_geom(g, level + 1)[:2]) * g.num_systems for g in grids)
    rc = host(solver.apply_op(_lib.OP_RESTRICT_RESIDUAL, level, bd, xd, out_numel=int(ncoarse)))
    for g, lg, xa, ba, gr, grc in zip(grids, group_shifts(grids, lam), xs, bs, split(r, grids, level),
                                      split(rc, grids, level, coarse=True)):
        _, _, h = level_geom(g, level)
        ref = ops.residual(xa, ba, lg, h)
        # b - L x cancels: compare against the size of the terms, |L x|
        scale = np.max(np.abs(ops.apply_shifted_laplacian(xa, lg, h)))
        assert np.max(np.abs(gr - ref)) <= 1e-14 * scale
        refc = ops.restrict_full_weighting(ref)
        assert np.max(np.abs(grc - refc)) <= 1e-14 * scale


@pytest.mark.parametrize("level", [0, 1, 2])
def test_prolongation_parity(two_grids, level):
    from paper_2203_11154_amd import _lib
    solver, grids, lam = two_grids
    xs = random_level(grids, level, 5)
    es = random_level(grids, level, 6, coarse=True)
    xd = dev(np.concatenate([a.ravel() for a in xs]))
    out = host(solver.apply_op(_lib.OP_PROLONG_CORRECT, level, dev(np.concatenate([a.ravel() for a in es])), xd,
                               out_numel=xd.numel()))
    for xa, ea, got in zip(xs, es, split(out, grids, level)):
        ref = xa + ops.prolong_bilinear(ea)
        assert maxrel(got, ref) <= 1e-15


def test_coarse_solve_parity(two_grids):
    from paper_2203_11154_amd import _lib
    solver, grids, lam = two_grids
    level = 3
    bs = random_level(grids, level, 7)
    out = host(solver.apply_op(_lib.OP_COARSE_SOLVE, level, dev(np.concatenate([a.ravel() for a in bs]))))
    for g, lg, ba, got in zip(grids, group_shifts(grids, lam), bs, split(out, grids, level)):
        _, _, h = level_geom(g, level)
        ref = exact.dense_solve(ba, lg, h)
        assert maxrel(got, ref) <= 1e-12


@pytest.mark.parametrize("level", [0, 1])
def test_cycle_parity(two_grids, level):
    from paper_2203_11154_amd import _lib
    solver, grids, lam = two_grids
    xs = random_level(grids, level, 8)
    bs = random_level(grids, level, 9)
    out = host(solver.apply_op(_lib.OP_CYCLE, level, dev(np.concatenate([a.ravel() for a in bs])),
                               dev(np.concatenate([a.ravel() for a in xs]))))
    for g, lg, xa, ba, got in zip(grids, group_shifts(grids, lam), xs, bs, split(out, grids, level)):
        nx, ny, h = level_geom(g, level)
        shapes = ops.level_shapes(nx, ny, h, levels=4 - level)
        ref = omg.mg_cycle(0, xa, ba, lg, shapes)
        assert maxrel(got, ref) <= 1e-12


def test_sweep_on_sine_mode_matches_symbol():
    """One GPU sweep maps phi_kl to S~(k pi h, l pi h) phi_kl (eq. (7))."""
    from paper_2203_11154_amd import Grid, VankaMG, _lib
    n, k, l = 127, 5, 77
    h = 1.0 / (n + 1)
    lam = np.array([40.0 + 300.0j])
    solver = VankaMG([Grid(n, num_systems=1)], lam)
    phi = exact.sine_mode(k, l, n, n)[None].astype(np.complex128)
    out = host(solver.apply_op(_lib.OP_SWEEP, 0, dev(np.zeros_like(phi)), dev(phi))).reshape(1, n, n)
    t1, t2, eta = k * np.pi * h, l * np.pi * h, lam[0] * h * h
    a, b, c = ops.vanka_abc_paper(eta)
    s = 1 - OMEGA * (a + b * np.cos(t1) + b * np.cos(t2) + c * np.cos(t1) * np.cos(t2)) * (
        4 + eta - 2 * np.cos(t1) - 2 * np.cos(t2))
    assert np.max(np.abs(out - s * phi)) <= 1e-13


def test_plain_small_workload_parity():
    """63 x 63, 8 alpha-circulant shifts, V(2,2), 5 levels, tol 1e-10."""
    from paper_2203_11154_amd import Grid, VankaMG
    n = 63
    h = 1.0 / 64
    lam = inputs.alpha_circulant_shifts(8)
    b = inputs.rhs(8, n, n)
    z_or, it_or, rr_or, _ = omg.solve(b, lam, h, tol=1e-10, levels=5)
    solver = VankaMG([Grid(n, num_systems=8, levels=5)], lam)
    Z, iters, relres, status = solver.solve(dev(b.ravel()), tol=1e-10)
    assert status == 0
    # the oracle's final residuals are well inside tol here (< 0.2 tol), so the
    # counts must agree exactly
    assert np.all(rr_or < 0.5e-10)
    np.testing.assert_array_equal(iters, it_or)
    # at 1e-11 the residual b - L z is a cancellation of O(1) terms: its
    # rounding (~eps |L z| / |r| ~ 1e-5 relative) differs between the two
    # summation orders
    np.testing.assert_allclose(relres, rr_or, rtol=1e-3)
    z = host(Z).reshape(8, n, n)
    for j in range(8):
        assert relerr(z[j], z_or[j]) <= 1e-10
    # fixed iteration counts: same number of cycles as the oracle
    Z2, it2, _, _ = solver.solve(dev(b.ravel()), fixed_iters=it_or)
    np.testing.assert_array_equal(it2, it_or)
    assert relerr(host(Z2).reshape(8, n, n), z_or) <= 1e-12


def test_multi_grid_solve_parity(two_grids):
    solver, grids, lam = two_grids
    bs = random_level(grids, 0, 11)
    Z, iters, relres, status = solver.solve(dev(np.concatenate([a.ravel() for a in bs])), tol=1e-10)
    assert status == 0 and np.all(relres <= 1e-10)
    zs = split(host(Z), grids, 0)
    off = 0
    for g, lg, ba, got in zip(grids, group_shifts(grids, lam), bs, zs):
        zr, itr, rr, _ = omg.solve(ba, lg, g.h, tol=1e-10, levels=4)
        for a, w, r in zip(iters[off:off + g.num_systems], itr, rr):
            # equal counts unless the oracle stopped within 5% of tol
            assert a == w or (abs(int(a) - int(w)) == 1 and r > 0.95e-10)
        off += g.num_systems
    counts = np.concatenate([omg.solve(ba, lg, g.h, tol=1e-10, levels=4)[1]
                             for g, lg, ba in zip(grids, group_shifts(grids, lam), bs)])
    Z2, _, _, _ = solver.solve(dev(np.concatenate([a.ravel() for a in bs])), fixed_iters=counts)
    for g, lg, ba, got in zip(grids, group_shifts(grids, lam), bs, split(host(Z2), grids, 0)):
        zr, _, _, _ = omg.solve(ba, lg, g.h, tol=1e-10, levels=4)
        for j in range(g.num_systems):
            assert relerr(got[j], zr[j]) <= 1e-10


def test_conjugate_solve_and_adjoint_identity():
    """conj=True solves (A + conj(lambda) I) z = b; <L^{-1} b, g> = <b, L^{-H} g>."""
    from paper_2203_11154_amd import Grid, VankaMG
    n = 63
    h = 1.0 / 64
    lam = inputs.alpha_circulant_shifts(4) + 3j
    solver = VankaMG([Grid(n, num_systems=4)], lam)
    b = inputs.rhs(4, n, n, seed=21)
    g = inputs.rhs(4, n, n, seed=22)
    z, _, rr, _ = solver.solve(dev(b.ravel()), tol=1e-12)
    w, _, rr2, _ = solver.solve(dev(g.ravel()), tol=1e-12, conj=True)
    z, w = host(z).reshape(4, n, n), host(w).reshape(4, n, n)
    ref = exact.dst_solve(g, np.conj(lam), h)
    assert relerr(w, ref) <= 1e-9
    for j in range(4):
        lhs = np.vdot(g[j], z[j])
        rhs = np.vdot(w[j], b[j])
        assert abs(lhs - rhs) <= 1e-9 * abs(lhs)


def test_refinement_precision_reaches_fp64_tolerance():
    """complex64 cycles inside FP64 refinement: same final residual bar as the
    FP64 solve, and the same solution to within the conditioning."""
    from paper_2203_11154_amd import Grid, VankaMG
    n = 127
    h = 1.0 / 128
    lam = inputs.alpha_circulant_shifts(8)
    b = inputs.rhs(8, n, n)
    solver = VankaMG([Grid(n, num_systems=8)], lam, precision="c64_ir")
    Z, iters, relres, status = solver.solve(dev(b.ravel()), tol=1e-10)
    assert status == 0 and np.all(relres <= 1e-10)
    z = host(Z).reshape(8, n, n)
    zx = exact.dst_solve(b, lam, h)
    # FP64 residual check independent of the library
    r = omg.residual_norms(z, b, lam, h) / np.linalg.norm(b.reshape(8, -1), axis=1)
    assert np.all(r <= 1.01e-10)
    assert relerr(z, zx) <= 1e-8


def test_transform_parity():
    from paper_2203_11154_amd import transform
    rng = np.random.default_rng(5)
    # n = 8, 16, 32, 64 take the register-resident kernel (ragged node tails
    # included), the others the LDS-chunked one; for n <= 32 the long rows
    # (m = 100003, 200001, 300007: rows that start off cache lines) give each
    # block a run of several tiles, whose stores into a line that the next
    # tile completes wait for that tile
    for n, m in [(8, 1), (8, 100003), (13, 100), (16, 33), (16, 200001), (32, 1000), (32, 300007), (64, 31),
                 (64, 4097), (128, 3000), (200, 777)]:
        M = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        F = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
        G = host(transform(dev(M), dev(F)))
        assert maxrel(G.reshape(n, m), M @ F) <= 1e-13
        GH = host(transform(dev(M), dev(F), trans_conj=True))
        assert maxrel(GH.reshape(n, m), M.conj().T @ F) <= 1e-13


def test_transform_calls_on_two_streams():
    """paradiag_transform keeps its expanded matrix in one library buffer per
    device: calls on two streams, the second growing that buffer (larger n)
    and a third reusing it while the others may still run, all give their own
    products."""
    from paper_2203_11154_amd import transform
    rng = np.random.default_rng(17)
    cases = [(64, 200003), (128, 50001), (64, 100001)]
    data = []
    for n, m in cases:
        M = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        F = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
        data.append((M, F, dev(M), dev(F)))
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()]
    outs = []
    for (M, F, Md, Fd), st in zip(data, streams):
        with torch.cuda.stream(st):
            outs.append(transform(Md, Fd))
    torch.cuda.synchronize()
    for (M, F, _, _), G in zip(data, outs):
        assert maxrel(G.cpu().numpy().reshape(F.shape), M @ F) <= 1e-13


@pytest.mark.parametrize("conj", [False, True])
def test_paradiag_apply_parity(conj):
    from paper_2203_11154_amd import Grid, VankaMG
    n_t, nx = 16, 31
    h = 1.0 / (nx + 1)
    lam = inputs.alpha_circulant_shifts(n_t)
    V, Vinv = inputs.alpha_circulant_vectors(n_t)
    rng = np.random.default_rng(9)
    F = rng.standard_normal((n_t, nx, nx)) + 1j * rng.standard_normal((n_t, nx, nx))
    solver = VankaMG([Grid(nx, num_systems=n_t)], lam)
    U, status = solver.paradiag_apply(dev(V), dev(Vinv), dev(F.ravel()), tol=1e-12, conj=conj)
    if conj:
        ref = opd.paradiag_apply(F, np.conj(lam), np.linalg.inv(V.conj().T), V.conj().T, h, solver="dst")
    else:
        ref = opd.paradiag_apply(F, lam, V, Vinv, h, solver="dst")
    assert relerr(host(U).reshape(F.shape), ref) <= 1e-9


def test_error_paths():
    from paper_2203_11154_amd import Grid, VankaMG, _lib
    with pytest.raises(_lib.VankaMGError) as e:
        VankaMG([Grid(64, num_systems=1)], np.array([1.0 + 0j]))
    assert e.value.code == _lib.VMG_INVALID_ARG
    with pytest.raises(_lib.VankaMGError) as e:
        # coarsest grid 1 x 1 with h = 0.5: A_c + lambda = 4/0.25 + lambda = 0
        VankaMG([Grid(3, h=0.25, num_systems=1, levels=2)], np.array([-16.0 + 0j]))
    assert e.value.code == _lib.VMG_SINGULAR
    s = VankaMG([Grid(31, num_systems=2)], np.array([1 + 1j, 2 + 2j]), max_iter=1)
    b = inputs.rhs(2, 31, 31)
    _, it, rr, status = s.solve(dev(b.ravel()), tol=1e-10)
    assert status == _lib.VMG_NOT_CONVERGED and list(it) == [1, 1]
    b[0, 3, 4] = np.nan
    s2 = VankaMG([Grid(31, num_systems=2)], np.array([1 + 1j, 2 + 2j]))
    with pytest.raises(_lib.VankaMGError) as e:
        s2.solve(dev(b.ravel()))
    assert e.value.code == _lib.VMG_NAN_DETECTED


def test_zero_rhs_and_determinism():
    from paper_2203_11154_amd import Grid, VankaMG
    n = 63
    lam = inputs.alpha_circulant_shifts(4)
    b = inputs.rhs(4, n, n)
    b[2] = 0
    s = VankaMG([Grid(n, num_systems=4)], lam)
    Z1, it1, _, _ = s.solve(dev(b.ravel()))
    Z2, it2, _, _ = s.solve(dev(b.ravel()))
    assert it1[2] == 0 and np.all(host(Z1).reshape(4, n, n)[2] == 0)
    assert torch.equal(Z1, Z2) and list(it1) == list(it2)
