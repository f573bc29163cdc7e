"""FP64 V-cycles whose coarse-grid correction runs in complex64 (precision
"c128_c64"): the finest level, the stopping test and the result stay in
FP64, so a solve reaches the FP64 tolerance, checked here independently of
the library (host FP64 residual, exact DST solution, the oracle's FP64
cycles)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import exact, multigrid as omg
from paper_2203_11154_amd import inputs

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.complex128))).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


GRIDS = [(255, 255, 3), (383, 191, 2), (127, 127, 2)]


def solvers(grids, monkeypatch, edge, **kw):
    from paper_2203_11154_amd import Grid, VankaMG
    monkeypatch.setenv("VMG_EDGE", edge)
    lam = inputs.alpha_circulant_shifts(sum(s for _, _, s in grids))
    gs = [Grid(nx, ny, num_systems=s) for nx, ny, s in grids]
    return (VankaMG(gs, lam, precision="c128_c64", **kw), VankaMG(gs, lam, **kw), lam)


def rhs(grids, seed):
    return [inputs.rhs(s, ny, nx, seed=seed + k) for k, (nx, ny, s) in enumerate(grids)]


@pytest.mark.parametrize("edge", ["0", "2"])
def test_mixed_solve_reaches_fp64_tolerance(edge, monkeypatch):
    mixed, fp64, lam = solvers(GRIDS, monkeypatch, edge)
    bs = rhs(GRIDS, 30)
    bd = dev(np.concatenate([b.ravel() for b in bs]))
    Z, it, rr, st = mixed.solve(bd, tol=1e-10)
    Z64, it64, rr64, st64 = fp64.solve(bd, tol=1e-10)
    assert st == 0 and st64 == 0 and np.all(rr <= 1e-10)
    # a complex64 coarse correction is accurate to ~u32 kappa_H relative, far
    # below the cycle's contraction (~0.1): the counts stay the FP64 ones, or
    # one more where the FP64 solve stopped just under the tolerance
    assert np.all(it >= it64) and np.all(it <= it64 + 1), (it, it64)
    z = host(Z)
    off = 0
    s0 = 0
    for (nx, ny, s), b in zip(GRIDS, bs):
        zg = z[off:off + nx * ny * s].reshape(s, ny, nx)
        lg = lam[s0:s0 + s]
        h = 1.0 / (nx + 1)
        # FP64 residual, computed on the host
        r = omg.residual_norms(zg, b, lg, h) / np.linalg.norm(b.reshape(s, -1), axis=1)
        assert np.all(r <= 1.01e-10), r
        if nx == ny:
            assert relerr(zg, exact.dst_solve(b, lg, h)) <= 1e-8
        off += nx * ny * s
        s0 += s


def test_mixed_cycles_against_oracle(monkeypatch):
    """At fixed cycle counts the iterate is the oracle's FP64 one up to the
    complex64 rounding of each cycle's coarse correction: the k-th iterate
    differs by at most ~k u32 kappa_H times the correction (relative 1e-5
    covers kappa_H ~ 1e2 on 255^2 with room)."""
    grids = [(255, 255, 2)]
    mixed, _, lam = solvers(grids, monkeypatch, "2")
    b = rhs(grids, 40)[0]
    h = 1.0 / 256
    for k in (1, 2, 4):
        Z, it, _, _ = mixed.solve(dev(b.ravel()), fixed_iters=np.full(2, k, np.int32))
        np.testing.assert_array_equal(it, [k, k])
        zr, _, _, _ = omg.solve(b, lam, h, fixed_iters=np.full(2, k))
        z = host(Z).reshape(2, 255, 255)
        for j in range(2):
            assert relerr(z[j], zr[j]) <= 1e-5, (k, j, relerr(z[j], zr[j]))


def test_mixed_edge_and_separate_kernels_agree(monkeypatch):
    """The cycle-edge kernel and the separate finest-level kernels at fixed
    counts, with mixed per-system counts (including zero): FP64 rounding-order
    differences reach the complex64 coarse right-hand side, whose rounding
    may then differ (relative u32 of a correction that is a fraction of the
    iterate)."""
    out = {}
    for edge in ("0", "2"):
        mixed, _, lam = solvers(GRIDS, monkeypatch, edge)
        assert [mixed.plan(g)[0] for g in range(len(GRIDS))] == [edge == "2"] * len(GRIDS)
        S = sum(s for _, _, s in GRIDS)
        bd = dev(np.concatenate([b.ravel() for b in rhs(GRIDS, 50)]))
        fi = (np.arange(S) % 4 + 1).astype(np.int32)
        fi[1] = 0
        Z, it, rr, _ = mixed.solve(bd, fixed_iters=fi)
        np.testing.assert_array_equal(it, fi)
        out[edge] = (host(Z), rr)
    z0, z2 = out["0"][0], out["2"][0]
    assert relerr(z2, z0) <= 1e-6
    np.testing.assert_allclose(out["2"][1], out["0"][1], rtol=1e-3)


def test_mixed_setup_limits():
    """V-cycles only, and finest levels the streaming kernels run."""
    from paper_2203_11154_amd import Grid, VankaMG, _lib
    lam = inputs.alpha_circulant_shifts(2)
    for kw in ({"gamma": 2}, {}):
        n = 255 if kw else 63
        with pytest.raises(_lib.VankaMGError) as e:
            VankaMG([Grid(n, num_systems=2)], lam, precision="c128_c64", **kw)
        assert e.value.code == _lib.VMG_INVALID_ARG


@pytest.mark.parametrize("conj", [False, True])
def test_mixed_paradiag_step_and_adjoint(conj):
    """The ParaDIAG step (MFMA transforms around the shifted solves) and its
    adjoint with the complex64 coarse-grid correction, against the FP64
    handle: every system stops below 1e-10 (host FP64 check of the shifted
    solves via the oracle's residual), so the two results agree to the
    solves' conditioning."""
    from paper_2203_11154_amd import Grid, VankaMG
    n, S = 255, 8
    h = 1.0 / (n + 1)
    lam = inputs.alpha_circulant_shifts(S)
    V, Vinv = inputs.alpha_circulant_vectors(S)
    F = inputs.rhs(S, n, n, seed=61)
    Vd, Vinvd, Fd = dev(V), dev(Vinv), dev(F.ravel())
    out = {}
    for prec in ("c128", "c128_c64"):
        s = VankaMG([Grid(n, num_systems=S)], lam, precision=prec)
        U, st = s.paradiag_apply(Vd, Vinvd, Fd, tol=1e-10, conj=conj)
        it, rr = s.last_stats()
        assert st == 0 and np.all(rr <= 1e-10)
        out[prec] = (host(U).reshape(S, n, n), it)
    # the shifted solves' right-hand sides and solutions, recovered on the
    # host: G = V^{-1} F, Z = V^{-1} U (adjoint: G = V^H F, Z = V^H U)
    M = V.conj().T if conj else Vinv
    G = (M @ F.reshape(S, -1)).reshape(S, n, n)
    Zm = (M @ out["c128_c64"][0].reshape(S, -1)).reshape(S, n, n)
    lj = lam.conj() if conj else lam
    r = omg.residual_norms(Zm, G, lj, h) / np.linalg.norm(G.reshape(S, -1), axis=1)
    assert np.all(r <= 2e-10), r
    assert relerr(out["c128_c64"][0], out["c128"][0]) <= 1e-7
    assert np.all(out["c128_c64"][1] <= out["c128"][1] + 1)


def test_mixed_uneven_batch():
    """Grids of different depths in one handle (their complex64 coarse cycles
    are batched per level phase): each reaches 1e-10 in FP64."""
    from paper_2203_11154_amd import Grid, VankaMG
    grids = [(511, 511, 2), (127, 127, 4), (255, 127, 3)]
    S = sum(s for _, _, s in grids)
    lam = inputs.alpha_circulant_shifts(S)
    bs = rhs(grids, 70)
    s = VankaMG([Grid(nx, ny, num_systems=k) for nx, ny, k in grids], lam, precision="c128_c64")
    Z, it, rr, st = s.solve(dev(np.concatenate([b.ravel() for b in bs])), tol=1e-10)
    assert st == 0 and np.all(rr <= 1e-10)
    z = host(Z)
    off = s0 = 0
    for (nx, ny, k), b in zip(grids, bs):
        zg = z[off:off + nx * ny * k].reshape(k, ny, nx)
        r = omg.residual_norms(zg, b, lam[s0:s0 + k], 1.0 / (nx + 1)) / np.linalg.norm(b.reshape(k, -1), axis=1)
        assert np.all(r <= 1.01e-10), (nx, ny, r)
        off += nx * ny * k
        s0 += k


def test_mixed_autotune(monkeypatch, tmp_path):
    """Autotuning a precision-2 handle (the finest level's rows among the
    streaming candidates, the complex64 levels' schedules, the edge choice)
    changes rounding only: fixed-count results agree to the complex64
    rounding of the coarse corrections, and the choices are cached under
    their own precision key."""
    from paper_2203_11154_amd import Grid, VankaMG
    monkeypatch.setenv("VMG_EDGE", "1")
    grids = [(255, 255, 3), (1023, 1023, 2)]
    S = sum(s for _, _, s in grids)
    lam = inputs.alpha_circulant_shifts(S)
    solver = VankaMG([Grid(nx, ny, num_systems=s) for nx, ny, s in grids], lam, precision="c128_c64")
    bd = dev(np.concatenate([b.ravel() for b in rhs(grids, 80)]))
    fi = np.full(S, 3, np.int32)
    Z0, _, rr0, _ = solver.solve(bd, fixed_iters=fi)
    z0 = host(Z0)
    cache = tmp_path / "tune.txt"
    solver.autotune(cache)
    assert all(solver.schedule(g)[0] > 0 for g in range(len(grids)))
    Z1, _, rr1, _ = solver.solve(bd, fixed_iters=fi)
    assert relerr(host(Z1), z0) <= 1e-5
    np.testing.assert_allclose(rr1, rr0, rtol=1e-3)
    lines = cache.read_text().splitlines()
    assert lines and all(" c128c64 " in line for line in lines)
    assert sum(1 for line in lines if " edge " in line) == len(grids)
    _, it, rr, st = solver.solve(bd, tol=1e-10)
    assert st == 0 and np.all(rr <= 1e-10)


@pytest.mark.parametrize("nu1,nu2", [(1, 1), (0, 1), (2, 1), (1, 2)])
def test_mixed_other_smoothing_counts(nu1, nu2, monkeypatch):
    """Other pre-/post-smoothing counts (with nu1 = 0 the finest level's first
    iterate is cleared by a fill instead of a sweep; the edge kernel runs for
    nu1, nu2 >= 1): fixed counts follow the oracle's FP64 cycles to complex64
    rounding, free-running solves reach 1e-10 in FP64."""
    from paper_2203_11154_amd import Grid, VankaMG
    monkeypatch.setenv("VMG_EDGE", "2")
    grids = [(255, 255, 2)]
    lam = inputs.alpha_circulant_shifts(2)
    b = rhs(grids, 90)[0]
    s = VankaMG([Grid(255, num_systems=2)], lam, precision="c128_c64", nu1=nu1, nu2=nu2)
    assert s.plan(0)[0] == (nu1 >= 1 and nu2 >= 1)
    Z, it, _, _ = s.solve(dev(b.ravel()), fixed_iters=np.full(2, 3, np.int32))
    zr, _, _, _ = omg.solve(b, lam, 1.0 / 256, fixed_iters=np.full(2, 3), nu1=nu1, nu2=nu2)
    z = host(Z).reshape(2, 255, 255)
    for j in range(2):
        assert relerr(z[j], zr[j]) <= 1e-5, (j, relerr(z[j], zr[j]))
    Z, it, rr, st = s.solve(dev(b.ravel()), tol=1e-10)
    assert st == 0 and np.all(rr <= 1e-10)
    r = omg.residual_norms(host(Z).reshape(2, 255, 255), b, lam, 1.0 / 256) / np.linalg.norm(b.reshape(2, -1), axis=1)
    assert np.all(r <= 1.01e-10)


def test_mixed_circulant_step():
    """The alpha-circulant ParaDIAG step with DFT transforms (the norm sums of
    the transformed right-hand sides fused into the forward transform) with
    the complex64 coarse-grid correction: every system below 1e-10, the
    result within 1e-7 of the FP64 handle's."""
    from paper_2203_11154_amd import Grid, VankaMG
    n, S, alpha = 255, 16, 0.01
    lam = inputs.alpha_circulant_shifts(S, alpha)
    Fd = dev(inputs.rhs(S, n, n, seed=62).ravel())
    out = {}
    for prec in ("c128", "c128_c64"):
        s = VankaMG([Grid(n, num_systems=S)], lam, precision=prec)
        U, st = s.paradiag_apply_circulant(alpha, Fd, tol=1e-10)
        it, rr = s.last_stats()
        assert st == 0 and np.all(rr <= 1e-10)
        out[prec] = host(U)
    assert relerr(out["c128_c64"], out["c128"]) <= 1e-7
