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
