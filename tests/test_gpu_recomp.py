"""Coarse-level ascents that recompute the pre-smoothed iterate (k_recomp).

A V-cycle visits each coarse level once, from zero, so the pre-smoothed
iterate is a function of that level's right-hand side: the descent stores no
iterate and the ascent rebuilds it from b before the correction and the
post-smoothing.  Every stage is the same row stencil as in the storing
descent and plain ascent, so the iterates, counts and residuals equal those
of VMG_RECOMP=0 (equal arrays: both take a zero start's residual to be b,
so a zero may differ in sign only; VMG_RECOMP=2: on every level that can; by
default only on large levels), in every precision and smoothing count
the kernel takes, on grids whose strips and runs end ragged, and in batches of
grids of different sizes; and the solves still meet the oracle.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import multigrid as omg
from paper_2203_11154_amd import inputs

pytestmark = pytest.mark.gpu

GRIDS = [dict(nx=223, ny=111, h=1.0 / 224, S=3), dict(nx=127, ny=255, h=1.0 / 128, S=2),
         dict(nx=255, ny=255, h=1.0 / 256, S=2)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.complex128))).to("cuda")


def host(t):
    return t.cpu().numpy()


def solve_both(monkeypatch, grids, nu1, nu2, precision, autotune=False, **kw):
    from paper_2203_11154_amd import Grid, VankaMG
    S = sum(g["S"] for g in grids)
    lam = np.concatenate([inputs.alpha_circulant_shifts(S - 2), inputs.uniform_shifts(2)])
    bs = [inputs.rhs(g["S"], g["ny"], g["nx"], seed=110 + k) for k, g in enumerate(grids)]
    bd = dev(np.concatenate([x.ravel() for x in bs]))
    out = {}
    for rec in ("0", "2"):
        monkeypatch.setenv("VMG_RECOMP", rec)
        gs = [Grid(g["nx"], g["ny"], h=g["h"], num_systems=g["S"], levels=5) for g in grids]
        solver = VankaMG(gs, lam, nu1=nu1, nu2=nu2, precision=precision, **kw)
        if autotune:
            solver.autotune()
        Z, iters, relres, status = solver.solve(bd, tol=1e-10)
        assert status == 0 and np.all(relres <= 1e-10)
        fixed = (np.arange(S, dtype=np.int32) % 4) + 1
        Zf, itf, rrf, _ = solver.solve(bd, fixed_iters=fixed)
        np.testing.assert_array_equal(itf, fixed)
        Za, ita, rra, _ = solver.solve(bd, tol=1e-10, conj=True)
        out[rec] = (host(Z), iters, relres, host(Zf), rrf, host(Za), ita, rra)
        del solver
    return out, bs, lam


@pytest.mark.parametrize("nu1,nu2,precision", [(2, 2, "c128"), (2, 1, "c128"), (1, 2, "c128"), (1, 1, "c128"),
                                               (2, 2, "c64_ir"), (2, 2, "c128_c64"), (1, 2, "c128_c64")])
def test_recompute_equal_stored(nu1, nu2, precision, monkeypatch):
    out, _, _ = solve_both(monkeypatch, GRIDS, nu1, nu2, precision)
    a, b = out["0"], out["2"]
    for k, (u, v) in enumerate(zip(a, b)):
        assert np.array_equal(u, v), (k, nu1, nu2, precision)


def test_recompute_autotuned_vs_oracle(monkeypatch):
    """The autotuned schedule (each level timed with the recomputing ascent)
    on one grid with three systems: the storing path's iterates, and
    every system at the oracle's V(2,2) count within 1e-10 of its iterate."""
    from paper_2203_11154_amd import Grid, VankaMG
    g = GRIDS[0]
    out, bs, lam = solve_both(monkeypatch, [g], 2, 2, "c128", autotune=True)
    a, b = out["0"], out["2"]
    for k, (u, v) in enumerate(zip(a, b)):
        assert np.array_equal(u, v), k
    zr, itr, rr, _ = omg.solve(bs[0], lam[:g["S"]], g["h"], tol=1e-10, levels=5, nu1=2, nu2=2)
    iters = b[1]
    for k in range(g["S"]):
        assert iters[k] == itr[k] or (abs(int(iters[k]) - int(itr[k])) == 1 and rr[k] > 0.95e-10)
    monkeypatch.setenv("VMG_RECOMP", "2")
    solver = VankaMG([Grid(g["nx"], g["ny"], h=g["h"], num_systems=g["S"], levels=5)], lam[:g["S"]], nu1=2, nu2=2)
    Z, _, _, _ = solver.solve(dev(bs[0].ravel()), fixed_iters=itr.astype(np.int32))
    z = host(Z).reshape(g["S"], g["ny"], g["nx"])
    for k in range(g["S"]):
        assert np.linalg.norm(z[k] - zr[k]) <= 1e-10 * np.linalg.norm(zr[k]), k
