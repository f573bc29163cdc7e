"""Whole solves in one tail launch: where every level of every grid runs in
the tail kernel (one workgroup per system), a solve's cycles and their
stopping tests run inside one launch.  Checked against the same solves with
one launch and one stopping test a cycle (VMG_TAIL_SOLVE=0, the path the
larger grids take): fixed counts (zero included) give bitwise the same
iterates, free-running solves the same counts and residuals to rounding; and
against the oracle at its counts."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import multigrid as omg
from paper_2203_11154_amd import inputs

pytestmark = pytest.mark.gpu

GRIDS = [(63, 63, 4, 5), (63, 31, 3, 4)]  # nx, ny, systems, levels


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.complex128)).ravel()).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def make(monkeypatch, whole, **kw):
    from paper_2203_11154_amd import Grid, VankaMG
    monkeypatch.setenv("VMG_TAIL_SOLVE", "1" if whole else "0")
    S = sum(c for _, _, c, _ in GRIDS)
    lam = np.concatenate([inputs.alpha_circulant_shifts(4), inputs.uniform_shifts(3)])
    s = VankaMG([Grid(nx, ny, num_systems=c, levels=lv) for nx, ny, c, lv in GRIDS], lam, **kw)
    for g in range(len(GRIDS)):
        assert s.plan(g)[1] == 0, (g, s.plan(g))
    return s, lam, S


@pytest.mark.parametrize("nu1,nu2,gamma", [(2, 2, 1), (1, 1, 2), (1, 0, 2)])
def test_whole_solve_equals_cycle_by_cycle(nu1, nu2, gamma, monkeypatch):
    b = np.concatenate([inputs.rhs(c, ny, nx, seed=110 + k).ravel() for k, (nx, ny, c, _) in enumerate(GRIDS)])
    bd = dev(b)
    fixed = np.array([3, 0, 5, 1, 2, 0, 4], np.int32)
    res = {}
    for whole in (True, False):
        s, lam, S = make(monkeypatch, whole, nu1=nu1, nu2=nu2, gamma=gamma)
        out = {}
        for conj in (False, True):
            Z, it, rr, st = s.solve(bd, tol=1e-10, conj=conj)
            assert st == 0 and np.all(rr <= 1e-10)
            Zf, itf, _, stf = s.solve(bd, fixed_iters=fixed, conj=conj)
            assert stf == 0
            np.testing.assert_array_equal(itf, fixed)
            Za, _, _, _ = s.solve(bd, fixed_iters=fixed, conj=conj, stats=False)
            out[conj] = (host(Z), it, rr, host(Zf), host(Za))
        res[whole] = out
        del s
    for conj in (False, True):
        z1, it1, rr1, zf1, za1 = res[True][conj]
        z0, it0, rr0, zf0, za0 = res[False][conj]
        assert np.array_equal(zf1, zf0) and np.array_equal(za1, za0) and np.array_equal(za1, zf1)
        np.testing.assert_array_equal(it1, it0)
        assert np.array_equal(z1, z0)
        np.testing.assert_allclose(rr1, rr0, rtol=1e-12)


def test_whole_solve_against_oracle(monkeypatch):
    s, lam, S = make(monkeypatch, True)
    bs = [inputs.rhs(c, ny, nx, seed=120 + k) for k, (nx, ny, c, _) in enumerate(GRIDS)]
    Z, it, rr, st = s.solve(dev(np.concatenate([b.ravel() for b in bs])), tol=1e-10)
    assert st == 0
    z = host(Z)
    off, s0 = 0, 0
    for (nx, ny, c, lv), b in zip(GRIDS, bs):
        zr, itr, rrr, _ = omg.solve(b, lam[s0:s0 + c], 1.0 / (nx + 1), tol=1e-10, levels=lv)
        for k in range(c):
            assert it[s0 + k] == itr[k] or (abs(int(it[s0 + k]) - int(itr[k])) == 1 and rrr[k] > 0.95e-10)
            if it[s0 + k] == itr[k]:
                zg = z[off + k * nx * ny:off + (k + 1) * nx * ny].reshape(ny, nx)
                assert np.linalg.norm(zg - zr[k]) <= 1e-10 * np.linalg.norm(zr[k])
        off += nx * ny * c
        s0 += c
