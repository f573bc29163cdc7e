"""Parity of the fused streaming level kernels (used on levels at least 96
nodes wide) with the oracle's cycle, for every smoothing-count combination
they implement, V- and W-cycles, several column tiles, several row strips and
ragged tails."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import exact, multigrid as omg, operators as ops
from paper_2203_11154_amd import inputs

pytestmark = pytest.mark.gpu

# 223 x 111 (h = 1/224): levels 223x111 and 111x55 are streamed (5 column
# tiles, ragged); 127 x 255 (h = 1/128): level 0 streamed with two row strips.
GRIDS = [dict(nx=223, ny=111, h=1.0 / 224, S=2), dict(nx=127, ny=255, h=1.0 / 128, S=2)]
LEVELS = 5


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.complex128))).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def maxrel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def make(nu1, nu2, gamma=1):
    from paper_2203_11154_amd import Grid, VankaMG
    grids = [Grid(g["nx"], g["ny"], h=g["h"], num_systems=g["S"], levels=LEVELS) for g in GRIDS]
    lam = np.concatenate([inputs.alpha_circulant_shifts(2), inputs.uniform_shifts(2)])
    return VankaMG(grids, lam, nu1=nu1, nu2=nu2, gamma=gamma), lam


def split_shifts(lam):
    out, off = [], 0
    for g in GRIDS:
        out.append(lam[off:off + g["S"]])
        off += g["S"]
    return out


@pytest.mark.parametrize("nu1,nu2,gamma", [(2, 2, 1), (1, 1, 1), (1, 0, 2), (0, 2, 1), (2, 1, 2)])
@pytest.mark.parametrize("with_x", [True, False])
def test_streamed_cycle_parity(nu1, nu2, gamma, with_x):
    from paper_2203_11154_amd import _lib
    solver, lam = make(nu1, nu2, gamma)
    rng = np.random.default_rng(nu1 * 10 + nu2 + 100 * gamma)
    xs, bs = [], []
    for g in GRIDS:
        shape = (g["S"], g["ny"], g["nx"])
        xs.append(rng.uniform(-1, 1, shape) + 1j * rng.uniform(-1, 1, shape))
        bs.append(rng.uniform(-1, 1, shape) + 1j * rng.uniform(-1, 1, shape))
    xd = dev(np.concatenate([a.ravel() for a in xs])) if with_x else None
    out = host(solver.apply_op(_lib.OP_CYCLE, 0, dev(np.concatenate([a.ravel() for a in bs])), xd))
    off = 0
    for g, lg, xa, ba in zip(GRIDS, split_shifts(lam), xs, bs):
        n = g["nx"] * g["ny"] * g["S"]
        got = out[off:off + n].reshape(g["S"], g["ny"], g["nx"])
        off += n
        shapes = ops.level_shapes(g["nx"], g["ny"], g["h"], levels=LEVELS)
        x0 = xa if with_x else np.zeros_like(xa)
        ref = omg.mg_cycle(0, x0, ba, lg, shapes, nu1=nu1, nu2=nu2, gamma=gamma)
        assert maxrel(got, ref) <= 1e-12, (nu1, nu2, gamma, with_x)


def counts_agree(got, want, oracle_relres, tol):
    """Cycle counts must match, except where the oracle stopped within 5% of
    tol: there the final residual (a cancellation with rounding noise of order
    eps |L| |z|) may fall on either side of tol in another summation order."""
    for g, w, r in zip(got, want, oracle_relres):
        if g != w and not (abs(int(g) - int(w)) == 1 and r > 0.95 * tol):
            return False
    return True


@pytest.mark.parametrize("nu1,nu2", [(2, 2), (1, 1)])
def test_streamed_solve_parity(nu1, nu2):
    """Free-running solves with the fused finest-level norm reach the
    tolerance with the oracle's cycle counts; at the oracle's counts the
    solutions agree to 1e-10."""
    solver, lam = make(nu1, nu2)
    bs = [inputs.rhs(g["S"], g["ny"], g["nx"], seed=40 + k) for k, g in enumerate(GRIDS)]
    bd = dev(np.concatenate([b.ravel() for b in bs]))
    Z, iters, relres, status = solver.solve(bd, tol=1e-10)
    assert status == 0 and np.all(relres <= 1e-10)
    refs, counts, sys = [], [], 0
    for g, lg, b in zip(GRIDS, split_shifts(lam), bs):
        zr, itr, rr, _ = omg.solve(b, lg, g["h"], tol=1e-10, levels=LEVELS, nu1=nu1, nu2=nu2)
        assert counts_agree(iters[sys:sys + g["S"]], itr, rr, 1e-10), (iters[sys:sys + g["S"]], itr, rr)
        sys += g["S"]
        refs.append(zr)
        counts.extend(itr)
    Z2, it2, _, _ = solver.solve(bd, fixed_iters=counts)
    np.testing.assert_array_equal(it2, counts)
    z, off = host(Z2), 0
    for g, zr in zip(GRIDS, refs):
        n = g["nx"] * g["ny"] * g["S"]
        zg = z[off:off + n].reshape(zr.shape)
        off += n
        for j in range(g["S"]):
            assert np.linalg.norm(zg[j] - zr[j]) <= 1e-10 * np.linalg.norm(zr[j])


@pytest.mark.parametrize("precision", ["c128", "c128_c64"])
def test_streamed_full_size_sampled_sweep_and_solve(precision):
    """The 1023 x 1023 benchmark grid (64 alpha-circulant shifts, 8 levels, the
    launch configuration bench.py times, without the transforms): every system
    reaches 1e-10, and the solution matches the exact DST solution of the same
    systems within the conditioning; 8 systems are compared in full.  Also
    with the complex64 coarse-grid correction (the bench's leg of it)."""
    from paper_2203_11154_amd import Grid, VankaMG
    n, S = 1023, 64
    h = 1.0 / (n + 1)
    lam = inputs.alpha_circulant_shifts(S)
    b = inputs.rhs(S, n, n)
    solver = VankaMG([Grid(n, num_systems=S)], lam, precision=precision)
    Z, iters, relres, status = solver.solve(dev(b.ravel()), tol=1e-10)
    assert status == 0 and np.all(relres <= 1e-10) and np.all(iters == iters[0])
    z = host(Z).reshape(S, n, n)
    pick = np.arange(0, S, 8)
    zx = exact.dst_solve(b[pick], lam[pick], h)
    # residual recomputed on the host in FP64 (independent of the library)
    rr = omg.residual_norms(z[pick], b[pick], lam[pick], h) / np.linalg.norm(b[pick].reshape(len(pick), -1), axis=1)
    assert np.all(rr <= 1.01e-10)
    err = np.linalg.norm((z[pick] - zx).reshape(len(pick), -1), axis=1) / np.linalg.norm(zx.reshape(len(pick), -1), axis=1)
    assert np.all(err <= 1e-7)


@pytest.mark.parametrize("edge", ["0", "2"])
@pytest.mark.parametrize("nu1,nu2", [(2, 2), (1, 1), (0, 1)])
def test_fused_norm_equals_host_residual(nu1, nu2, edge, monkeypatch):
    """The stopping-test norm that the finest-level streaming kernel forms
    equals the residual norm of the iterate it writes, recomputed on the host
    in FP64, after 1 and 2 cycles (large residuals, so no cancellation noise):
    every owned column of every strip carries exactly its own residual.
    edge = "2": the norm formed by the cycle-edge kernel (where it applies)."""
    monkeypatch.setenv("VMG_EDGE", edge)
    solver, lam = make(nu1, nu2)
    if edge == "2" and nu1 > 0:
        assert all(solver.plan(g)[0] for g in range(len(GRIDS)))
    bs = [inputs.rhs(g["S"], g["ny"], g["nx"], seed=50 + k) for k, g in enumerate(GRIDS)]
    bd = dev(np.concatenate([b.ravel() for b in bs]))
    S = sum(g["S"] for g in GRIDS)
    for cycles in (1, 2):
        Z, it, rr, _ = solver.solve(bd, fixed_iters=np.full(S, cycles, dtype=np.int32))
        z, off, sys = host(Z), 0, 0
        for g, lg, b in zip(GRIDS, split_shifts(lam), bs):
            n = g["nx"] * g["ny"] * g["S"]
            zg = z[off:off + n].reshape(b.shape)
            off += n
            ref = omg.residual_norms(zg, b, lg, g["h"]) / np.linalg.norm(b.reshape(g["S"], -1), axis=1)
            np.testing.assert_allclose(rr[sys:sys + g["S"]], ref, rtol=1e-9)
            sys += g["S"]


def test_timing_mask_times_only_the_chosen_classes(monkeypatch):
    """With a class mask only those launches are timed (the others run
    without events); the results do not depend on timing."""
    from paper_2203_11154_amd import Grid, VankaMG
    monkeypatch.setenv("VMG_EDGE", "2")
    lam = inputs.alpha_circulant_shifts(2)
    s = VankaMG([Grid(255, num_systems=2)], lam)
    bd = dev(inputs.rhs(2, 255, 255, seed=33).ravel())
    Z0, it0, _, _ = s.solve(bd, tol=1e-10)
    z0 = host(Z0)
    s.set_timing(True, reset=True, classes=["edge"])
    Z1, it1, _, _ = s.solve(bd, tol=1e-10)
    stats = s.kernel_stats()
    s.set_timing(False, reset=False)
    assert stats["edge"][0] >= int(it1.max()) and stats["edge"][1] > 0
    assert all(v[0] == 0 for k, v in stats.items() if k != "edge")
    s.set_timing(True, reset=True)
    s.solve(bd, tol=1e-10)
    stats = s.kernel_stats()
    s.set_timing(False, reset=False)
    assert stats["edge"][0] > 0 and stats["down"][0] > 0 and stats["up"][0] > 0
    np.testing.assert_array_equal(it1, it0)
    assert np.array_equal(host(Z1), z0)
