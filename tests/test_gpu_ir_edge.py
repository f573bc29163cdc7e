"""Complex64 V-cycles inside FP64 refinement with the step boundary in one
pass (k_ir_edge: the last inner cycle's correction and post-smoothing, the
FP64 update x' = x + e and residual, the next step's first pre-smoothing and
restriction) against the same refinement with separate passes
(VMG_IR_EDGE=0), and against the FP64 bar checked independently on the host
(residual of the result, the exact DST solution)."""
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
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


# ragged strips and runs (223 = 5 x 44 + 3 columns), a rectangle, a square
GRIDS = [(223, 111, 2), (255, 255, 2), (127, 255, 1)]


def make(grids, monkeypatch, ir_edge, pace="0", **kw):
    from paper_2203_11154_amd import Grid, VankaMG
    monkeypatch.setenv("VMG_EDGE", "2")
    monkeypatch.setenv("VMG_IR_EDGE", "1" if ir_edge else "0")
    monkeypatch.setenv("VMG_EDGE_PACE", pace)
    lam = inputs.alpha_circulant_shifts(sum(s for _, _, s in grids))
    gs = [Grid(nx, ny, num_systems=s) for nx, ny, s in grids]
    return VankaMG(gs, lam, precision="c64_ir", **kw), lam


def host_relres(z, bs, lam, grids):
    out, off, s0 = [], 0, 0
    for (nx, ny, s), b in zip(grids, bs):
        zg = z[off:off + nx * ny * s].reshape(s, ny, nx)
        h = 1.0 / (nx + 1)
        r = omg.residual_norms(zg, b, lam[s0:s0 + s], h) / np.linalg.norm(b.reshape(s, -1), axis=1)
        out.append(r)
        off += nx * ny * s
        s0 += s
    return np.concatenate(out)


@pytest.mark.parametrize("nu1,nu2,inner,smoother,pace", [(2, 2, 2, "vanka", "0"), (2, 2, 1, "vanka", "0"),
                                                          (2, 2, 3, "vanka", "0"), (1, 2, 2, "vanka", "0"),
                                                          (2, 1, 2, "vanka", "0"), (1, 1, 2, "vanka", "0"),
                                                          (2, 2, 2, "jacobi", "0"), (2, 2, 2, "vanka", "1"),
                                                          (2, 1, 3, "vanka", "1")])
def test_boundary_kernel_matches_separate_passes(nu1, nu2, inner, smoother, pace, monkeypatch):
    """(pace = 1: the boundary pass in paced blocks, whose waves come from
    the three grids with their different trip counts.)"""
    bs = [inputs.rhs(s, ny, nx, seed=80 + k) for k, (nx, ny, s) in enumerate(GRIDS)]
    bd = dev(np.concatenate([b.ravel() for b in bs]))
    res = {}
    for ir_edge in (True, False):
        s, lam = make(GRIDS, monkeypatch, ir_edge, pace=pace, nu1=nu1, nu2=nu2, ir_inner=inner, smoother=smoother)
        for g in range(len(GRIDS)):
            assert s.plan(g)[0], g
        Z, it, rr, st = s.solve(bd, tol=1e-10)
        assert st == 0 and np.all(rr <= 1e-10), (ir_edge, rr)
        z = host(Z)
        rh = host_relres(z, bs, lam, GRIDS)
        assert np.all(rh <= 1.01e-10), (ir_edge, rh)
        # fixed step counts, no host outputs (enqueued without waits)
        Z2, _, _, _ = s.solve(bd, fixed_iters=it, stats=False)
        z2 = host(Z2)
        assert np.array_equal(z2, z)
        res[ir_edge] = (z, it)
        del s
    (za, ita), (zb, itb) = res[True], res[False]
    print(f"nu=({nu1},{nu2}) inner={inner}: steps {ita.tolist()} (separate passes {itb.tolist()}), "
          f"rel. diff {relerr(za, zb):.2e}")
    # the same arithmetic up to the rounding order of the FP64 residual: the
    # same step counts (one more or fewer only where a step ends at the bar),
    # and with equal counts iterates that differ by rounding only
    assert np.all(np.abs(ita.astype(int) - itb.astype(int)) <= 1)
    if np.array_equal(ita, itb):
        assert relerr(za, zb) <= 1e-8


def test_boundary_kernel_exact_solution_and_graphs(monkeypatch, tmp_path):
    """Square grids: the refined solution within the conditioning of the exact
    (DST) solution; replayed graphs give bitwise the eager launches, also for
    the adjoint (conjugate-shift) systems (both handles take the schedule the
    first one tuned, through the autotuner's cache file)."""
    grids = [(255, 255, 3)]
    b = inputs.rhs(3, 255, 255, seed=90)
    bd = dev(b.ravel())
    from paper_2203_11154_amd import Grid, VankaMG
    monkeypatch.setenv("VMG_IR_EDGE", "1")
    lam = inputs.alpha_circulant_shifts(3)
    out = {}
    for graphs in (True, False):
        s = VankaMG([Grid(255, num_systems=3)], lam, precision="c64_ir", ir_inner=2, graphs=graphs)
        s.autotune(cache_path=tmp_path / "tune.txt")
        for conj in (False, True):
            Z, it, rr, st = s.solve(bd, tol=1e-10, conj=conj)
            assert st == 0 and np.all(rr <= 1e-10)
            out[(graphs, conj)] = (host(Z), it)
        del s
    for conj in (False, True):
        (za, ia), (zb, ib) = out[(True, conj)], out[(False, conj)]
        np.testing.assert_array_equal(ia, ib)
        assert np.array_equal(za, zb)
    z = out[(True, False)][0].reshape(3, 255, 255)
    assert relerr(z, exact.dst_solve(b, lam, 1.0 / 256)) <= 1e-7
    zc = out[(True, True)][0].reshape(3, 255, 255)
    assert relerr(zc, exact.dst_solve(b, np.conj(lam), 1.0 / 256)) <= 1e-7
