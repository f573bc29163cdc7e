"""Fixed-count solves without host outputs only enqueue work: several such
calls in a row (more than the library's ring of pinned count buffers) give
bitwise the results of the synchronous calls, and the last call's counts are
reported afterwards."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2203_11154_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["c128", "c128_c64"])
def test_async_fixed_solves_match_sync(precision):
    from paper_2203_11154_amd import Grid, VankaMG
    grids = [Grid(255, num_systems=3), Grid(127, num_systems=2)]
    S = 5
    solver = VankaMG(grids, inputs.alpha_circulant_shifts(S), precision=precision)
    b = np.concatenate([inputs.rhs(3, 255, 255, seed=90).ravel(), inputs.rhs(2, 127, 127, seed=91).ravel()])
    bd = torch.from_numpy(b).to("cuda")
    counts = [np.array([k % 4, 1, 2, 3, 4], np.int32) + k for k in range(7)]
    sync = []
    for fi in counts:
        Z, it, _, st = solver.solve(bd, fixed_iters=fi)
        assert st == 0
        np.testing.assert_array_equal(it, fi)
        sync.append(Z.cpu().numpy())
    outs = [torch.empty_like(bd) for _ in counts]
    for fi, o in zip(counts, outs):
        Z, it, rr, st = solver.solve(bd, fixed_iters=fi, out=o, stats=False)
        assert it is None and rr is None and st == 0
    torch.cuda.synchronize()
    for o, z in zip(outs, sync):
        assert np.array_equal(o.cpu().numpy(), z)
    it, rr = solver.last_stats()
    np.testing.assert_array_equal(it, counts[-1])


@pytest.mark.parametrize("precision", ["c128", "c64_ir", "c128_c64"])
def test_graph_replay_equals_eager(precision, monkeypatch):
    """Cycles replayed as captured graphs give bitwise the eagerly launched
    results (free-running and fixed counts, and the adjoint systems), with
    eager work and synchronisation between the replays."""
    from paper_2203_11154_amd import Grid, VankaMG
    monkeypatch.setenv("VMG_EDGE", "2")
    grids = [Grid(255, num_systems=3), Grid(383, 191, num_systems=2)]
    lam = inputs.alpha_circulant_shifts(5)
    b = np.concatenate([inputs.rhs(3, 255, 255, seed=92).ravel(), inputs.rhs(2, 191, 383, seed=93).ravel()])
    bd = torch.from_numpy(b).to("cuda")
    res = {}
    for graphs in (False, True):
        s = VankaMG(grids, lam, precision=precision, graphs=graphs)
        out = []
        for rep in range(3):
            for kw in ({"tol": 1e-10}, {"fixed_iters": np.array([1, 2, 3, 4, 5], np.int32)},
                       {"tol": 1e-10, "conj": True}):
                Z, it, rr, st = s.solve(bd, **kw)
                assert st == 0
                out.append((Z.cpu().numpy(), it.copy()))
            torch.cuda.synchronize()
            _ = (bd * 2).sum().item()  # eager work between replays
        res[graphs] = out
        del s
    for (za, ia), (zb, ib) in zip(res[False], res[True]):
        np.testing.assert_array_equal(ia, ib)
        assert np.array_equal(za, zb)
