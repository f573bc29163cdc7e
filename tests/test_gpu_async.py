"""Fixed-count solves without host outputs only enqueue work: several such
calls in a row (more than the library's ring of pinned count buffers) give
bitwise the results of the synchronous calls, and the last call's counts are
reported afterwards."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2203_11154_amd import inputs

pytestmark = pytest.mark.gpu


def test_async_fixed_solves_match_sync():
    from paper_2203_11154_amd import Grid, VankaMG
    grids = [Grid(255, num_systems=3), Grid(127, num_systems=2)]
    S = 5
    solver = VankaMG(grids, inputs.alpha_circulant_shifts(S))
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
