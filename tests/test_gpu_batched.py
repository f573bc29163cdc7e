"""Batched solves of many systems on grids of uneven size (one launch per
phase for all grids, cycles replayed as captured hipGraphs) against the
oracle, graph replays against eager launches, and the full uneven workload
(256 x 127^2, 96 x 255^2, 32 x 511^2) against exact DST solutions."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import exact, multigrid as omg
from paper_2203_11154_amd import inputs

pytestmark = pytest.mark.gpu

# three unit-square grids with 3, 4 and 5 levels (coarsest 7 x 7 for all)
SMALL = [(31, 6), (63, 4), (127, 3)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.complex128))).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def setup(groups, **kw):
    from paper_2203_11154_amd import Grid, VankaMG
    S = sum(c for _, c in groups)
    lam = inputs.uniform_shifts(S)
    solver = VankaMG([Grid(n, num_systems=c) for n, c in groups], lam, **kw)
    bs = [inputs.rhs(c, n, n, seed=60 + k) for k, (n, c) in enumerate(groups)]
    return solver, lam, bs


def split(vec, groups):
    out, off = [], 0
    for n, c in groups:
        out.append(vec[off:off + n * n * c].reshape(c, n, n))
        off += n * n * c
    return out


@pytest.mark.parametrize("graphs", [True, False])
def test_batched_uneven_parity(graphs):
    solver, lam, bs = setup(SMALL, graphs=graphs)
    bd = dev(np.concatenate([b.ravel() for b in bs]))
    Z, iters, relres, status = solver.solve(bd, tol=1e-10)
    assert status == 0 and np.all(relres <= 1e-10)
    counts, refs, off = [], [], 0
    for (n, c), b in zip(SMALL, bs):
        zr, itr, rr, _ = omg.solve(b, lam[off:off + c], 1.0 / (n + 1), tol=1e-10)
        for a, w, r in zip(iters[off:off + c], itr, rr):
            assert a == w or (abs(int(a) - int(w)) == 1 and r > 0.95e-10)
        counts.extend(itr)
        refs.append(zr)
        off += c
    Z2, it2, _, _ = solver.solve(bd, fixed_iters=counts)
    np.testing.assert_array_equal(it2, counts)
    for got, zr in zip(split(host(Z2), SMALL), refs):
        for j in range(len(zr)):
            assert np.linalg.norm(got[j] - zr[j]) <= 1e-10 * np.linalg.norm(zr[j])


def test_graph_replays_match_eager():
    """The same solves through captured graphs and through eager launches are
    bitwise identical, over repeated replays with other GPU work and host
    synchronisations in between."""
    sg, lam, bs = setup(SMALL, graphs=True)
    se, _, _ = setup(SMALL, graphs=False)
    bd = dev(np.concatenate([b.ravel() for b in bs]))
    ze, ie, _, _ = se.solve(bd, tol=1e-10)
    for rep in range(4):
        scratch = torch.randn(1 << 20, device="cuda").cumsum(0)  # unrelated eager work
        torch.cuda.synchronize()
        zg, ig, _, _ = sg.solve(bd, tol=1e-10)
        torch.cuda.synchronize()
        assert torch.equal(zg, ze), rep
        np.testing.assert_array_equal(ig, ie)
        del scratch
    # conjugate shifts through their own graphs
    zc_e, _, _, _ = se.solve(bd, tol=1e-10, conj=True)
    zc_g, _, _, _ = sg.solve(bd, tol=1e-10, conj=True)
    assert torch.equal(zc_e, zc_g)


def test_w_cycle_multi_grid_parity():
    """W(1,0) cycles (the paper's Sec. 3 protocol) on grids of uneven depth,
    run grid by grid, against the oracle at fixed counts."""
    solver, lam, bs = setup(SMALL, nu1=1, nu2=0, gamma=2)
    bd = dev(np.concatenate([b.ravel() for b in bs]))
    Z, iters, relres, status = solver.solve(bd, tol=1e-8)
    assert status == 0 and np.all(relres <= 1e-8)
    counts, refs, off = [], [], 0
    for (n, c), b in zip(SMALL, bs):
        zr, itr, rr, _ = omg.solve(b, lam[off:off + c], 1.0 / (n + 1), tol=1e-8, nu1=1, nu2=0, gamma=2)
        for a, w, r in zip(iters[off:off + c], itr, rr):
            assert a == w or (abs(int(a) - int(w)) == 1 and r > 0.95e-8)
        counts.extend(itr)
        refs.append(zr)
        off += c
    Z2, _, _, _ = solver.solve(bd, fixed_iters=counts)
    for got, zr in zip(split(host(Z2), SMALL), refs):
        for j in range(len(zr)):
            assert np.linalg.norm(got[j] - zr[j]) <= 1e-10 * np.linalg.norm(zr[j])


def test_refinement_batched_uneven():
    solver, lam, bs = setup(SMALL, precision="c64_ir")
    bd = dev(np.concatenate([b.ravel() for b in bs]))
    Z, iters, relres, status = solver.solve(bd, tol=1e-10)
    assert status == 0 and np.all(relres <= 1e-10)
    off = 0
    for (n, c), b, got in zip(SMALL, bs, split(host(Z), SMALL)):
        r = omg.residual_norms(got, b, lam[off:off + c], 1.0 / (n + 1)) / np.linalg.norm(b.reshape(c, -1), axis=1)
        assert np.all(r <= 1.01e-10)
        off += c


def test_full_uneven_workload():
    """256 x 127^2 + 96 x 255^2 + 32 x 511^2 systems, shifts Re ~ U(1, 1e4),
    Im ~ U(-1e4, 1e4), V(2,2) to 1e-10 in one batched solve; two systems per
    grid are checked against the exact DST solution."""
    groups = [(127, 256), (255, 96), (511, 32)]
    solver, lam, bs = setup(groups)
    bd = dev(np.concatenate([b.ravel() for b in bs]))
    Z, iters, relres, status = solver.solve(bd, tol=1e-10)
    assert status == 0 and np.all(relres <= 1e-10)
    off = 0
    for (n, c), b, got in zip(groups, bs, split(host(Z), groups)):
        pick = np.array([0, c - 1])
        zx = exact.dst_solve(b[pick], lam[off + pick], 1.0 / (n + 1))
        err = np.linalg.norm((got[pick] - zx).reshape(2, -1), axis=1) / np.linalg.norm(zx.reshape(2, -1), axis=1)
        assert np.all(err <= 1e-8)
        off += c


def test_autotuned_schedule_parity(tmp_path):
    """The autotuner's per-level choice (LDS-tiled or streaming with 16/32/64/128
    rows) is a valid schedule, is reused from its cache, and the tuned solve
    matches the oracle at fixed counts."""
    cache = tmp_path / "tune.txt"
    solver, lam, bs = setup(SMALL)
    scheds = solver.autotune(cache)
    for (n, c), sc in zip(SMALL, scheds):
        assert sc[-1] == -1 and all(v in (0, 16, 32, 64, 128) for v in sc[:-1])
    text = cache.read_text()
    # one line per grid and level, plus one "edge" line for each grid whose
    # finest level was tuned to stream (the cycle-edge kernel is timed only
    # then, so that line follows the timing of the level choice), and one
    # "edgepace" line for each grid that then uses the cycle-edge kernel
    lines = [ln.split() for ln in text.splitlines()]
    level_lines = [ln for ln in lines if ln[-2] not in ("edge", "edgepace")]
    edge_lines = [ln for ln in lines if ln[-2] == "edge"]
    pace_lines = [ln for ln in lines if ln[-2] == "edgepace"]
    assert len(level_lines) == sum(len(sc) - 1 for sc in scheds)
    streamed = {(n, n) for (n, c), sc in zip(SMALL, scheds) if sc[0] > 0}
    assert all((int(ln[2]), int(ln[3])) in streamed for ln in edge_lines)
    assert all((int(ln[2]), int(ln[3])) in streamed for ln in pace_lines)
    assert all(int(ln[-1]) in (0, 1) for ln in pace_lines)
    again, _, _ = setup(SMALL)
    assert again.autotune(cache) == scheds
    assert cache.read_text() == text
    bd = dev(np.concatenate([b.ravel() for b in bs]))
    counts, refs, off = [], [], 0
    for (n, c), b in zip(SMALL, bs):
        zr, itr, _, _ = omg.solve(b, lam[off:off + c], 1.0 / (n + 1), tol=1e-10)
        counts.extend(itr)
        refs.append(zr)
        off += c
    Z, _, _, _ = solver.solve(bd, fixed_iters=counts)
    for got, zr in zip(split(host(Z), SMALL), refs):
        for j in range(len(zr)):
            assert np.linalg.norm(got[j] - zr[j]) <= 1e-10 * np.linalg.norm(zr[j])
