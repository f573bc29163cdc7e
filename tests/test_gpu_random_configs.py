"""Seeded random configurations of the whole solver against the oracle's
cycles at fixed counts: uneven batches of rectangular grids, every smoothing
count pair the kernels take, V- and W-cycles, the cycle-edge kernel forced on
or off, and the adjoint systems.  One system of every grid is checked in full
(the oracle is slow in Python), the rest only for finite values."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import multigrid as omg
from paper_2203_11154_amd import inputs

pytestmark = pytest.mark.gpu

SIZES = [(31, 31), (63, 31), (95, 47), (127, 63), (63, 127), (191, 95), (127, 127)]


def config(seed):
    rng = np.random.default_rng(1000 + seed)
    ng = int(rng.integers(1, 4))
    grids = [SIZES[int(k)] + (int(rng.integers(1, 4)),) for k in rng.choice(len(SIZES), ng, replace=False)]
    nu1, nu2 = [(0, 1), (1, 0), (1, 1), (2, 1), (1, 2), (2, 2), (0, 2), (2, 0)][int(rng.integers(0, 8))]
    gamma = int(rng.integers(1, 3))
    edge = str(int(rng.integers(0, 2)) * 2)
    conj = bool(rng.integers(0, 2))
    cycles = int(rng.integers(2, 5))
    return grids, nu1, nu2, gamma, edge, conj, cycles


@pytest.mark.parametrize("seed", range(12))
def test_random_configuration_against_oracle(seed, monkeypatch):
    from paper_2203_11154_amd import Grid, VankaMG
    grids, nu1, nu2, gamma, edge, conj, cycles = config(seed)
    monkeypatch.setenv("VMG_EDGE", edge)
    S = sum(g[2] for g in grids)
    lam = inputs.uniform_shifts(S, seed=seed, re=(1.0, 2e3), im=(-2e3, 2e3))
    solver = VankaMG([Grid(nx, ny, num_systems=s) for nx, ny, s in grids], lam, nu1=nu1, nu2=nu2, gamma=gamma)
    bs = [inputs.rhs(s, ny, nx, seed=seed * 10 + k) for k, (nx, ny, s) in enumerate(grids)]
    bd = torch.from_numpy(np.concatenate([b.ravel() for b in bs])).to("cuda")
    Z, it, rr, st = solver.solve(bd, conj=conj, fixed_iters=np.full(S, cycles, np.int32))
    assert st == 0
    z = Z.cpu().numpy()
    assert np.all(np.isfinite(z))
    off, sys0 = 0, 0
    for (nx, ny, s), b in zip(grids, bs):
        j = seed % s
        lj = lam[sys0 + j]
        zr, _, _, _ = omg.solve(b[j:j + 1], np.array([np.conj(lj) if conj else lj]), 1.0 / (nx + 1),
                                fixed_iters=[cycles], nu1=nu1, nu2=nu2, gamma=gamma)
        zg = z[off + j * nx * ny: off + (j + 1) * nx * ny].reshape(ny, nx)
        err = np.linalg.norm(zg - zr[0]) / np.linalg.norm(zr[0])
        assert err <= 1e-11, (grids, nu1, nu2, gamma, edge, conj, cycles, (nx, ny), err)
        off += s * nx * ny
        sys0 += s
