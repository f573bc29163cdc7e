"""Size limits: the streaming kernels address a plane through a 32-bit
checked buffer range, so FP64 planes of 1 GiB and more run the LDS-tiled
kernels.  The largest finest level on each side of that limit (a single
system; both solved to 1e-10, the residual recomputed on the host in FP64),
and the complex64 coarse-grid correction, which needs a streamed finest
level, is refused on the larger one."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import multigrid as omg
from paper_2203_11154_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nx,ny,streamed", [(8191, 6143, True), (8191, 8191, False)])
def test_largest_planes_each_side_of_the_streaming_limit(nx, ny, streamed):
    from paper_2203_11154_amd import Grid, VankaMG, _lib
    lam = np.array([40.0 + 25.0j])
    b = inputs.rhs(1, ny, nx, seed=21)
    # plane bytes: (ny + 2) rows of nx + 2 complex128 rounded up to 128 bytes
    pitch = -(-(nx + 2) * 16 // 128) * 128
    assert ((ny + 2) * pitch < 2 ** 30) == streamed
    solver = VankaMG([Grid(nx, ny, num_systems=1)], lam)
    assert (solver.schedule(0)[0] > 0) == streamed
    Z, it, rr, st = solver.solve(torch.from_numpy(b.ravel()).to("cuda"), tol=1e-10)
    assert st == 0 and rr[0] <= 1e-10
    torch.cuda.synchronize()
    z = Z.cpu().numpy().reshape(1, ny, nx)
    del Z, solver
    r = omg.residual_norms(z, b, lam, 1.0 / (nx + 1)) / np.linalg.norm(b)
    assert r[0] <= 1.01e-10, r
    if not streamed:
        with pytest.raises(_lib.VankaMGError):
            VankaMG([Grid(nx, ny, num_systems=1)], lam, precision="c128_c64")
