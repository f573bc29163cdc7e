"""Parity at the benchmark's own workloads and launch configurations.

* 64 x 1023^2 (the plain workload at scale): the autotuned plan the benchmark
  times (cycle-edge kernel on the finest level, tail kernel on the small
  levels); sampled systems against the oracle's V(2,2) iterate at the
  oracle's cycle counts (eq. (2) under the Sec. 3 components).
* 32 x 2047^2 (the precision workload): FP64 cycles, complex64 cycles inside
  FP64 refinement, and FP64 cycles with a complex64 coarse-grid correction;
  the FP64 residual of every system recomputed on the host, a sampled system
  against the oracle, and each result's error against the oracle printed.
* V(2,2) with the cycle-edge kernel forced on grids with ragged strips,
  against the oracle at fixed counts.
* Example 2 (eq. (10)) on two shifts, one with a negative real part, against
  the oracle at the GPU's counts (W(1,0), Sec. 3).
* More than 32 grids in one handle: replayed graphs against eager launches.
"""
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


def host_relres(z, b, lam, h, chunk=4):
    """FP64 relative residuals ||b_j - L_j z_j|| / ||b_j|| recomputed on the
    host by the oracle's operator (independent of the library)."""
    out = []
    for s in range(0, len(lam), chunk):
        sl = slice(s, s + chunk)
        r = omg.residual_norms(z[sl], b[sl], lam[sl], h)
        out.append(r / np.linalg.norm(b[sl].reshape(len(r), -1), axis=1))
    return np.concatenate(out)


def test_plain_1023_autotuned_plan_vs_oracle():
    """64 alpha-circulant shifts on 1023^2, the schedule bench.py times
    (autotuned; the finest level on the cycle-edge kernel, the small levels in
    the tail kernel): free-running counts equal the oracle's on sampled
    systems, and at the oracle's counts the iterates agree to 1e-10."""
    from paper_2203_11154_amd import Grid, VankaMG
    n, S = 1023, 64
    h = 1.0 / (n + 1)
    lam = inputs.alpha_circulant_shifts(S)
    b = inputs.rhs(S, n, n)
    solver = VankaMG([Grid(n, num_systems=S)], lam)
    solver.autotune()
    edge, tail = solver.plan(0)
    assert edge and tail > 0, (edge, tail)
    bd = dev(b.ravel())
    Z, iters, relres, status = solver.solve(bd, tol=1e-10)
    assert status == 0 and np.all(relres <= 1e-10)
    pick = np.array([5, 44])
    zr, itr, rr, _ = omg.solve(b[pick], lam[pick], h, tol=1e-10)
    for k, j in enumerate(pick):
        assert iters[j] == itr[k] or (abs(int(iters[j]) - int(itr[k])) == 1 and rr[k] > 0.95e-10), (j, iters[j], itr[k])
    fixed = iters.astype(np.int32).copy()
    fixed[pick] = itr
    Z2, it2, _, _ = solver.solve(bd, fixed_iters=fixed, out=Z)
    np.testing.assert_array_equal(it2, fixed)
    z = host(Z2).reshape(S, n, n)
    errs = [relerr(z[j], zr[k]) for k, j in enumerate(pick)]
    print(f"1023^2 x 64 autotuned: cycles {iters.min()}-{iters.max()}, oracle {itr.tolist()}, "
          f"rel. err vs oracle {['%.2e' % e for e in errs]}")
    assert max(errs) <= 1e-10


@pytest.fixture(scope="module")
def precision_workload():
    """32 alpha-circulant shifts (tau = 1/32) on 2047^2, right-hand sides as
    in the benchmark's precision leg, and the oracle's solution of system 3
    at tol 1e-10 (about 9 V(2,2) cycles on 2047^2: tens of seconds on the
    host)."""
    n, S = 2047, 32
    h = 1.0 / (n + 1)
    lam = inputs.alpha_circulant_shifts(S, 0.01)
    b = inputs.rhs(S, n, n, seed=4)
    j = 3
    zr, itr, rr, _ = omg.solve(b[[j]], lam[[j]], h, tol=1e-10)
    return dict(n=n, S=S, h=h, lam=lam, b=b, j=j, z_or=zr[0], it_or=int(itr[0]), rr_or=float(rr[0]))


@pytest.mark.parametrize("precision", ["c128", "c64_ir", "c128_c64"])
def test_precision_2047_vs_oracle(precision_workload, precision):
    """The precision workload in each precision: every system's FP64 residual,
    recomputed on the host, is at most 1.01e-10; the result of system 3
    against the oracle's FP64 solution (FP64 cycles: at the oracle's count,
    within 1e-10; the complex64 variants: both residuals at most 1e-10 apart
    by the conditioning, printed per result, within 1e-6)."""
    from paper_2203_11154_amd import Grid, VankaMG
    w = precision_workload
    n, S, h, lam, b, j = w["n"], w["S"], w["h"], w["lam"], w["b"], w["j"]
    kw = {"c128": {}, "c64_ir": {"precision": "c64_ir", "ir_inner": 2}, "c128_c64": {"precision": "c128_c64"}}[precision]
    solver = VankaMG([Grid(n, num_systems=S)], lam, **kw)
    solver.autotune()
    bd = dev(b.ravel())
    Z, iters, relres, status = solver.solve(bd, tol=1e-10)
    assert status == 0 and np.all(relres <= 1e-10)
    z = host(Z).reshape(S, n, n)
    rr_host = host_relres(z, b, lam, h)
    assert np.all(rr_host <= 1.01e-10), rr_host.max()
    err = relerr(z[j], w["z_or"])
    print(f"2047^2 x 32 {precision}: cycles/steps {iters.min()}-{iters.max()}, host relres max {rr_host.max():.3e}, "
          f"system {j}: rel. err vs oracle {err:.3e} (oracle {w['it_or']} cycles, relres {w['rr_or']:.3e})")
    if precision == "c128":
        assert iters[j] == w["it_or"] or (abs(int(iters[j]) - w["it_or"]) == 1 and w["rr_or"] > 0.95e-10)
        fixed = iters.astype(np.int32).copy()
        fixed[j] = w["it_or"]
        Z2, _, _, _ = solver.solve(bd, fixed_iters=fixed, out=Z)
        zj = host(Z2[j * n * n:(j + 1) * n * n]).reshape(n, n)
        assert relerr(zj, w["z_or"]) <= 1e-10
    else:
        assert err <= 1e-6
    del solver


@pytest.mark.parametrize("nu1,nu2,pace,precision", [(2, 2, "0", "c128"), (2, 1, "0", "c128"), (2, 2, "1", "c128"),
                                                    (1, 2, "1", "c128"), (2, 2, "1", "c128_c64")])
def test_forced_edge_kernel_vs_oracle(nu1, nu2, pace, precision, monkeypatch):
    """The cycle-edge kernel on every grid (VMG_EDGE=2), V(nu1, nu2), on
    grids whose strips and runs end ragged (223 x 111: 223 = 5 x 44 + 3
    columns for 44 owned columns a strip; 127 x 255), in plain and in paced
    blocks (VMG_EDGE_PACE=1: blocks of waves from both grids, of different
    trip counts, meet at barriers), FP64 and with the complex64 coarse-grid
    correction: counts equal the oracle's and, at the oracle's counts, the
    iterates agree to 1e-10."""
    from paper_2203_11154_amd import Grid, VankaMG
    monkeypatch.setenv("VMG_EDGE", "2")
    monkeypatch.setenv("VMG_EDGE_PACE", pace)
    grids = [dict(nx=223, ny=111, h=1.0 / 224, S=2), dict(nx=127, ny=255, h=1.0 / 128, S=2)]
    gs = [Grid(g["nx"], g["ny"], h=g["h"], num_systems=g["S"], levels=5) for g in grids]
    lam = np.concatenate([inputs.alpha_circulant_shifts(2), inputs.uniform_shifts(2)])
    solver = VankaMG(gs, lam, nu1=nu1, nu2=nu2, precision=precision)
    for g in range(len(grids)):
        assert solver.plan(g)[0], g
    bs = [inputs.rhs(g["S"], g["ny"], g["nx"], seed=70 + k) for k, g in enumerate(grids)]
    bd = dev(np.concatenate([x.ravel() for x in bs]))
    _, iters, relres, status = solver.solve(bd, tol=1e-10)
    assert status == 0 and np.all(relres <= 1e-10)
    refs, counts, off = [], [], 0
    for g, b in zip(grids, bs):
        lg = lam[off:off + g["S"]]
        zr, itr, rr, _ = omg.solve(b, lg, g["h"], tol=1e-10, levels=5, nu1=nu1, nu2=nu2)
        for k in range(g["S"]):
            if precision == "c128":
                assert iters[off + k] == itr[k] or (abs(int(iters[off + k]) - int(itr[k])) == 1 and rr[k] > 0.95e-10)
            else:
                # (the complex64 correction: the FP64 counts, or one more)
                assert itr[k] <= iters[off + k] <= itr[k] + 1
        refs.append(zr)
        counts.extend(itr.tolist())
        off += g["S"]
    Z, it2, _, _ = solver.solve(bd, fixed_iters=counts)
    np.testing.assert_array_equal(it2, counts)
    z, off = host(Z), 0
    # (complex64 coarse-grid correction: each cycle's correction carries its
    # complex64 rounding, ~u32 kappa_H relative; 1e-5 bounds that as in the
    # mixed-precision tests)
    bound = 1e-10 if precision == "c128" else 1e-5
    for g, zr in zip(grids, refs):
        m = g["nx"] * g["ny"]
        for k in range(g["S"]):
            assert relerr(z[off:off + m].reshape(g["ny"], g["nx"]), zr[k]) <= bound, (g, k)
            off += m


@pytest.mark.parametrize("precision", ["c128", "c128_c64"])
def test_paced_blocks_bitwise_equal_plain(precision, monkeypatch):
    """Paced blocks change when the waves run, not what they compute: with
    VMG_EDGE_PACE=1 the cycle-edge kernel, the first pre-smoothing and
    restriction and the finishing pass of V(2,2) on the finest level (both
    grids of one launch, ragged strips and runs) give bitwise the iterates
    of the plain blocks, at free-running and at fixed counts."""
    from paper_2203_11154_amd import Grid, VankaMG
    monkeypatch.setenv("VMG_EDGE", "2")
    grids = [dict(nx=223, ny=111, h=1.0 / 224, S=3), dict(nx=127, ny=255, h=1.0 / 128, S=2)]
    lam = np.concatenate([inputs.alpha_circulant_shifts(3), inputs.uniform_shifts(2)])
    bs = [inputs.rhs(g["S"], g["ny"], g["nx"], seed=90 + k) for k, g in enumerate(grids)]
    bd = dev(np.concatenate([x.ravel() for x in bs]))
    out = {}
    for pace in ("0", "1"):
        monkeypatch.setenv("VMG_EDGE_PACE", pace)
        gs = [Grid(g["nx"], g["ny"], h=g["h"], num_systems=g["S"], levels=5) for g in grids]
        solver = VankaMG(gs, lam, nu1=2, nu2=2, precision=precision)
        assert all(solver.plan(g)[0] == (2 if pace == "1" else 1) for g in range(len(grids)))
        Z, iters, relres, status = solver.solve(bd, tol=1e-10)
        assert status == 0 and np.all(relres <= 1e-10)
        fixed = np.arange(len(lam), dtype=np.int32) % 3 + 1
        Zf, itf, _, _ = solver.solve(bd, fixed_iters=fixed)
        np.testing.assert_array_equal(itf, fixed)
        out[pace] = (host(Z), iters, relres, host(Zf))
        del solver
    (z0, i0, r0, f0), (z1, i1, r1, f1) = out["0"], out["1"]
    np.testing.assert_array_equal(i0, i1)
    np.testing.assert_array_equal(r0, r1)
    assert np.array_equal(z0, z1) and np.array_equal(f0, f1)


def test_example2_vs_oracle():
    """Example 2 (eq. (10), beta = 0.01, h = tau = 1/256): the shift with the
    most negative real part and the one with the largest real part, W(1,0)
    to 1e-8 (Sec. 3); the GPU iterate equals the oracle's at the GPU's
    counts to 1e-10."""
    from paper_2203_11154_amd import Grid, VankaMG
    n, nt = 255, 256
    h = 1.0 / (n + 1)
    lam_all = inputs.example2_shifts(nt)
    lam = np.array([lam_all[np.argmin(lam_all.real)], lam_all[np.argmax(lam_all.real)]])
    assert lam[0].real < 0 < lam[1].real
    b = inputs.rhs(2, n, n, seed=12)
    solver = VankaMG([Grid(n, num_systems=2)], lam, nu1=1, nu2=0, gamma=2)
    Z, it, rr, status = solver.solve(dev(b.ravel()), tol=1e-8)
    assert status == 0 and np.all(rr <= 1e-8)
    zr, itr, rro, _ = omg.solve(b, lam, h, tol=1e-8, nu1=1, nu2=0, gamma=2)
    for k in range(2):
        assert it[k] == itr[k] or (abs(int(it[k]) - int(itr[k])) == 1 and rro[k] > 0.95e-8)
    zf, _, _, _ = omg.solve(b, lam, h, fixed_iters=it, nu1=1, nu2=0, gamma=2)
    z = host(Z).reshape(2, n, n)
    for k in range(2):
        assert relerr(z[k], zf[k]) <= 1e-10, k
    # and the exact solution within the conditioning of the 1e-8 residual
    zx = exact.dst_solve(b, lam, h)
    for k in range(2):
        assert relerr(z[k], zx[k]) <= 1e-5


def test_many_grids_graphs_equal_eager(monkeypatch):
    """33 grids in one handle, V(2,1): grid 0 on the cycle-edge kernel (its
    finest iterate changes buffers once a cycle from the second cycle on),
    grid 32 on the tiled kernels at level 0 (three buffer flips a cycle),
    the rest small.  Cycles replayed from captured graphs give bitwise the
    eager launches' iterates at fixed counts of several cycles, so the graph
    of one cycle is never replayed for another buffer state."""
    from paper_2203_11154_amd import Grid, VankaMG
    monkeypatch.setenv("VMG_EDGE", "2")
    sizes = [(127, 1)] + [(31, 1)] * 31 + [(95, 1)]
    gs = [Grid(nx, num_systems=s) for nx, s in sizes]
    lam = inputs.alpha_circulant_shifts(len(sizes))
    b = np.concatenate([inputs.rhs(s, nx, nx, seed=200 + k).ravel() for k, (nx, s) in enumerate(sizes)])
    bd = dev(b)
    res = {}
    for graphs in (True, False):
        s = VankaMG(gs, lam, nu1=2, nu2=1, graphs=graphs)
        assert s.plan(0)[0] and s.schedule(32)[0] == 0 and s.plan(32)[1] > 0
        outs = []
        for fi in (3, 4, 5):
            Z, it, _, _ = s.solve(bd, fixed_iters=np.full(len(sizes), fi, np.int32))
            np.testing.assert_array_equal(it, fi)
            outs.append(host(Z))
        res[graphs] = outs
        del s
    for a, e in zip(res[True], res[False]):
        np.testing.assert_array_equal(a, e)
