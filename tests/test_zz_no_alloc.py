"""The transform entry point that allocates nothing
(paradiag_transform_noalloc), called through the C ABI: its results equal
paradiag_transform's bit for bit on two calls in a row, the second on a
smaller input (the fixed per-GPU array keeps the first call's contents), and
sizes beyond its array are refused before any device work."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2203_11154_amd import _lib

pytestmark = pytest.mark.gpu


def _c128(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to("cuda")


def _call(fn, n, m, M, F, trans_conj, out):
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return fn(n, m, ctypes.c_void_p(M.data_ptr()), trans_conj, ctypes.c_void_p(F.data_ptr()),
              ctypes.c_void_p(out.data_ptr()), stream)


@pytest.mark.parametrize("first,second", [((64, 3001, 0), (16, 517, 1)), ((128, 1500, 1), (8, 333, 0))])
def test_noalloc_transform_equals_allocating_entry_point(first, second):
    lib = _lib.load()
    rng = np.random.default_rng(91)
    for n, m, tc in (first, second):
        print(f"noalloc transform n={n} m={m} trans_conj={tc}", flush=True)
        M = rng.uniform(-1, 1, (n, n)) + 1j * rng.uniform(-1, 1, (n, n))
        F = rng.uniform(-1, 1, (n, m)) + 1j * rng.uniform(-1, 1, (n, m))
        Md, Fd = _c128(M), _c128(F)
        ref = torch.empty_like(Fd)
        got = torch.full_like(Fd, float("nan"))
        assert _call(lib.paradiag_transform, n, m, Md, Fd, tc, ref) == _lib.VMG_OK
        assert _call(lib.paradiag_transform_noalloc, n, m, Md, Fd, tc, got) == _lib.VMG_OK
        torch.cuda.synchronize()
        r, g = ref.cpu().numpy(), got.cpu().numpy()
        np.testing.assert_array_equal(g, r)
        # and the product itself, against a host FP64 matmul
        exp = (M.conj().T if tc else M) @ F
        assert np.linalg.norm(g - exp) <= 1e-13 * np.linalg.norm(exp)


def test_noalloc_transform_refuses_sizes_beyond_its_array():
    lib = _lib.load()
    n, m = 257, 64
    Md = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
    Fd = torch.zeros((n, m), dtype=torch.complex128, device="cuda")
    out = torch.zeros_like(Fd)
    assert _call(lib.paradiag_transform_noalloc, n, m, Md, Fd, 0, out) == _lib.VMG_INVALID_ARG
    assert _call(lib.paradiag_transform_noalloc, 0, m, Md, Fd, 0, out) == _lib.VMG_INVALID_ARG
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0
