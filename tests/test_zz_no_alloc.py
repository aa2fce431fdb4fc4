"""The allocation-free entry point sbr_tridiag_eigvals_noalloc, through the
C ABI, against sbr_tridiag_eigvals (the same kernels on plan workspace): two
calls in a row on one GPU, the second on a smaller tridiagonal (the shared
scratch keeps the first call's contents), each compared element by element;
plus the host-side rejection of orders beyond the fixed scratch."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

EPS64 = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def sbr():
    import paper_1604_03703_amd as m
    assert torch.cuda.is_available()
    return m


def _call(lib, fn, d, e, w):
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ep = ctypes.c_void_p(e.data_ptr()) if e is not None else ctypes.c_void_p(0)
    return getattr(lib, fn)(d.shape[0], ctypes.c_void_p(d.data_ptr()), ep, s, ctypes.c_void_p(w.data_ptr()))


def test_noalloc_matches_plan_entry_point_twice(sbr, oracle_mod):
    lib = sbr.lib()
    rng = np.random.default_rng(2024)
    for n in (200000, 3001):          # second call smaller: stale scratch beyond n
        print("noalloc n=%d" % n, flush=True)
        d = rng.standard_normal(n)
        e = rng.standard_normal(n - 1)
        e[::97] = 0.0
        dd, ed = torch.from_numpy(d).cuda(), torch.from_numpy(e).cuda()
        w_ref = torch.empty(n, dtype=torch.float64, device="cuda")
        w_na = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        assert _call(lib, "sbr_tridiag_eigvals", dd, ed, w_ref) == 0
        assert _call(lib, "sbr_tridiag_eigvals_noalloc", dd, ed, w_na) == 0
        torch.cuda.synchronize()
        a, b = w_na.cpu().numpy(), w_ref.cpu().numpy()
        nrm = float(np.max(np.abs(b)))
        assert np.max(np.abs(a - b)) <= 4 * EPS64 * nrm
        assert np.array_equal(a, b)       # the same kernels on the same data
        if n <= 5000:
            ref = oracle_mod.tridiag_eigvals(d, e)
            assert np.max(np.abs(a - ref)) <= 4 * EPS64 * np.max(np.abs(ref))


def test_noalloc_small_orders_and_limit(sbr):
    lib = sbr.lib()
    one = torch.tensor([2.5], dtype=torch.float64, device="cuda")
    w = torch.empty(1, dtype=torch.float64, device="cuda")
    assert _call(lib, "sbr_tridiag_eigvals_noalloc", one, None, w) == 0
    torch.cuda.synchronize()
    assert float(w[0]) == 2.5
    # beyond the fixed scratch: refused on the host, nothing enqueued
    n = (1 << 18) + 1
    big = torch.zeros(n, dtype=torch.float64, device="cuda")
    wb = torch.full((n,), 7.0, dtype=torch.float64, device="cuda")
    assert _call(lib, "sbr_tridiag_eigvals_noalloc", big, big, wb) == 3      # SBR_ENOTSUP
    torch.cuda.synchronize()
    assert bool((wb == 7.0).all())
