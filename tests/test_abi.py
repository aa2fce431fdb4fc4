"""CPU-side checks of the C ABI: the library loads, exports every function the
headers declare, and rejects invalid arguments on the host (LAPACK-style
negative codes) before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in ("sbr.h", "sbr_stages.h"):
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(sbr_\w+)\s*\(", src))
    return names


@pytest.fixture(scope="module")
def sbr():
    import paper_1604_03703_amd as m
    return m


def test_every_declared_symbol_is_exported(sbr):
    lib = sbr.lib()
    declared = _declared()
    assert {"sbr_syev_eigvals", "sbr_syev_eigvals_ex", "sbr_syev_eigvals_batched",
            "sbr_tridiag_eigvals", "sbr_plan_create", "sbr_plan_destroy",
            "sbr_workspace_size"} <= declared
    for name in declared:
        assert hasattr(lib, name), name
    assert set(sbr.EXPORTED) == declared


def test_invalid_arguments_rejected_on_host(sbr):
    lib = sbr.lib()
    null = ctypes.c_void_p(0)
    dummy = ctypes.c_void_p(16)
    assert lib.sbr_syev_eigvals(-1, dummy, 1, 0, null, dummy) == -1
    assert lib.sbr_syev_eigvals(4, null, 4, 0, null, dummy) == -2
    assert lib.sbr_syev_eigvals(4, dummy, 3, 0, null, dummy) == -3
    assert lib.sbr_syev_eigvals(4, dummy, 4, 3, null, dummy) == -4       # not a power of two
    assert lib.sbr_syev_eigvals(4, dummy, 4, 256, null, dummy) == -4     # too wide
    assert lib.sbr_syev_eigvals(4, dummy, 4, 0, null, null) == -6
    assert lib.sbr_syev_eigvals(0, null, 1, 0, null, null) == 0          # empty problem: no-op
    assert lib.sbr_tridiag_eigvals(3, dummy, null, null, dummy) == -3
    assert lib.sbr_syev_eigvals_ex(null, 4, dummy, 4, 0, 0, null, dummy) == -1
    assert lib.sbr_plan_create(None, 10, 0, 0) == -1
    assert lib.sbr_gemm(2, 0, 1, 1, 1, 1.0, dummy, 1, dummy, 1, 0.0, dummy, 1, 0, null) == -1
    assert lib.sbr_band_halve(null, 10, dummy, 3, 2, 0, null) == -1
    assert lib.sbr_band_reduce(null, 10, dummy, 65, 32, 8, 0, null) == -1
    assert lib.sbr_plan_set_band_stages(null, 0, None) == -1
    assert lib.sbr_plan_get_band_stages(null, 10, 32, None, 0) == -1
    assert lib.sbr_plan_set_update_depth(null, 2) == -1


def test_unsupported_sizes_rejected_on_host(sbr):
    # SBR_ENOTSUP (3), returned before any device call
    lib = sbr.lib()
    null = ctypes.c_void_p(0)
    dummy = ctypes.c_void_p(16)
    # the Sturm counts of the bisection are 32-bit
    assert lib.sbr_tridiag_eigvals(2 ** 31, dummy, dummy, null, dummy) == 3
    assert lib.sbr_tridiag_eigvals(0, null, null, null, null) == 0
    # the symmetric product addresses 128 columns of A with 32-bit byte offsets
    assert lib.sbr_symm_lower(10, 4, dummy, 1 << 21, dummy, 10, dummy, 10, 0, null) == 3


def test_workspace_size_and_default_band(sbr):
    lib = sbr.lib()
    sz = ctypes.c_size_t()
    assert lib.sbr_workspace_size(8192, 64, 0, ctypes.byref(sz)) == 0
    small = sz.value
    assert lib.sbr_workspace_size(32768, 128, 0, ctypes.byref(sz)) == 0
    big = sz.value
    assert 0 < small < big
    # n x b buffers dominate: at least five of them
    assert big >= 5 * 32768 * 128 * 8
    assert lib.sbr_workspace_size(100, 12, 0, ctypes.byref(sz)) == -2
    assert sbr.default_band(256) == 16 and sbr.default_band(8192) == 64 and sbr.default_band(32768) == 128


def test_binding_has_no_cpu_fallback(sbr):
    import torch
    A = torch.zeros((4, 4), dtype=torch.float64)       # a CPU tensor is refused, not computed
    with pytest.raises(TypeError):
        sbr.eigvalsh(A)
