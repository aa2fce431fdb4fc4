"""MI355X-native successive-band-reduction symmetric eigensolver.

Thin ctypes binding over ``lib/libsbr.so`` (the C ABI declared in
``include/sbr.h`` and ``include/sbr_stages.h``).  Every step of the method runs
in the library's HIP kernels; this module only marshals arguments: device
pointers from torch tensors and the current torch stream.  There is no CPU
fallback -- if the library is missing, importing the binding raises.

Layout note: the library works on column-major matrices.  A row-major torch
tensor ``A`` of shape (n, n) is the column-major matrix ``A^T``; for the
symmetric inputs of the eigensolver this is the same matrix.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libsbr.so")

FP64 = 0
FP32_MFMA = 1
_PREC = {"fp64": FP64, "fp32": FP32_MFMA, "fp32_mfma": FP32_MFMA, FP64: FP64, FP32_MFMA: FP32_MFMA}

_i64, _i32, _dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
_vp = ctypes.c_void_p


class SbrError(RuntimeError):
    pass


class _Timing(ctypes.Structure):
    _fields_ = [
        ("ms_total", _dbl), ("ms_f2b", _dbl), ("ms_band", _dbl), ("ms_bisect", _dbl),
        ("ms_update_kernels", _dbl), ("update_launches", _i64),
        ("ms_syr2k", _dbl), ("syr2k_launches", _i64),
        ("ms_symm", _dbl), ("symm_launches", _i64),
        ("ms_stage", _dbl * 8), ("n_stages", _i32),
        ("ms_syr2k_big", _dbl), ("syr2k_big_launches", _i64),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsbr.so not built (run paper_1604_03703_amd.build.build() or "
                          "__graft_entry__.build()); there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "sbr_syev_eigvals": ([_i64, _vp, _i64, _i32, _vp, _vp], ctypes.c_int),
        "sbr_syev_eigvals_ex": ([_vp, _i64, _vp, _i64, _i32, ctypes.c_int, _vp, _vp], ctypes.c_int),
        "sbr_syev_eigvals_batched": ([_vp, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_vp),
                                      ctypes.POINTER(_i64), _i32, ctypes.c_int, _vp,
                                      ctypes.POINTER(_vp)], ctypes.c_int),
        "sbr_tridiag_eigvals": ([_i64, _vp, _vp, _vp, _vp], ctypes.c_int),
        "sbr_tridiag_eigvals_noalloc": ([_i64, _vp, _vp, _vp, _vp], ctypes.c_int),
        "sbr_plan_create": ([ctypes.POINTER(_vp), _i64, _i32, ctypes.c_int], ctypes.c_int),
        "sbr_plan_destroy": ([_vp], ctypes.c_int),
        "sbr_workspace_size": ([_i64, _i32, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "sbr_default_band": ([_i64], _i32),
        "sbr_last_hip_error": ([], ctypes.c_int),
        "sbr_full_to_band": ([_vp, _i64, _vp, _i64, _i32, ctypes.c_int, _vp], ctypes.c_int),
        "sbr_dense_to_band": ([_i64, _vp, _i64, _i32, _vp, _i64, _vp], ctypes.c_int),
        "sbr_band_halve": ([_vp, _i64, _vp, _i64, _i32, ctypes.c_int, _vp], ctypes.c_int),
        "sbr_panel_qr": ([_vp, _i64, _i32, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
        "sbr_gemm": ([_i32, _i32, _i64, _i64, _i64, _dbl, _vp, _i64, _vp, _i64, _dbl, _vp, _i64,
                      ctypes.c_int, _vp], ctypes.c_int),
        "sbr_syr2k_lower": ([_i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, ctypes.c_int, _vp], ctypes.c_int),
        "sbr_symm_lower": ([_i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, ctypes.c_int, _vp], ctypes.c_int),
        "sbr_plan_set_timing": ([_vp, ctypes.c_int], ctypes.c_int),
        "sbr_plan_get_timing": ([_vp, ctypes.POINTER(_Timing)], ctypes.c_int),
        "sbr_plan_set_chase_blocks": ([_vp, _i32], ctypes.c_int),
        "sbr_plan_set_panel_cus": ([_vp, _i32], ctypes.c_int),
        "sbr_plan_status": ([_vp, ctypes.POINTER(_i32)], ctypes.c_int),
        "sbr_plan_set_wait_limit": ([_vp, _i64], ctypes.c_int),
        "sbr_plan_set_group_max_band": ([_vp, _i32], ctypes.c_int),
        "sbr_plan_set_tridiag_band": ([_vp, _i32, _i32], ctypes.c_int),
        "sbr_band_to_tridiag": ([_vp, _i64, _vp, _i64, _i32, _vp], ctypes.c_int),
        "sbr_plan_set_batch_bands": ([_vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32)], ctypes.c_int),
        "sbr_band_reduce": ([_vp, _i64, _vp, _i64, _i32, _i32, ctypes.c_int, _vp], ctypes.c_int),
        "sbr_plan_set_band_stages": ([_vp, _i32, ctypes.POINTER(_i32)], ctypes.c_int),
        "sbr_plan_get_band_stages": ([_vp, _i64, _i32, ctypes.POINTER(_i32), _i32], ctypes.c_int),
        "sbr_plan_set_update_depth": ([_vp, _i32], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = _load()
EXPORTED = (
    "sbr_syev_eigvals", "sbr_syev_eigvals_ex", "sbr_syev_eigvals_batched", "sbr_tridiag_eigvals",
    "sbr_plan_create", "sbr_plan_destroy", "sbr_workspace_size", "sbr_default_band",
    "sbr_last_hip_error", "sbr_full_to_band", "sbr_dense_to_band", "sbr_band_halve", "sbr_panel_qr",
    "sbr_gemm", "sbr_syr2k_lower", "sbr_symm_lower", "sbr_plan_set_timing", "sbr_plan_get_timing",
    "sbr_plan_set_chase_blocks", "sbr_plan_set_panel_cus", "sbr_plan_status",
    "sbr_plan_set_wait_limit", "sbr_plan_set_group_max_band", "sbr_tridiag_eigvals_noalloc",
    "sbr_plan_set_tridiag_band", "sbr_band_to_tridiag", "sbr_plan_set_batch_bands",
    "sbr_band_reduce", "sbr_plan_set_band_stages", "sbr_plan_get_band_stages", "sbr_plan_set_update_depth",
)

STATUS_STALLED = 1      # SBR_STATUS_STALLED
STATUS_NONFINITE = 2    # SBR_STATUS_NONFINITE


def lib():
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        extra = ""
        if rc == 2:
            extra = " (hipError %d)" % _lib.sbr_last_hip_error()
        raise SbrError("%s failed with code %d%s" % (what, rc, extra))


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f64(t: torch.Tensor, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError("%s must be a CUDA float64 tensor" % name)
    return ctypes.c_void_p(t.data_ptr())


def _prec(p):
    try:
        return _PREC[p]
    except KeyError:
        raise ValueError("precision must be 'fp64' or 'fp32_mfma'") from None


def default_band(n: int) -> int:
    return int(_lib.sbr_default_band(int(n)))


class Plan:
    """Device workspace for problems up to ``n_max`` (grows on demand)."""

    def __init__(self, n_max: int = 0, batch_max: int = 0, precision="fp64"):
        h = ctypes.c_void_p()
        _check(_lib.sbr_plan_create(ctypes.byref(h), int(n_max), int(batch_max), _prec(precision)),
               "sbr_plan_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def set_timing(self, on=True):
        """True / 1: every event pair; 2: phase totals and bulk SYR2K pairs only; False / 0: off."""
        level = 2 if on == 2 else (1 if on else 0)
        _check(_lib.sbr_plan_set_timing(self._h, level), "sbr_plan_set_timing")

    def timing(self) -> dict:
        t = _Timing()
        _check(_lib.sbr_plan_get_timing(self._h, ctypes.byref(t)), "sbr_plan_get_timing")
        out = {f: getattr(t, f) for f, _ in _Timing._fields_ if f != "ms_stage"}
        out["ms_stage"] = [t.ms_stage[i] for i in range(t.n_stages)]
        return out

    def set_chase_blocks(self, max_blocks: int):
        _check(_lib.sbr_plan_set_chase_blocks(self._h, int(max_blocks)), "sbr_plan_set_chase_blocks")

    def set_panel_cus(self, cus: int):
        _check(_lib.sbr_plan_set_panel_cus(self._h, int(cus)), "sbr_plan_set_panel_cus")

    def set_update_depth(self, depth: int):
        """Panels whose two-sided updates are aggregated (Eq. (4.2)); 1 = per panel."""
        _check(_lib.sbr_plan_set_update_depth(self._h, int(depth)), "sbr_plan_set_update_depth")

    def set_group_max_band(self, b: int):
        _check(_lib.sbr_plan_set_group_max_band(self._h, int(b)), "sbr_plan_set_group_max_band")

    def set_tridiag_band(self, b: int, variant: int = 0):
        _check(_lib.sbr_plan_set_tridiag_band(self._h, int(b), int(variant)), "sbr_plan_set_tridiag_band")

    def set_batch_bands(self, table):
        """Band per size bucket for the batched form with b0 = 0: a list of
        (n_max, band) pairs, ascending n_max ([] = the built-in rule)."""
        k = len(table)
        nm = (_i32 * max(k, 1))(*[int(x) for x, _ in table])
        bd = (_i32 * max(k, 1))(*[int(y) for _, y in table])
        _check(_lib.sbr_plan_set_batch_bands(self._h, k, nm, bd), "sbr_plan_set_batch_bands")

    def use_tuned_batch_bands(self, precision="fp64") -> list:
        """Apply the band table a tuning run stored for this device (see
        autotune.py); returns the table ([] when there is none)."""
        from . import autotune
        table = autotune.batch_table(precision)
        self.set_batch_bands(table)
        return table

    def set_band_stages(self, widths):
        """Band widths a solve reduces to, in decreasing order (powers of two);
        [] restores the built-in sequence."""
        k = len(widths)
        arr = (_i32 * max(k, 1))(*[int(x) for x in widths])
        _check(_lib.sbr_plan_set_band_stages(self._h, k, arr), "sbr_plan_set_band_stages")

    def band_stages(self, n: int, b0: int) -> list:
        """The band width after each band-to-band stage of a solve of order n
        from band b0 with the current settings."""
        arr = (_i32 * 32)()
        rc = _lib.sbr_plan_get_band_stages(self._h, int(n), int(b0), arr, 32)
        if rc < 0:
            raise SbrError("sbr_plan_get_band_stages failed with code %d" % rc)
        return [int(arr[i]) for i in range(min(rc, 32))]

    def use_tuned_stages(self, n: int, b0: int, precision="fp64") -> list:
        """Apply the band-stage sequence (and direct-stage launch shape) a
        tuning run stored for this device and the nearest order to n (see
        autotune.py); returns the widths ([] when there is none: the built-in
        sequence stays)."""
        from . import autotune
        widths, variant = autotune.stage_sequence(n, b0, precision)
        if widths:
            self.set_band_stages(widths)
            self.set_tridiag_band(4, variant)
        return widths

    def set_wait_limit(self, ticks: int):
        _check(_lib.sbr_plan_set_wait_limit(self._h, int(ticks)), "sbr_plan_set_wait_limit")

    def status(self) -> int:
        """SBR_STATUS_* bits raised since the previous query (waits for the device, then clears)."""
        v = _i32()
        _check(_lib.sbr_plan_status(self._h, ctypes.byref(v)), "sbr_plan_status")
        return int(v.value)

    def close(self):
        if self._h:
            _lib.sbr_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _leading_dim(A: torch.Tensor) -> int:
    """Leading dimension of the column-major matrix behind A, or 0 when A's
    layout is not one: rows of A (= columns of the column-major matrix, A
    being symmetric) must be contiguous and at least n apart."""
    n = A.shape[0]
    if n <= 1:
        return max(n, 1)
    if A.stride(1) == 1 and A.stride(0) >= n:
        return int(A.stride(0))
    return 0


def eigvalsh(A: torch.Tensor, b0: int = 0, precision="fp64", plan: Plan | None = None,
             overwrite: bool = False, stream=None, out: torch.Tensor | None = None) -> torch.Tensor:
    """Ascending eigenvalues of the symmetric CUDA float64 matrix ``A``.

    With ``overwrite`` the solver works in A's own storage when its rows are
    contiguous (a view of a wider buffer passes that buffer's row stride as the
    leading dimension); otherwise on a contiguous copy."""
    n = A.shape[0]
    if A.dim() != 2 or A.shape[1] != n:
        raise ValueError("A must be square")
    lda = _leading_dim(A) if overwrite else 0
    work = A if lda else A.contiguous().clone()
    lda = lda or max(n, 1)
    w = out if out is not None else torch.empty(n, dtype=torch.float64, device=A.device)
    if plan is None and _prec(precision) == FP64:
        rc = _lib.sbr_syev_eigvals(n, _dev_f64(work, "A"), lda, int(b0), _stream(stream),
                                   _dev_f64(w, "w"))
        _check(rc, "sbr_syev_eigvals")
    else:
        if plan is None:
            plan = Plan(n, 0, precision)
        rc = _lib.sbr_syev_eigvals_ex(plan.handle, n, _dev_f64(work, "A"), lda, int(b0),
                                      _prec(precision), _stream(stream), _dev_f64(w, "w"))
        _check(rc, "sbr_syev_eigvals_ex")
    return w


class BatchedSolve:
    """A prepared batched call: the matrices (solved in place), the output
    vectors and the plan are checked and marshalled once; every ``run()``
    hands the same pointer arrays to ``sbr_syev_eigvals_batched``, which then
    replays its captured launch (the pattern of a self-consistent-field loop
    that refills the same buffers every iteration)."""

    def __init__(self, mats, b0: int = 0, precision="fp64", plan: Plan | None = None, out=None):
        k = len(mats)
        for m in mats:
            if m.dim() != 2 or m.shape[0] != m.shape[1]:
                raise ValueError("every matrix must be square")
            if not _leading_dim(m):
                raise ValueError("every matrix needs contiguous rows at least n apart (it is solved in place)")
        if out is None:
            out = [torch.empty(int(m.shape[0]), dtype=torch.float64, device=m.device) for m in mats]
        elif len(out) != k:
            raise ValueError("out must have one vector per matrix")
        self.mats, self.out = list(mats), list(out)
        self._k = k
        self._ns = (_i64 * k)(*[int(m.shape[0]) for m in mats])
        self._ldas = (_i64 * k)(*[_leading_dim(m) for m in mats])
        self._aps = (_vp * k)(*[_dev_f64(m, "A").value for m in mats])
        self._wps = (_vp * k)(*[_dev_f64(x, "w").value for x in self.out])
        if plan is None:
            plan = Plan(max(int(m.shape[0]) for m in mats) if k else 0, k, precision)
            if b0 == 0:
                plan.use_tuned_batch_bands(precision)
        self.plan, self._b0, self._prec = plan, int(b0), _prec(precision)

    def run(self, stream=None):
        rc = _lib.sbr_syev_eigvals_batched(self.plan.handle, self._k, self._ns, self._aps, self._ldas, self._b0,
                                           self._prec, _stream(stream), self._wps)
        _check(rc, "sbr_syev_eigvals_batched")
        return self.out


def eigvalsh_batched(mats, b0: int = 0, precision="fp64", plan: Plan | None = None, stream=None, out=None):
    """Eigenvalues of a list of symmetric CUDA float64 matrices (overwritten).

    ``out``: optional list of float64 CUDA vectors (one per matrix) to write
    into; with the same matrices and outputs a plan replays its captured
    launch instead of rebuilding it (``BatchedSolve`` also keeps the
    marshalled arguments)."""
    return BatchedSolve(mats, b0, precision, plan, out).run(stream)


def tridiag_eigvals(d: torch.Tensor, e: torch.Tensor | None, stream=None) -> torch.Tensor:
    n = d.shape[0]
    w = torch.empty(n, dtype=torch.float64, device=d.device)
    ep = _dev_f64(e, "e") if (e is not None and n > 1) else ctypes.c_void_p(0)
    _check(_lib.sbr_tridiag_eigvals(n, _dev_f64(d, "d"), ep, _stream(stream), _dev_f64(w, "w")),
           "sbr_tridiag_eigvals")
    return w


def tridiag_eigvals_noalloc(d: torch.Tensor, e: torch.Tensor | None, out: torch.Tensor, stream=None) -> torch.Tensor:
    """sbr_tridiag_eigvals_noalloc: the library allocates nothing (n <= 2^18);
    the caller provides the output vector."""
    n = d.shape[0]
    ep = _dev_f64(e, "e") if (e is not None and n > 1) else ctypes.c_void_p(0)
    _check(_lib.sbr_tridiag_eigvals_noalloc(n, _dev_f64(d, "d"), ep, _stream(stream), _dev_f64(out, "w")),
           "sbr_tridiag_eigvals_noalloc")
    return out


def full_to_band(A: torch.Tensor, b: int, plan: Plan, precision="fp64", stream=None) -> torch.Tensor:
    """Reduce the symmetric A (in place, column-major view) to bandwidth b.

    Returns A; its column-major lower band (= the row-major upper band of the
    torch tensor) holds the band matrix, the rest of that triangle is zero.
    """
    n = A.shape[0]
    _check(_lib.sbr_full_to_band(plan.handle, n, _dev_f64(A, "A"), max(n, 1), int(b), _prec(precision),
                                 _stream(stream)), "sbr_full_to_band")
    return A


def dense_to_band(A: torch.Tensor, b: int, ldband: int, stream=None) -> torch.Tensor:
    """Band storage (torch shape (n, ldband): row j holds B(j + d, j) at column d)."""
    n = A.shape[0]
    band = torch.empty((n, ldband), dtype=torch.float64, device=A.device)
    _check(_lib.sbr_dense_to_band(n, _dev_f64(A, "A"), max(n, 1), int(b), _dev_f64(band, "band"),
                                  int(ldband), _stream(stream)), "sbr_dense_to_band")
    return band


def band_halve(band: torch.Tensor, b: int, plan: Plan, precision="fp64", stream=None) -> torch.Tensor:
    n, ld = band.shape
    _check(_lib.sbr_band_halve(plan.handle, n, _dev_f64(band, "band"), ld, int(b), _prec(precision),
                               _stream(stream)), "sbr_band_halve")
    return band


def band_reduce(band: torch.Tensor, b: int, h: int, plan: Plan, precision="fp64", stream=None) -> torch.Tensor:
    """Band of width b reduced to width h = b / k in place (one stage)."""
    n, ld = band.shape
    _check(_lib.sbr_band_reduce(plan.handle, n, _dev_f64(band, "band"), ld, int(b), int(h), _prec(precision),
                                _stream(stream)), "sbr_band_reduce")
    return band


def band_to_tridiag(band: torch.Tensor, b: int, plan: Plan, stream=None) -> torch.Tensor:
    """Band of width b (4, 8, 16) straight to tridiagonal form, in place."""
    n, ld = band.shape
    _check(_lib.sbr_band_to_tridiag(plan.handle, n, _dev_f64(band, "band"), ld, int(b), _stream(stream)),
           "sbr_band_to_tridiag")
    return band


def panel_qr(P_colmajor: torch.Tensor, b: int, plan: Plan, stream=None):
    """TSQR + Householder reconstruction of the m x b panel given column-major
    as a torch tensor of shape (b, m).  Returns column-major (Q, R, U, T, S)."""
    bb, m = P_colmajor.shape
    assert bb == b
    dev = P_colmajor.device
    Q = torch.empty((b, m), dtype=torch.float64, device=dev)
    U = torch.empty((b, m), dtype=torch.float64, device=dev)
    R = torch.empty((b, b), dtype=torch.float64, device=dev)
    T = torch.empty((b, b), dtype=torch.float64, device=dev)
    S = torch.empty(b, dtype=torch.float64, device=dev)
    _check(_lib.sbr_panel_qr(plan.handle, m, b, _dev_f64(P_colmajor, "P"), m, _dev_f64(Q, "Q"),
                             _dev_f64(R, "R"), _dev_f64(U, "U"), _dev_f64(T, "T"), _dev_f64(S, "S"),
                             _stream(stream)), "sbr_panel_qr")
    return Q, R, U, T, S


def gemm(transa: int, transb: int, m: int, n: int, k: int, alpha: float, A, lda: int, B, ldb: int,
         beta: float, C, ldc: int, precision="fp64", stream=None):
    _check(_lib.sbr_gemm(transa, transb, m, n, k, alpha, _dev_f64(A, "A"), lda, _dev_f64(B, "B"), ldb, beta,
                         _dev_f64(C, "C"), ldc, _prec(precision), _stream(stream)), "sbr_gemm")
    return C


def syr2k_lower(m: int, k: int, U, ldu: int, V, ldv: int, C, ldc: int, precision="fp64", stream=None):
    _check(_lib.sbr_syr2k_lower(m, k, _dev_f64(U, "U"), ldu, _dev_f64(V, "V"), ldv, _dev_f64(C, "C"), ldc,
                                _prec(precision), _stream(stream)), "sbr_syr2k_lower")
    return C


def symm_lower(m: int, k: int, A, lda: int, Y, ldy: int, W, ldw: int, precision="fp64", stream=None):
    _check(_lib.sbr_symm_lower(m, k, _dev_f64(A, "A"), lda, _dev_f64(Y, "Y"), ldy, _dev_f64(W, "W"), ldw,
                               _prec(precision), _stream(stream)), "sbr_symm_lower")
    return W
