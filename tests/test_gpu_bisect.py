"""Sturm bisection on adversarial tridiagonals, GPU against the oracle.

The GPU counts eigenvalues below x as the sign changes of the leading
principal minors (their three-term recurrence on data scaled by a power of
two, rescaled every 16 steps, with a recount by the guarded ratio recurrence
when the minors come near underflow), starting each index from a cell of a
shared first grid; the oracle counts negative pivots of the ratio recurrence
with a division and bisects the whole interval.  These cases aim at the
places where either could break: eigenvalues spread over many orders of
magnitude (graded diagonal), tight pairs (Wilkinson matrices glued by 1e-14,
2 x 2 blocks split by 1e-13), exact zero pivots (integer diagonals with zero
couplings), pivots that underflow, one eigenvalue of multiplicity n (every
index in one grid cell), no couplings at all (a split at every step), and
matrices scaled by 1e150 and 1e-140.  Both entry points run them: the
tridiagonal call (sturm_grid_kernel, bisect_kernel) and the batched solver on
the same matrices in dense form, whose reductions leave a tridiagonal input
as it is, so its bisection (batched_bisect_kernel) sees the same (d, e).

Bar: max |lam - lam_oracle| <= 4 eps ||T||_2, the accuracy of bisection
itself (both sides stop no wider than the same width).
"""
import numpy as np
import pytest
import torch

from bisect_cases import CASES

pytestmark = pytest.mark.gpu

EPS64 = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def sbr():
    import paper_1604_03703_amd as m
    assert torch.cuda.is_available()
    return m


@pytest.mark.parametrize("name", sorted(CASES))
def test_tridiag_eigvals_adversarial(sbr, oracle_mod, name):
    d, e = CASES[name]
    print("bisect", name, len(d), flush=True)
    ref = oracle_mod.tridiag_eigvals(d, e)
    w = sbr.tridiag_eigvals(torch.from_numpy(d).cuda(), torch.from_numpy(e).cuda()).cpu().numpy()
    nrm = max(np.max(np.abs(ref)), 1e-300)
    err = np.max(np.abs(w - ref))
    print("%s: max err %.3e (x ||T||)" % (name, err / nrm), flush=True)
    assert np.all(np.diff(w) >= 0.0)
    assert err <= 4 * EPS64 * nrm


@pytest.mark.parametrize("name", ["glued_wilkinson", "integer_zero_pivots", "graded", "underflowing_pivots",
                                  "identity", "diagonal_only", "scaled_1e150", "scaled_1e-140", "pair_clusters"])
def test_batched_bisection_adversarial(sbr, oracle_mod, name):
    d, e = CASES[name]
    n = len(d)
    if n > 512:
        pytest.skip("batched kernels take n <= 512")
    print("batched bisect", name, n, flush=True)
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    ref = oracle_mod.tridiag_eigvals(d, e)
    mats = [torch.from_numpy(T.copy()).cuda() for _ in range(3)]
    ws = sbr.eigvalsh_batched(mats, b0=8)
    torch.cuda.synchronize()
    nrm = max(np.max(np.abs(ref)), 1e-300)
    for w in ws:
        w = w.cpu().numpy()
        err = np.max(np.abs(w - ref))
        print("%s batched: max err %.3e (x ||T||)" % (name, err / nrm), flush=True)
        assert err <= 4 * EPS64 * nrm
