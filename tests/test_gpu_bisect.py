"""Sturm bisection on adversarial tridiagonals, GPU against the oracle.

The count recurrence on the GPU takes 1/q from a Newton-refined hardware
reciprocal instead of a division; the oracle divides.  Kahan's argument that
the count is monotone in x assumes correctly rounded, monotone arithmetic, so
these cases aim at the places where a count could break: eigenvalues spread
over many orders of magnitude (graded diagonal), tight pairs of eigenvalues
(Wilkinson matrices glued by 1e-14), exact zero pivots (integer diagonals with
zero couplings), and pivots that underflow.  Both entry points run them: the
tridiagonal call (bisect_kernel) and the batched solver on the same matrices
in dense form, whose reductions leave a tridiagonal input as it is, so its
bisection (batched_bisect_kernel) sees the same (d, e).

Bar: max |lam - lam_oracle| <= 4 eps ||T||_2, the accuracy of bisection
itself (both sides stop at the same width).
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


@pytest.mark.parametrize("name", ["glued_wilkinson", "integer_zero_pivots", "graded", "underflowing_pivots"])
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
