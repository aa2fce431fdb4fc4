"""Helpers shared by the GPU tests (column-major views of numpy arrays)."""
import numpy as np
import torch


def dev():
    return torch.device("cuda:0")


def to_col(M: np.ndarray, ld: int | None = None) -> torch.Tensor:
    """Column-major device copy of the rows x cols array M, as a torch tensor
    of shape (cols, ld) (row-major storage of the transpose)."""
    M = np.asarray(M, dtype=np.float64)
    rows, cols = M.shape
    ld = rows if ld is None else ld
    buf = np.zeros((cols, ld))
    buf[:, :rows] = M.T
    return torch.from_numpy(buf).to(dev())


def from_col(t: torch.Tensor, rows: int) -> np.ndarray:
    """Inverse of to_col: the rows x cols column-major matrix held in t."""
    return t.detach().cpu().numpy()[:, :rows].T.copy()


def band_to_dense(band: np.ndarray, n: int, keep: int | None = None) -> np.ndarray:
    """Symmetric dense matrix from band storage band[j, d] = B(j + d, j)."""
    ld = band.shape[1]
    keep = ld - 1 if keep is None else keep
    A = np.zeros((n, n))
    for d in range(min(ld, keep + 1, n)):
        idx = np.arange(n - d)
        A[idx + d, idx] = band[: n - d, d]
        A[idx, idx + d] = band[: n - d, d]
    return A


def random_band(n: int, b: int, rng) -> np.ndarray:
    """Symmetric matrix with exactly bandwidth b (Gaussian entries)."""
    A = rng.standard_normal((n, n))
    A = 0.5 * (A + A.T)
    i, j = np.indices((n, n))
    A[np.abs(i - j) > b] = 0.0
    return A
