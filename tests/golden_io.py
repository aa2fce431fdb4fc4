"""Reading the stored oracle eigenvalues under tests/golden/ (written by
tests/golden/make_oracle_golden.py) and fingerprinting the matrices they
belong to."""
import hashlib
import json
import os

import numpy as np

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
META = os.path.join(GOLDEN_DIR, "oracle_golden.json")


def matrix_sha256(A: np.ndarray) -> str:
    """SHA-256 of the float64 C-order bytes of A, hashed in row blocks."""
    A = np.asarray(A, dtype=np.float64)
    h = hashlib.sha256()
    rows = max(1, (1 << 24) // max(A.shape[1], 1))
    for r0 in range(0, A.shape[0], rows):
        h.update(np.ascontiguousarray(A[r0:r0 + rows]).tobytes())
    return h.hexdigest()


def load_meta() -> dict:
    if os.path.exists(META):
        with open(META) as f:
            return json.load(f)
    return {}


def load(name: str):
    """(record, eigenvalues) of a stored workload, e.g. name = "n32768"."""
    rec = load_meta()[name]
    return rec, np.load(os.path.join(GOLDEN_DIR, rec["file"]), allow_pickle=False)
