"""Write the oracle's eigenvalues of the two full-size Gaussian workloads.

Stored expected values for the GPU parity tests at the benchmark sizes, where
the CPU oracle takes too long to run inside a test:

* n = 32768, A = (G + G^T)/2, G_ij ~ N(0, 1), seed (1604, 3703, 2, 0)
  -> ``oracle_eigs_n32768_gaussian.npy``
* n = 16384, same recipe, seed (1604, 3703, 3, 0)
  -> ``oracle_eigs_n16384_gaussian.npy``

Each file holds the ascending eigenvalues from ``oracle.eigvalsh`` (FP64
Householder tridiagonalisation plus Sturm bisection).  ``oracle_golden.json``
records, per workload, the SHA-256 of the generated matrix bytes (float64,
C order), so a test can tell that the generator still produces the matrix the
values belong to, and the oracle's timings and thread count.

This script calls only the oracle and the seeded input generators.  Run it
from the repository root:

    OMP_NUM_THREADS=6 python tests/golden/make_oracle_golden.py [n32768|n16384 ...]

The n = 32768 case needs about 26 GB of host memory and on the order of an
hour on eight cores (the unblocked reduction streams the trailing matrix from
DRAM twice per column).
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
for p in (ROOT, os.path.dirname(HERE)):
    if p not in sys.path:
        sys.path.insert(0, p)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import sbr_inputs as si  # noqa: E402
from golden_io import META, load_meta, matrix_sha256  # noqa: E402

CASES = {
    "n32768": (si.CFG_LARGE, 0, 32768, "oracle_eigs_n32768_gaussian.npy"),
    "n16384": (si.CFG_FP32, 0, 16384, "oracle_eigs_n16384_gaussian.npy"),
}


def run(name: str) -> None:
    cfg, inp, n, fname = CASES[name]
    oracle.build()
    t0 = time.time()
    A, _ = si.workload(cfg, inp)
    assert A.shape == (n, n)
    digest = matrix_sha256(A)
    t_gen = time.time() - t0
    print("%s: generated in %.1f s, sha256 %s" % (name, t_gen, digest), flush=True)
    w, (t_tri, t_bis) = oracle.eigvalsh(A, return_seconds=True)
    del A
    print("%s: oracle tridiagonalisation %.1f s, bisection %.1f s" % (name, t_tri, t_bis), flush=True)
    assert np.all(np.diff(w) >= 0.0)
    np.save(os.path.join(HERE, fname), w)
    meta = load_meta()
    meta[name] = {
        "workload": "(G + G^T)/2, G_ij ~ N(0,1), n = %d" % n,
        "seed": [*si.SEED_PREFIX, cfg, inp],
        "generator": "sbr_inputs.workload(%d, %d)" % (cfg, inp),
        "matrix_sha256": digest,
        "file": fname,
        "oracle_seconds": {"tridiagonalize": round(t_tri, 1), "bisect": round(t_bis, 1)},
        "oracle_threads": oracle.num_threads(),
        "norm2": float(np.max(np.abs(w))),
    }
    with open(META, "w") as f:
        json.dump(meta, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    for nm in (sys.argv[1:] or ["n16384", "n32768"]):
        run(nm)
