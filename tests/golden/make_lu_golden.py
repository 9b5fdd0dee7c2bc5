"""Write the expected values of the full-size QD Lotkin LU (n = 2048, panel
width b = 256 and b = 128, Ozaki-II INT8 Schur updates) from the CPU oracle
only.

Stores the pivot vector, info, SHA-256 digests of the factor array and of the
solution of A x = A*ones (little-endian float64 bytes, shape (cols, rows, 4)),
and a few hundred sampled factor entries.  Run:
python tests/golden/make_lu_golden.py [b ...]   (default: 256 128; about two
minutes per panel width on 8 cores).
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402


def main(n=2048, b=256, nc=4):
    t0 = time.time()
    A = W.lotkin(n, nc)
    rhs = W.rhs_ones(A)
    LU, ipiv, info, tm = O.getrf(A, b, O.METHOD_OZAKI)
    X = O.getrs(LU, ipiv, rhs)
    rng = np.random.default_rng(7)
    idx = rng.integers(0, n, size=(256, 2))
    out = {
        "what": f"oracle getrf+getrs, Lotkin QD n={n} b={b}, Ozaki-II INT8 (plan rule of Sec. 3.2)",
        "n": n, "b": b, "nc": nc, "info": int(info),
        "ipiv": [int(v) for v in ipiv],
        "lu_sha256": hashlib.sha256(np.ascontiguousarray(LU, dtype="<f8").tobytes()).hexdigest(),
        "x_sha256": hashlib.sha256(np.ascontiguousarray(X, dtype="<f8").tobytes()).hexdigest(),
        "samples": [[int(i), int(j), [float(v) for v in LU[j, i]]] for i, j in idx],
        "oracle_seconds": time.time() - t0,
    }
    path = os.path.join(HERE, f"lu_lotkin_qd{n}_b{b}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, "in", round(time.time() - t0, 1), "s")


if __name__ == "__main__":
    for blk in [int(a) for a in sys.argv[1:]] or [256, 128]:
        main(b=blk)
