"""Write the 2p-bit reference solutions that bench.py measures the QD LU's
error against, from the CPU oracle only.

For each input (quad-double, n = 2048): the matrix A from the seeded
generator in workloads/, b = A 1 formed exactly and rounded to QD (as the
GPU run forms it), both converted to p' = 448 >= 2 * 212 bits (the exact
value of every QD entry, rounded once to p' bits), then the oracle's p'-bit
LU with partial pivoting and substitution (oracle/lfloat.c: every operation
rounded once to p' bits).  Stored: the solution's mantissas, exponents and
signs (npz, element-major), the seed and the generator.

Inputs (the M* workloads besides the Lotkin matrix, whose condition number
leaves no correct bit at QD precision, Sec. 4.3):
  * wellcond: R + n I, R random expansions (a stand-in for the paper's
    diagonally dominant random matrices, Sec. 4.2);
  * graded40: D R D with D = diag(2^round(log2 10^(20 i/(n-1)))), R with
    N(0, 1) leading components (condition about 10^40).

Run: python tests/golden/make_ref2p.py   (about a minute per input on 8 cores)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle.lfloat as LF  # noqa: E402
import workloads as W  # noqa: E402

N, NC, NL = 2048, 4, 7
INPUTS = {"wellcond": 20261001, "graded40": 20261002}


def matrix(kind, n=N, nc=NC):
    rng = np.random.default_rng(INPUTS[kind])
    if kind == "wellcond":
        return W.wellcond(n, nc, rng)
    return W.graded(n, nc, 40.0, rng)


def main(kinds):
    for kind in kinds:
        t0 = time.time()
        A = matrix(kind)
        b = W.rhs_ones(A)
        Al = LF.from_doubles(A, NL)           # (cols, rows, NL)
        bl = LF.from_doubles(b, NL)           # (1, n, NL)
        LU, ipiv, info = LF.getrf(Al)
        X = LF.getrs(LU, ipiv, bl)
        path = os.path.join(HERE, f"ref2p_qd{N}_{kind}.npz")
        np.savez_compressed(path, m=X[0][0], e=X[1][0], s=X[2][0], info=np.int32(info),
                            seed=np.int64(INPUTS[kind]), nl=np.int32(NL))
        print("wrote", path, f"({time.time() - t0:.1f} s, info {info})", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(INPUTS))
