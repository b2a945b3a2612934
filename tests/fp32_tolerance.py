"""The FP32 iterate tolerance of the parity tests.

An FP32 round computes each partial gradient a_j^T r as one FP32 dot product of `terms`
products (m for a dense column, the column's nonzeros for a sparse one) and keeps r and x
in FP32.  The rounding error of such a dot product grows like sqrt(terms) * 2^-24 relative
to the scale of its terms (random rounding), and x itself carries a few units of 2^-24 of
its magnitude, so the iterates follow the FP64 trajectory of the oracle to within
X_TOL(terms) = (sqrt(terms) + 16) * 2^-24 of max(1, ||x||_inf): 9.4e-6 at 20000 rows,
6.9e-6 at 10000, 1.5e-6 for a sparse column of 100 nonzeros.  The iteration contracts, so
these errors do not add up over rounds.  Measured on MI355X over the first 20 rounds of the
full-size workloads: 2.4e-7 (20000 x 100000 LASSO), 6.8e-7 (10000 x 50000 box-nonconvex),
1.6e-7 (sparse 1e5 x 1e6).  Objectives are held to the stated 1e-4 relative target.
"""
import math


def x_tol(terms: int) -> float:
    return (math.sqrt(max(int(terms), 1)) + 16.0) * 2.0 ** -24
