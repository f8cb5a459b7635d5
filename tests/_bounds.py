"""Rigorous error bounds for solutions of the five-point systems (test
infrastructure; the oracle's product and solver only, nothing from the device
path).

The operator is a symmetric M-matrix (positive diagonal, non-positive
couplings; land rows are identity rows).  For such a matrix and any vector
v > 0, the Collatz-Wielandt inequality gives

    lambda_min(A) >= min_i (A v)_i / v_i,

so ||A^-1||_2 <= 1 / that minimum.  With v the (approximate) solution of
A v = 1 the bound is close to ||A^-1 1||_inf^-1, the classical estimate for
M-matrices; any inaccuracy of v only loosens the bound, never invalidates
it.  Two approximate solutions x, y of A x = b then satisfy

    ||x - y||_2 <= (||b - A x||_2 + ||b - A y||_2) / lambda_min_lower.
"""
import numpy as np


def lambda_min_lower(ora, p, F=None, tol=1e-8):
    """A lower bound of the smallest eigenvalue of A (Collatz-Wielandt with
    v = A^-1 1 from the oracle's PCG; Jacobi factor unless F is given)."""
    if F is None:
        F = ora.ainv_setup(p, np.inf)
    one = np.ones(p.n)
    v = ora.pcg(p, F, b=one, tol=tol).x
    if not np.all(v > 0):
        raise AssertionError("A^-1 1 must be positive for an M-matrix")
    av = ora.spmv(p, v)
    # the product's own rounding: at most 8 ulp of the magnitude of each row
    mag = ora.spmv(type(p)(p.nx, p.ny, p.periodic, np.abs(p.diag), np.abs(p.ae), np.abs(p.an),
                           p.ocean, p.b), v)
    lo = np.min((av - 8 * np.finfo(np.float64).eps * mag) / v)
    if not lo > 0:
        raise AssertionError("no positive lower bound")
    return float(lo)


def solution_gap_bound(ora, p, b, x, y, lam_lo):
    """Upper bound of ||x - y||_2 for two approximate solutions of A z = b."""
    rx = np.linalg.norm(b - ora.spmv(p, x))
    ry = np.linalg.norm(b - ora.spmv(p, y))
    return 1.001 * (rx + ry) / lam_lo
