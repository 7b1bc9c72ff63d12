"""Finite-difference and interpolation weights on arbitrary 1D nodes (oracle).

Section 3.1 obtains the weights of the staggered first-derivative operators
D+ / D- and of the source/receiver interpolation from the inverse of the
transposed Vandermonde matrix V^T(x_0 - x, ..., x_n - x): row 0 of the inverse
gives interpolation weights at x, row 1 gives first-derivative weights at x.
Those rows are exactly the weights of the Lagrange interpolating polynomial
and of its derivative.  The oracle computes them with Fornberg's recursion
(B. Fornberg, Math. Comp. 51 (1988) 699-706), a different algorithm from the
Vandermonde solve, so the two table builders cross-check each other.
"""
from __future__ import annotations

import numpy as np


def fornberg(z: float, nodes: np.ndarray, m: int) -> np.ndarray:
    """Weights c[j, k] such that sum_j c[j, k] f(nodes[j]) approximates the
    k-th derivative of f at z, k = 0..m, exact for polynomials of degree
    < len(nodes).  Fornberg's recursion over nodes and derivative order."""
    x = np.asarray(nodes, dtype=np.float64)
    n = len(x)
    c = np.zeros((n, m + 1))
    c[0, 0] = 1.0
    prod_prev = 1.0
    dz_prev = x[0] - z
    for i in range(1, n):
        top = min(i, m)
        prod = 1.0
        dz_i = x[i] - z
        for j in range(i):
            dx_ij = x[i] - x[j]
            prod *= dx_ij
            if j == i - 1:
                # the new node i: weights from the previous node's column
                for k in range(top, 0, -1):
                    c[i, k] = prod_prev * (k * c[i - 1, k - 1] - dz_prev * c[i - 1, k]) / prod
                c[i, 0] = -prod_prev * dz_prev * c[i - 1, 0] / prod
            # update the weights of the older node j
            for k in range(top, 0, -1):
                c[j, k] = (dz_i * c[j, k] - k * c[j, k - 1]) / dx_ij
            c[j, 0] = dz_i * c[j, 0] / dx_ij
        prod_prev = prod
        dz_prev = dz_i
    return c


def lagrange_weights(z: float, nodes: np.ndarray) -> np.ndarray:
    """Lagrange basis values L_j(z) = prod_{m != j} (z - x_m)/(x_j - x_m):
    the interpolation row (row 0) of the inverse Vandermonde matrix."""
    x = np.asarray(nodes, dtype=np.float64)
    w = np.ones(len(x))
    for j in range(len(x)):
        for m in range(len(x)):
            if m != j:
                w[j] *= (z - x[m]) / (x[j] - x[m])
    return w


def derivative_weights(z: float, nodes: np.ndarray) -> np.ndarray:
    """First-derivative weights at z (row 1 of the inverse Vandermonde)."""
    return fornberg(z, nodes, 1)[:, 1]
