"""1-D polynomial tools for the oracle (FP64).

* Gauss--Legendre nodes/weights: solution points of the hexahedra and flux points
  on their faces (tensor products of these, Sec. "Flux Reconstruction": solution
  and flux points; the Gauss--Legendre choice is the reading used for the hex
  configurations).
* Lagrange basis on arbitrary nodes (the nodal basis l_zeta with l_zeta(x_sigma) =
  delta, same section).
* Legendre polynomials and the left/right Radau polynomials that define the DG
  correction functions of Huynh (cited in the same section as the source of FR).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def gauss_legendre(n: int):
    """n-point Gauss--Legendre rule on [-1, 1] (numpy's Golub--Welsch + Newton)."""
    x, w = npleg.leggauss(n)
    return x.astype(np.float64), w.astype(np.float64)


def legendre(n: int, x):
    """P_n(x)."""
    c = np.zeros(n + 1)
    c[n] = 1.0
    return npleg.legval(np.asarray(x, dtype=np.float64), c)


def legendre_deriv(n: int, x):
    """P_n'(x)."""
    c = np.zeros(n + 1)
    c[n] = 1.0
    return npleg.legval(np.asarray(x, dtype=np.float64), npleg.legder(c))


def lagrange_matrix(nodes, x):
    """L[i, j] = l_j(x_i) for the Lagrange basis on `nodes`, by the product formula."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = nodes.size
    L = np.ones((x.size, n))
    for j in range(n):
        for m in range(n):
            if m != j:
                L[:, j] *= (x - nodes[m]) / (nodes[j] - nodes[m])
    return L


def lagrange_deriv_matrix(nodes, x):
    """D[i, j] = l_j'(x_i), by differentiating the product formula term by term."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = nodes.size
    D = np.zeros((x.size, n))
    for j in range(n):
        denom = 1.0
        for m in range(n):
            if m != j:
                denom *= nodes[j] - nodes[m]
        for k in range(n):             # d/dx of prod_{m != j} (x - x_m): drop factor k
            if k == j:
                continue
            term = np.ones(x.size)
            for m in range(n):
                if m != j and m != k:
                    term *= x - nodes[m]
            D[:, j] += term
        D[:, j] /= denom
    return D


def radau_right_deriv(p: int, x):
    """g_R'(x) for g_R = (P_{p+1} + P_p)/2: g_R(1) = 1, g_R(-1) = 0 (DG correction)."""
    return 0.5 * (legendre_deriv(p + 1, x) + legendre_deriv(p, x))


def radau_left_deriv(p: int, x):
    """g_L'(x) for g_L = (-1)^{p+1} (P_{p+1} - P_p)/2: g_L(-1) = 1, g_L(1) = 0."""
    s = (-1.0) ** (p + 1)
    return 0.5 * s * (legendre_deriv(p + 1, x) - legendre_deriv(p, x))


def radau_right(p: int, x):
    return 0.5 * (legendre(p + 1, x) + legendre(p, x))


def radau_left(p: int, x):
    return 0.5 * (-1.0) ** (p + 1) * (legendre(p + 1, x) - legendre(p, x))
