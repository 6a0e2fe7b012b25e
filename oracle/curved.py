"""Curved hexahedra and tetrahedra: the high-order geometric map and its metric terms
(oracle, FP64).

TEST INFRASTRUCTURE: only tests/, the smoke check and the benchmark's CPU leg use it.

The paper (Sec. "Curved elements") keeps a 3x3 matrix of metric terms per point of a
curved element and contrasts two ways of forming it:

  cross-product metric   S = J G^{-1} from the exact Jacobian G = dx/dxi at each
                         point (row i = g_j x g_k, i, j, k cyclic, g_j = dx/dxi_j);
                         its entries are polynomials of about twice the degree of the
                         map, which the solution polynomials cannot represent, so the
                         discrete divergence of the metric is not zero and a uniform
                         free stream is not preserved;
  conservative metric    the metric written as a curl (Kopriva 2006; Abe et al.
                         2015), which stays divergence-free whatever approximation
                         the curled function carries, so a uniform stream is kept.

Reading used for the conservative metric (the paper gives the idea, not the
discretisation): with (n, m, l) cyclic,
    S_in = J dxi_i/dx_n = -[curl_xi V^(n)]_i,   V^(n) = I_p( x_l grad_xi x_m ),
I_p the tensor interpolant of the solution order p on the (p+1)^3
Gauss--Lobatto--Legendre points.  Without I_p this is the cross-product metric
(curl(x_l grad x_m) = grad x_l x grad x_m).  With it each row is the curl of a
polynomial in Q_p: it lies in Q_p (so the solution points represent it exactly) and
has zero divergence; on a face xi_d = +-1 row d involves only tangential derivatives
of the interpolant's face values, and the Lobatto points include the face, so two
elements sharing a face agree on its normal.  J is det G of the exact map.
The factor x_l is taken relative to the element's node 0: for q <= p the
interpolant of grad x_m is exact and has zero curl, so the shift changes nothing in
exact arithmetic, while in floating point it keeps coordinates of size |x| out of a
result of size h^2 (without it two FP64 evaluations differ by ~|x| / h ulps).

Geometry of order q: x(xi) = sum_n N_n(xi) X_n, N the tensor Lagrange polynomials on
equispaced nodes, node n = i + (q+1)(j + (q+1)k) at (-1 + 2i/q, -1 + 2j/q, -1 + 2k/q).

Tetrahedra (solution order 4, the point set of Fig. mesh): the map is the Lagrange
interpolant of total degree q on the equispaced nodes (i, j, k), i + j + k <= q (k
outermost, then j, then i) at (-1 + 2i/q, -1 + 2j/q, -1 + 2k/q).  The conservative
metric takes the same curl form with I_p the interpolant of total degree 4 on the 35
solution points.  They include 15 points on every face, which fix a degree-4
polynomial on that face, so the tangential part of I_p V on a face -- all that the
face's normal row n~^T S depends on -- is the face interpolant of values the two
elements sharing the face have in common; their unit normals agree (the lengths
|S^T n~| differ by the ratio of the two reference faces' areas, as for straight
tetrahedra).  The cross-product metric has degree 2(q - 1) here too, beyond 4 for
q = 4.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg

from . import polys
from . import tet as otet


def gll_nodes(n: int):
    """n Gauss--Lobatto--Legendre nodes on [-1, 1]: the end points and the roots of P_{n-1}'."""
    c = np.zeros(n)
    c[n - 1] = 1.0
    inner = np.sort(npleg.legroots(npleg.legder(c))) if n > 2 else np.zeros(0)
    return np.concatenate([[-1.0], inner, [1.0]])


def _tensor_index(n1):
    I = np.arange(n1)
    k, j, i = np.meshgrid(I, I, I, indexing="ij")
    return i.ravel(), j.ravel(), k.ravel()


def _tensor_ops(nodes, xi):
    """Values [np][m] and gradients [3][np][m] of the tensor Lagrange basis on nodes^3 at xi."""
    xi = np.atleast_2d(xi)
    i, j, k = _tensor_index(len(nodes))
    L = [polys.lagrange_matrix(nodes, xi[:, a]) for a in range(3)]
    D = [polys.lagrange_deriv_matrix(nodes, xi[:, a]) for a in range(3)]
    val = L[0][:, i] * L[1][:, j] * L[2][:, k]
    grad = np.stack([D[0][:, i] * L[1][:, j] * L[2][:, k],
                     L[0][:, i] * D[1][:, j] * L[2][:, k],
                     L[0][:, i] * L[1][:, j] * D[2][:, k]])
    return val, grad


def geo_nodes(q: int):
    return np.linspace(-1.0, 1.0, q + 1)


def map_points(q: int, X, xi):
    """Physical points [n][np][3] of elements with nodes X [n][(q+1)^3][3]."""
    N, _ = _tensor_ops(geo_nodes(q), xi)
    return np.einsum("pc,ecd->epd", N, X)


def jacobian(q: int, X, xi):
    """G [n][np][3][3], G[..., i, j] = d x_i / d xi_j."""
    _, dN = _tensor_ops(geo_nodes(q), xi)
    return np.einsum("jpc,eci->epij", dN, X)


def cross_metric(q: int, X, xi):
    """(J, S) with S = J G^{-1} from the exact Jacobian."""
    G = jacobian(q, X, xi)
    J = np.linalg.det(G)
    return J, J[..., None, None] * np.linalg.inv(G)


def conservative_metric(q: int, p: int, X, xi):
    """(J, S) with S_in = -[curl V^(n)]_i, V^(n) = I_p(x_l grad x_m), (n, m, l) cyclic."""
    y = gll_nodes(p + 1)
    i, j, k = _tensor_index(p + 1)
    Y = np.stack([y[i], y[j], y[k]], axis=1)
    xY = map_points(q, X - X[:, :1, :], Y)            # [n][m][3], relative to node 0
    GY = jacobian(q, X, Y)                            # [n][m][3][3]
    _, dL = _tensor_ops(y, xi)                        # [3][np][m]: d/dxi_a of the GLL basis
    S = np.empty(X.shape[:1] + (np.atleast_2d(xi).shape[0], 3, 3))
    for n in range(3):
        m, l = (n + 1) % 3, (n + 2) % 3
        V = xY[..., l, None] * GY[..., m, :]          # V[e][node][a] = (x_l - x0_l) d x_m / d xi_a
        for r in range(3):
            a, b = (r + 1) % 3, (r + 2) % 3
            # [curl V]_r = d_a V_b - d_b V_a
            curl = np.einsum("pm,em->ep", dL[a], V[..., b]) - np.einsum("pm,em->ep", dL[b], V[..., a])
            S[:, :, r, n] = -curl
    J = np.linalg.det(jacobian(q, X, xi))
    return J, S


def metric(kind: str, q: int, p: int, X, xi):
    if kind == "conservative":
        return conservative_metric(q, p, X, xi)
    if kind == "cross":
        return cross_metric(q, X, xi)
    raise ValueError(kind)


# ------------------------------------------------------------------- tetrahedra

def tet_geo_nodes(q: int):
    """Reference points [(q+1)(q+2)(q+3)/6][3] of the order-q tetrahedron's nodes."""
    lat = [(i, j, k) for k in range(q + 1) for j in range(q + 1 - k) for i in range(q + 1 - k - j)]
    return -1.0 + 2.0 * np.array(lat, dtype=np.float64) / q


def tet_map_points(q: int, X, xi):
    """Physical points [n][np][3] of tetrahedra with nodes X [n][nn][3]."""
    N = otet.lagrange(tet_geo_nodes(q), np.atleast_2d(xi), q)        # [np][nn]
    return np.einsum("pc,ecd->epd", N, X)


def tet_jacobian(q: int, X, xi):
    """G [n][np][3][3], G[..., i, j] = d x_i / d xi_j."""
    dN = otet.lagrange_grad(tet_geo_nodes(q), np.atleast_2d(xi), q)  # [np][nn][3]
    return np.einsum("pcj,eci->epij", dN, X)


def tet_cross_metric(q: int, X, xi):
    G = tet_jacobian(q, X, xi)
    J = np.linalg.det(G)
    return J, J[..., None, None] * np.linalg.inv(G)


def tet_conservative_metric(q: int, X, xi):
    """(J, S) with S_in = -[curl V^(n)]_i, V^(n) = I_4(x_l grad x_m) on the 35 solution points."""
    Y = otet.SOL_PTS_P4
    xY = tet_map_points(q, X - X[:, :1, :], Y)                      # relative to node 0
    GY = tet_jacobian(q, X, Y)
    dL = np.moveaxis(otet.lagrange_grad(Y, np.atleast_2d(xi), 4), 2, 0)   # [3][np][35]
    S = np.empty(X.shape[:1] + (np.atleast_2d(xi).shape[0], 3, 3))
    for n in range(3):
        m, l = (n + 1) % 3, (n + 2) % 3
        V = xY[..., l, None] * GY[..., m, :]
        for r in range(3):
            a, b = (r + 1) % 3, (r + 2) % 3
            curl = np.einsum("pm,em->ep", dL[a], V[..., b]) - np.einsum("pm,em->ep", dL[b], V[..., a])
            S[:, :, r, n] = -curl
    J = np.linalg.det(tet_jacobian(q, X, xi))
    return J, S


def tet_metric(kind: str, q: int, X, xi):
    if kind == "conservative":
        return tet_conservative_metric(q, X, xi)
    if kind == "cross":
        return tet_cross_metric(q, X, xi)
    raise ValueError(kind)
