"""Geometric map, Jacobians and transformed metric (Sec. "Flux Reconstruction", mapping).

For element corners X (shape [n][n_corner][3]) and reference points xi:
    x(xi)   = sum_n N_n(xi) X_n                      (x = M_n(xi~))
    G_ij    = d x_i / d xi_j                         (J_nij)
    J       = det G                                  (J_n)
    S       = J G^{-1},  S_ij = J d xi_i / d x_j      (so f~_i = sum_j S_ij f_j; the transformed
                                                       flux J J^{-1} f of the transformed equation)
At a flux point with unit reference normal n~ the physical, area-scaled normal is
S^T n~ (its length is the surface-measure ratio, its direction the unit normal n^).
The paper writes the inverse Jacobian as a derivative with respect to the reference
coordinates; it is read as d xi_i / d x_j with det = 1/J, as the text beside it says.
"""
from __future__ import annotations

import numpy as np

from .elements import shape_funcs, shape_grads


def map_points(etype, X, xi):
    N = shape_funcs(etype, xi)                    # [np][nc]
    return np.einsum("pc,ecd->epd", N, X)


def jacobian(etype, X, xi):
    """G [n][np][3][3] with G[..., i, j] = d x_i / d xi_j."""
    dN = shape_grads(etype, xi)                   # [np][nc][3]
    return np.einsum("pcj,eci->epij", dN, X)


def metric(etype, X, xi):
    """(J [n][np], S [n][np][3][3]) at reference points xi."""
    G = jacobian(etype, X, xi)
    J = np.linalg.det(G)
    S = J[..., None, None] * np.linalg.inv(G)
    return J, S


def scaled_normals(etype, X, xi, nref):
    """S^T n~ at flux points: [n][nfp][3]."""
    _, S = metric(etype, X, xi)
    return np.einsum("epij,pi->epj", S, nref)
