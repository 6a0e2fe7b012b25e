"""Weak-form collocated nodal DG built by brute-force quadrature (a pin for the FR oracle).

On affine elements (parallelepiped hexahedra, tetrahedra) the FR scheme with the DG
correction function is known to reproduce the nodal discontinuous Galerkin method
(Huynh; Hesthaven & Warburton, both cited by the paper for the method).  This module
assembles that textbook method independently of the FR operators:

    J M du/dt = sum_i K_i f~_i - B F^C
    M_ij   = int l_i l_j,       K_i[z, n] = int (d l_z / d xt_i) l_n,
    B[z, s] = int_face l_z phi_s dS~   (phi_s: face Lagrange basis on the flux points)

with every integral done by a Gauss rule of higher degree than needed, f~ the
collocated transformed flux and F^C the same common flux as the FR oracle.
Euler only.
"""
from __future__ import annotations

import numpy as np

from . import fr, physics, polys, tet
from .elements import HEX


def _hex_matrices(ops, q):
    p = ops.order
    x1, _ = polys.gauss_legendre(p + 1)
    g, w = polys.gauss_legendre(q)
    n1 = p + 1
    I = np.arange(n1)
    k, j, i = [a.ravel() for a in np.meshgrid(I, I, I, indexing="ij")]
    Q = np.arange(q)
    qk, qj, qi = [a.ravel() for a in np.meshgrid(Q, Q, Q, indexing="ij")]
    L = polys.lagrange_matrix(x1, g)          # [q][n1]
    D = polys.lagrange_deriv_matrix(x1, g)
    W = w[qi] * w[qj] * w[qk]
    Lq = L[qi][:, i] * L[qj][:, j] * L[qk][:, k]
    dL = np.stack([D[qi][:, i] * L[qj][:, j] * L[qk][:, k],
                   L[qi][:, i] * D[qj][:, j] * L[qk][:, k],
                   L[qi][:, i] * L[qj][:, j] * D[qk][:, k]])
    M = Lq.T @ (W[:, None] * Lq)
    K = np.stack([dL[a].T @ (W[:, None] * Lq) for a in range(3)])
    B = np.zeros((ops.nsp, ops.nfp))
    for f in range(6):
        d, side = divmod(f, 2)
        t = [a for a in range(3) if a != d]
        cols = np.nonzero(ops.flux_face == f)[0]
        qa, qb = [a.ravel() for a in np.meshgrid(Q, Q, indexing="ij")]
        xq = np.zeros((q * q, 3))
        xq[:, d] = 1.0 if side else -1.0
        xq[:, t[0]] = g[qb]
        xq[:, t[1]] = g[qa]
        wq = w[qa] * w[qb]
        Lf = (polys.lagrange_matrix(x1, xq[:, 0])[:, i] * polys.lagrange_matrix(x1, xq[:, 1])[:, j]
              * polys.lagrange_matrix(x1, xq[:, 2])[:, k])
        # face Lagrange basis on the (p+1)^2 tensor flux points of this face
        phi = np.empty((q * q, len(cols)))
        for c, s in enumerate(cols):
            la = polys.lagrange_matrix(x1, xq[:, t[0]])[:, np.argmin(np.abs(x1 - ops.flux_pts[s, t[0]]))]
            lb = polys.lagrange_matrix(x1, xq[:, t[1]])[:, np.argmin(np.abs(x1 - ops.flux_pts[s, t[1]]))]
            phi[:, c] = la * lb
        B[:, cols] = Lf.T @ (wq[:, None] * phi)
    return M, K, B


def _tet_matrices(ops, q):
    p = ops.order
    qp, qw = tet.quad_tet(q)
    Lq = tet.lagrange(ops.sol_pts, qp, p)
    dL = np.moveaxis(tet.lagrange_grad(ops.sol_pts, qp, p), 2, 0)   # [3][q][nsp]
    M = Lq.T @ (qw[:, None] * Lq)
    K = np.stack([dL[a].T @ (qw[:, None] * Lq) for a in range(3)])
    B = np.zeros((ops.nsp, ops.nfp))
    tq, tw = tet.quad_tri(q)
    for f in range(4):
        X0, e1, e2, dA = tet.face_param(f)
        xq = X0 + tq[:, :1] * e1 + tq[:, 1:] * e2
        cols = np.nonzero(ops.flux_face == f)[0]
        fst = tet.face_coords(f, ops.flux_pts[cols])
        phi = tet.tri_monomials(tq, p) @ np.linalg.inv(tet.tri_monomials(fst, p))
        B[:, cols] = tet.lagrange(ops.sol_pts, xq, p).T @ ((tw * dA)[:, None] * phi)
    return M, K, B


def rhs(blocks, u_list, prm: fr.Params, q=None):
    """Nodal DG du/dt per block [n][5][nsp] (affine elements, Euler)."""
    uf = [fr._apply(b.ops.interp, u) for b, u in zip(blocks, u_list)]
    out = []
    for bi, (b, u) in enumerate(zip(blocks, u_list)):
        ops = b.ops
        qq = q or (ops.order + 3)
        M, K, B = _hex_matrices(ops, qq) if b.etype == HEX else _tet_matrices(ops, qq)
        Jc = b.J[:, 0]
        if np.abs(b.J - Jc[:, None]).max() > 1e-12 * np.abs(Jc).max():
            raise ValueError("nodal DG pin needs affine elements")
        ut = np.moveaxis(u, 1, 0)
        f = physics.euler_flux(ut, prm.gamma)
        ftil = np.einsum("esij,vjes->vies", b.S, f)                # [5][3][n][nsp]
        Fc = fr.common_flux(blocks, bi, uf, None, prm)             # [5][n][nfp]
        rhs_w = sum(ftil[:, a] @ K[a].T for a in range(3)) - Fc @ B.T
        du = np.linalg.solve(M, np.moveaxis(rhs_w, -1, 0).reshape(ops.nsp, -1))
        du = du.reshape((ops.nsp,) + rhs_w.shape[:-1])
        out.append(np.moveaxis(np.moveaxis(du, 0, -1) / Jc[None, :, None], 0, 1).copy())
    return out
