"""Weak-form collocated nodal DG built by brute-force quadrature (a pin for the FR oracle).

On affine elements (parallelepiped hexahedra, tetrahedra) the FR scheme with the DG
correction function is known to reproduce the nodal discontinuous Galerkin method
(Huynh; Hesthaven & Warburton, both cited by the paper for the method).  This module
assembles that textbook method independently of the FR operators:

    J M du/dt = sum_i K_i f~_i - B F^C
    M_ij   = int l_i l_j,       K_i[z, n] = int (d l_z / d xt_i) l_n,
    B[z, s] = int_face l_z phi_s dS~   (phi_s: face Lagrange basis on the flux points)

with every integral done by a Gauss rule of higher degree than needed and f~ the
collocated transformed flux.

Navier--Stokes (LDG, the viscous reading): the gradient is the weak-form DG
gradient of the same textbook method,

    M q~_i = -K_i u + B (n~_i u^),      grad u = G^{-T} q~   (affine: constant G),

with the common solution u^ = (1/2 + beta) u_L + (1/2 - beta) u_R taken from the
face's left (L) and right (R) traces; the flux is f = f_inv(u) - f_v(u, grad u)
collocated at the solution points, and the common normal flux along the left
side's unit normal n^_L is

    𝔉 = 𝔉_inv(u_L, u_R, n^_L) - [(1/2 - beta) f_v(L) + (1/2 + beta) f_v(R)] . n^_L
        + tau (u_L - u_R),

with the gradient traces interpolated from the solution points.  The left element
receives +|S^T n~| 𝔉 and the right one -|S^T n~| 𝔉 (n dS = S^T n~ dS~).  None of
these common values is taken from the FR oracle: only the connectivity (paired
flux points, left/right sides), the metric terms, the pointwise physics and the
Lagrange interpolation to flux points are shared, each pinned on its own.
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


def _paired(blocks, vals, b):
    """Values [C][n][nfp] of the neighbour's paired flux points (vals[t]: [n_t][C][nfp_t])."""
    C = vals[0].shape[1]
    out = np.empty((C,) + b.nbr_elem.shape)
    for t in range(len(blocks)):
        m = b.nbr_type == t
        if np.any(m):
            out[:, m] = vals[t][b.nbr_elem[m], :, b.nbr_fp[m]].T
    return out


def _sides(b, own, nbr):
    """(left trace, right trace) [C][n][nfp] from own [n][C][nfp] and neighbour [C][n][nfp]."""
    own = np.moveaxis(own, 1, 0)
    return np.where(b.is_left[None], own, nbr), np.where(b.is_left[None], nbr, own)


def _affine(b):
    Jc = b.J[:, 0]
    if np.abs(b.J - Jc[:, None]).max() > 1e-12 * np.abs(Jc).max():
        raise ValueError("nodal DG pin needs affine elements")
    return Jc


def _matrices(b, q):
    qq = q or (b.ops.order + 3)
    return _hex_matrices(b.ops, qq) if b.etype == HEX else _tet_matrices(b.ops, qq)


def gradients(blocks, u_list, prm: fr.Params, q=None):
    """Weak-form LDG gradients grad u [n][5][3][nsp] per block (affine elements)."""
    uf = [fr._apply(b.ops.interp, u) for b, u in zip(blocks, u_list)]
    out = []
    for bi, (b, u) in enumerate(zip(blocks, u_list)):
        M, K, B = _matrices(b, q)
        Jc = _affine(b)
        uL, uR = _sides(b, uf[bi], _paired(blocks, uf, b))
        uhat = (0.5 + prm.ldg_beta) * uL + (0.5 - prm.ldg_beta) * uR          # [5][n][nfp]
        qt = np.empty(u.shape[:2] + (3, u.shape[2]))
        for i in range(3):
            w = -(u @ K[i].T) + np.moveaxis(uhat * b.ops.normals[:, i], 0, 1) @ B.T     # [n][5][nsp]
            qt[:, :, i] = np.moveaxis(np.linalg.solve(M, np.moveaxis(w, -1, 0).reshape(M.shape[0], -1))
                                      .reshape((M.shape[0],) + w.shape[:-1]), 0, -1)
        Gi = b.S[:, 0] / Jc[:, None, None]                                      # G^{-1} = S / J
        out.append(np.einsum("eij,evis->evjs", Gi, qt))
    return out


def rhs(blocks, u_list, prm: fr.Params, q=None):
    """Nodal DG du/dt per block [n][5][nsp] (affine elements; Euler or Navier--Stokes)."""
    gam = prm.gamma
    ns = prm.system == fr.NAVIER_STOKES
    uf = [fr._apply(b.ops.interp, u) for b, u in zip(blocks, u_list)]
    if ns:
        g = gradients(blocks, u_list, prm, q)
        gf = [fr._apply(b.ops.interp, gg).reshape(len(b.elems), 15, -1) for b, gg in zip(blocks, g)]
    out = []
    for bi, (b, u) in enumerate(zip(blocks, u_list)):
        ops = b.ops
        M, K, B = _matrices(b, q)
        Jc = _affine(b)
        ut = np.moveaxis(u, 1, 0)
        f = physics.euler_flux(ut, gam)
        if ns:
            f = f - physics.viscous_flux(ut, np.moveaxis(g[bi], (1, 2), (0, 1)), gam, prm.mu, prm.prandtl)
        ftil = np.einsum("esij,vjes->vies", b.S, f)                # [5][3][n][nsp]
        # common normal flux along the left side's unit normal
        uL, uR = _sides(b, uf[bi], _paired(blocks, uf, b))
        mag = np.linalg.norm(b.snorm, axis=2)
        sgn = np.where(b.is_left, 1.0, -1.0)
        nL = np.moveaxis(b.snorm / mag[..., None], 2, 0) * sgn
        F = physics.riemann(prm.riemann, uL, uR, nL, gam)
        if ns:
            gL, gR = _sides(b, gf[bi], _paired(blocks, gf, b))
            fvL = physics.viscous_flux(uL, gL.reshape((5, 3) + gL.shape[1:]), gam, prm.mu, prm.prandtl)
            fvR = physics.viscous_flux(uR, gR.reshape((5, 3) + gR.shape[1:]), gam, prm.mu, prm.prandtl)
            fv = (0.5 - prm.ldg_beta) * fvL + (0.5 + prm.ldg_beta) * fvR
            F = F - (fv[:, 0] * nL[0] + fv[:, 1] * nL[1] + fv[:, 2] * nL[2]) + prm.ldg_tau * (uL - uR)
        Fc = mag * sgn * F                                         # [5][n][nfp]
        rhs_w = sum(ftil[:, a] @ K[a].T for a in range(3)) - Fc @ B.T
        du = np.linalg.solve(M, np.moveaxis(rhs_w, -1, 0).reshape(ops.nsp, -1))
        du = du.reshape((ops.nsp,) + rhs_w.shape[:-1])
        out.append(np.moveaxis(np.moveaxis(du, 0, -1) / Jc[None, :, None], 0, 1).copy())
    return out
