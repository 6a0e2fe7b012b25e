"""Dense element operator sets for the oracle (FP64, brute force, no sum factorisation).

For an element type with solution points x_zeta and flux points x_sigma
(Sec. "Flux Reconstruction"):

    interp[sigma, zeta]   = l_zeta(x_sigma)                  (step 1, eq:disu; step 3 trace)
    deriv[i, zeta, nu]    = d l_nu / d xt_i  at x_zeta       (step 4, eq:FRfinal volume term)
    lift[zeta, sigma]     = (div g_sigma)(x_zeta)            (step 4 correction term)
    normals[sigma]        = outward unit reference normal n~ at x_sigma
    weights[zeta]         = integral of l_zeta over the reference element

Correction functions (the paper names "a flux correction function" and cites
Huynh): the DG choice.  Hexahedra: tensor form of the 1-D Radau polynomials,
    face xi_d = +1: (div g_sigma)(x_abc) = g_R'(x_{a_d}) * delta(tangential indices)
    face xi_d = -1: (div g_sigma)(x_abc) = -g_L'(x_{a_d}) * delta(tangential indices)
Tetrahedra: the DG lifting M^{-1} E with M_ij = int l_i l_j and
E_{i sigma} = int_face l_i phi_sigma dS over the true reference face area.

Canonical solution-point order: hexahedra zeta = i + (p+1)(j + (p+1)k) with i along
xi_1 (Gauss--Legendre nodes increasing); tetrahedra the printed order of Fig. mesh(c).
Flux points of hexahedra: faces (xi1=-1, xi1=+1, xi2=-1, xi2=+1, xi3=-1, xi3=+1),
each a tensor Gauss--Legendre grid of the two tangential coordinates (lower axis
fastest).  Flux points of tetrahedra: faces in tet.FACES order, each listing the
solution points on that face.  Pyramids (p = 4, affine base): pyramid.py, the same
fields with the DG lifting of the rational pyramid space.
"""
from __future__ import annotations

from dataclasses import dataclass
from functools import lru_cache

import numpy as np

from . import polys, tet

HEX = 0
TET = 1
PYR = 2


@dataclass
class ElementOps:
    etype: int
    order: int
    sol_pts: np.ndarray     # [nsp][3]
    flux_pts: np.ndarray    # [nfp][3]
    flux_face: np.ndarray   # [nfp] face id
    normals: np.ndarray     # [nfp][3]
    interp: np.ndarray      # [nfp][nsp]
    deriv: np.ndarray       # [3][nsp][nsp]
    lift: np.ndarray        # [nsp][nfp]
    weights: np.ndarray     # [nsp]
    n_faces: int
    face_nfp: int
    modal_V: np.ndarray     # [nsp][nmodes] orthonormal modes at solution points
    modal_deg: np.ndarray   # hex: [nmodes][3] per-axis degrees; tet, pyramid: [nmodes] degree

    @property
    def nsp(self):
        return self.sol_pts.shape[0]

    @property
    def nfp(self):
        return self.flux_pts.shape[0]

    # ---------------- shape functions of the geometric map --------------------
    def shape(self, xi):
        return shape_funcs(self.etype, xi)

    def shape_grad(self, xi):
        return shape_grads(self.etype, xi)


def shape_funcs(etype, xi):
    xi = np.atleast_2d(xi)
    if etype == HEX:
        c = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                      [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], dtype=np.float64)
        return np.prod(1.0 + xi[:, None, :] * c[None, :, :], axis=2) / 8.0
    x, y, z = xi[:, 0], xi[:, 1], xi[:, 2]
    if etype == PYR:
        # affine map of a pyramid with a parallelogram base (corner 2 = 1 + 3 - 0):
        # u, v, w = (x+1)/2, (y+1)/2, (z+1)/2 and x = X0 + u e1 + v e3 + w (X4 - centre of base)
        u, v, w = (1 + x) / 2, (1 + y) / 2, (1 + z) / 2
        return np.stack([1 - u - v, u - w / 2, np.zeros_like(u), v - w / 2, w], axis=1)
    return np.stack([-(1 + x + y + z) / 2, (1 + x) / 2, (1 + z) / 2, (1 + y) / 2], axis=1)


def shape_grads(etype, xi):
    """[n_pts][n_corner][3] reference gradients of the shape functions."""
    xi = np.atleast_2d(xi)
    if etype == HEX:
        c = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                      [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], dtype=np.float64)
        f = 1.0 + xi[:, None, :] * c[None, :, :]          # [n][8][3]
        g = np.empty_like(f)
        g[..., 0] = c[None, :, 0] * f[..., 1] * f[..., 2] / 8
        g[..., 1] = c[None, :, 1] * f[..., 0] * f[..., 2] / 8
        g[..., 2] = c[None, :, 2] * f[..., 0] * f[..., 1] / 8
        return g
    if etype == PYR:
        g = np.array([[-0.5, -0.5, 0], [0.5, 0, -0.25], [0, 0, 0], [0, 0.5, -0.25], [0, 0, 0.5]])
        return np.broadcast_to(g, (xi.shape[0], 5, 3)).copy()
    g = np.array([[-0.5, -0.5, -0.5], [0.5, 0, 0], [0, 0, 0.5], [0, 0.5, 0]])
    return np.broadcast_to(g, (xi.shape[0], 4, 3)).copy()


@lru_cache(maxsize=None)
def hex_ops(p: int) -> ElementOps:
    x1, w1 = polys.gauss_legendre(p + 1)
    n1 = p + 1
    # solution points, zeta = i + n1*(j + n1*k)
    I = np.arange(n1)
    k, j, i = np.meshgrid(I, I, I, indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    sol = np.stack([x1[i], x1[j], x1[k]], axis=1)
    nsp = sol.shape[0]
    # flux points
    fpts, fface, fnorm = [], [], []
    for d in range(3):
        t = [a for a in range(3) if a != d]
        for s, sgn in ((0, -1.0), (1, 1.0)):
            for b in range(n1):
                for a in range(n1):
                    pt = np.zeros(3)
                    pt[d] = sgn
                    pt[t[0]] = x1[a]
                    pt[t[1]] = x1[b]
                    fpts.append(pt)
                    fface.append(2 * d + s)
                    nv = np.zeros(3)
                    nv[d] = sgn
                    fnorm.append(nv)
    fpts, fface, fnorm = np.array(fpts), np.array(fface), np.array(fnorm)
    nfp = fpts.shape[0]
    # dense 3-D Lagrange operators as Kronecker products of 1-D ones
    def lag3(x):
        Lx = polys.lagrange_matrix(x1, x[:, 0])
        Ly = polys.lagrange_matrix(x1, x[:, 1])
        Lz = polys.lagrange_matrix(x1, x[:, 2])
        return Lx[:, i] * Ly[:, j] * Lz[:, k]
    interp = lag3(fpts)
    D1 = polys.lagrange_deriv_matrix(x1, x1)
    L1 = polys.lagrange_matrix(x1, x1)
    Dx = np.kron(np.kron(L1, L1), D1)   # acts on zeta = i + n1*(j + n1*k): i is fastest
    Dy = np.kron(np.kron(L1, D1), L1)
    Dz = np.kron(np.kron(D1, L1), L1)
    deriv = np.stack([Dx, Dy, Dz])
    # DG correction: Radau derivatives
    gR = polys.radau_right_deriv(p, x1)
    gL = polys.radau_left_deriv(p, x1)
    lift = np.zeros((nsp, nfp))
    idx = np.stack([i, j, k], axis=1)
    for s_ in range(nfp):
        f = fface[s_]
        d, side = divmod(f, 2)
        t = [a for a in range(3) if a != d]
        ta = np.argmin(np.abs(x1 - fpts[s_, t[0]]))
        tb = np.argmin(np.abs(x1 - fpts[s_, t[1]]))
        mask = (idx[:, t[0]] == ta) & (idx[:, t[1]] == tb)
        lift[mask, s_] = gR[idx[mask, d]] if side == 1 else -gL[idx[mask, d]]
    weights = w1[i] * w1[j] * w1[k]
    # orthonormal tensor Legendre modes
    Pn = np.stack([polys.legendre(m, x1) * np.sqrt((2 * m + 1) / 2.0) for m in range(n1)], axis=1)
    modal_V = Pn[i][:, i] * Pn[j][:, j] * Pn[k][:, k]
    modal_deg = np.stack([i, j, k], axis=1)
    return ElementOps(HEX, p, sol, fpts, fface, fnorm, interp, deriv, lift, weights,
                      6, n1 * n1, modal_V, modal_deg)


@lru_cache(maxsize=None)
def tet_ops(p: int = 4) -> ElementOps:
    """Tet operators from the same definitions, assembled in extended precision
    (mpmath, tet.MP_DPS digits) and rounded to FP64 once."""
    import mpmath
    if p != 4:
        raise ValueError("tetrahedra are supported at p = 4 only (the paper's printed point set)")
    mpmath.mp.dps = tet.MP_DPS
    sol = tet.SOL_PTS_P4.copy()
    nsp = sol.shape[0]
    fpts, fface, fnorm = [], [], []
    for f in range(4):
        ids = tet.face_point_ids(f)
        st = tet.face_coords(f, sol[ids])
        order = np.lexsort((st[:, 0], st[:, 1]))
        for q in ids[order]:
            fpts.append(sol[q])
            fface.append(f)
            fnorm.append(tet.FACES[f][1])
    fpts, fface, fnorm = np.array(fpts), np.array(fface), np.array(fnorm)
    nfp = fpts.shape[0]
    # Lagrange coefficients: l_j = sum_m C[m, j] mono_m
    V = mpmath.matrix([tet.mp_mono_row(x, p) for x in sol])
    C = V ** -1
    to_np = lambda A: np.array([[float(A[i, j]) for j in range(A.cols)] for i in range(A.rows)])

    def lag(xs):
        return mpmath.matrix([tet.mp_mono_row(x, p) for x in xs]) * C

    interp = to_np(lag(fpts))
    deriv = np.stack([to_np(mpmath.matrix([tet.mp_mono_row(x, p, deriv=d) for x in sol]) * C) for d in range(3)])
    # mass matrix, weights and face matrices by extended-precision quadrature
    qp, qw = tet.mp_quad_tet(p + 3)
    Lq = lag(qp)
    M = mpmath.matrix(nsp, nsp)
    wts = mpmath.matrix(nsp, 1)
    for q in range(len(qw)):
        for a in range(nsp):
            la = Lq[q, a] * qw[q]
            wts[a] += la
            for b in range(nsp):
                M[a, b] += la * Lq[q, b]
    E = mpmath.matrix(nsp, nfp)
    tq, tw = tet.mp_quad_tri(p + 3)
    for f in range(4):
        i0, i1, i2 = tet.FACES[f][0]
        X0, X1, X2 = [[mpmath.mpf(float(v)) for v in tet.CORNERS[i]] for i in (i0, i1, i2)]
        e1 = [X1[k] - X0[k] for k in range(3)]
        e2 = [X2[k] - X0[k] for k in range(3)]
        cr = [e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]]
        dA = mpmath.sqrt(cr[0] ** 2 + cr[1] ** 2 + cr[2] ** 2)
        cols = np.nonzero(fface == f)[0]
        fst = tet.face_coords(f, fpts[cols])
        tri = lambda st: [st[0] ** a * st[1] ** (d - a) for d in range(p + 1) for a in range(d + 1)]
        Cf = mpmath.matrix([tri([mpmath.mpf(float(v)) for v in s_]) for s_ in fst]) ** -1
        xq = [[X0[k] + s_[0] * e1[k] + s_[1] * e2[k] for k in range(3)] for s_ in tq]
        Lf = lag(xq)
        phi = mpmath.matrix([tri(s_) for s_ in tq]) * Cf
        for q in range(len(tw)):
            wq = tw[q] * dA
            for a in range(nsp):
                la = Lf[q, a] * wq
                if la == 0:
                    continue
                for c_, s_ in enumerate(cols):
                    E[a, int(s_)] += la * phi[q, c_]
    lift = to_np(M ** -1 * E)
    weights = np.array([float(wts[a]) for a in range(nsp)])
    modal_V = tet.ortho_basis(sol, p)
    modal_deg = tet.ortho_degrees(p)
    return ElementOps(TET, p, sol, fpts, fface, fnorm, interp, deriv, lift, weights,
                      4, 15, modal_V, modal_deg)


def ops_for(etype: int, p: int) -> ElementOps:
    if etype == PYR:
        from .pyramid import pyr_ops
        return pyr_ops(p)
    return hex_ops(p) if etype == HEX else tet_ops(p)
