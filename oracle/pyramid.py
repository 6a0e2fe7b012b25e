"""Reference pyramid at p = 4, for the oracle (FP64): the element the paper names for the
transition layer between tetrahedra and hexahedra (Sec. "Mixed elements and domain
decomposition"), supported there only with an affine (parallelogram) base.

TEST INFRASTRUCTURE: only tests/ use it.  Pinned against closed forms, independent
quadrature and convergence (tests/test_oracle_pyramid.py); the GPU path's pyramids are
checked against it.

Reference pyramid: base square [-1, 1]^2 at z = -1, apex (0, 0, 1); corners
(-1,-1,-1) (1,-1,-1) (1,1,-1) (-1,1,-1) (0,0,1).  Faces: 0 the base (corners 0 1 2 3,
outward normal -e_z), then the triangles 1 (0 1 4), 2 (1 2 4), 3 (2 3 4), 4 (3 0 4).

Readings (the paper names the element, not its discretisation):

* Approximation space: the rational pyramid space of dimension (p+1)(p+2)(2p+3)/6 = 55
  spanned, with s = (1 - z)/2, a = x/s, b = y/s and m = max(i, j), by
      psi_ijk = P_i(a) P_j(b) s^m P_k^(2m+2, 0)(z),   0 <= i, j <= p, 0 <= k <= p - m
  (Legendre P_i, Jacobi P_k^(alpha, 0)).  It contains every polynomial of total degree
  <= p, its trace on the base is Q_p and on each triangle P_p, so a face shared with a
  hexahedron or a tetrahedron of order p carries the same space.  At the apex every
  function with m >= 1 vanishes (s^m -> 0 with a, b bounded), which gives the values
  there; derivatives are only taken at interior points.
* Solution points: p + 1 layers at the Gauss--Legendre nodes z_0 < ... < z_p, layer k a
  tensor Gauss--Legendre grid of p + 1 - k points per direction in (a, b), i.e.
  (x, y) = s_k (a_i, b_j): 25 + 16 + 9 + 4 + 1 = 55 interior points.
* Flux points: on the base the (p+1)^2 tensor Gauss--Legendre points (those of a
  hexahedron's face of order p); on each triangle the 15 surface points of a face of the
  p = 4 tetrahedron (Fig. mesh(b), a set invariant under the triangle's symmetries), in
  the triangle's barycentric coordinates.  Within a face: base lower axis fastest, a
  triangle (corners c0 c1 c2) in increasing (t, s) of x = c0 + s (c1 - c0) + t (c2 - c0).
* Correction: the DG lifting M^{-1} E as for tetrahedra (M_ij = int l_i l_j over the
  pyramid, E_i,sigma = int_face l_i phi_sigma dS over the true face area, phi the face's
  Lagrange basis: tensor on the base, total degree p on a triangle), with collapsed
  Gauss quadrature exact for these rational integrands.
* Divergence: collocated, d l_nu / d xi_i at the solution points, as for the other
  types.  The derivative of a rational member can leave the space, so the quadrature
  of the weights no longer integrates it exactly and the scheme conserves only up to
  that defect (zero for fluxes of degree <= p; it converges faster than the scheme's
  truncation error under refinement).

Lebesgue constant of the layered set: about 15 over the element, 20.5 at the triangle
flux points (the tetrahedron's set reaches its face points with weight 1), so large
random point-wise states overshoot there; smooth states are unaffected.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np
from numpy.polynomial import legendre as npleg
from scipy.special import eval_jacobi

from . import polys, tet

P = 4
CORNERS = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1], [0, 0, 1]], dtype=np.float64)
FACES = [(0, 1, 2, 3), (0, 1, 4), (1, 2, 4), (2, 3, 4), (3, 0, 4)]


def face_normal(f):
    """Outward unit reference normal of face f."""
    c = CORNERS[list(FACES[f])]
    n = np.cross(c[1] - c[0], c[2] - c[0])
    n /= np.linalg.norm(n)
    if n @ (c[0] - CORNERS.mean(axis=0)) < 0:
        n = -n
    return n


def face_area(f):
    c = CORNERS[list(FACES[f])]
    if len(c) == 4:
        return float(np.linalg.norm(np.cross(c[1] - c[0], c[3] - c[0])))
    return 0.5 * float(np.linalg.norm(np.cross(c[1] - c[0], c[2] - c[0])))


def modes(p=P):
    return [(i, j, k) for i in range(p + 1) for j in range(p + 1) for k in range(p + 1 - max(i, j))]


def _collapsed(pts):
    x, y, z = pts[:, 0], pts[:, 1], pts[:, 2]
    s = (1.0 - z) / 2.0
    apex = s <= 1e-14
    ss = np.where(apex, 1.0, s)
    return np.where(apex, 0.0, x / ss), np.where(apex, 0.0, y / ss), z, s, apex


def _leg(n, x, der=False):
    c = np.zeros(n + 1)
    c[n] = 1.0
    return npleg.legval(x, npleg.legder(c) if der else c)


def basis(pts, p=P):
    """[n_pts][n_modes] values of psi_ijk (apex values by continuity)."""
    a, b, z, s, apex = _collapsed(np.atleast_2d(pts))
    out = []
    for i, j, k in modes(p):
        m = max(i, j)
        v = _leg(i, a) * _leg(j, b) * s ** m * eval_jacobi(k, 2 * m + 2, 0, z)
        out.append(np.where(apex & (m > 0), 0.0, v))
    return np.stack(out, axis=1)


def basis_grad(pts, p=P):
    """[n_pts][n_modes][3] gradients d/dx, d/dy, d/dz of psi_ijk at interior points."""
    a, b, z, s, apex = _collapsed(np.atleast_2d(pts))
    if np.any(apex):
        raise ValueError("derivatives of the rational space are not defined at the apex")
    out = np.empty((a.shape[0], len(modes(p)), 3))
    for n_, (i, j, k) in enumerate(modes(p)):
        m = max(i, j)
        A, dA = _leg(i, a), _leg(i, a, True)
        B, dB = _leg(j, b), _leg(j, b, True)
        S = s ** m
        dS = -0.5 * m * s ** (m - 1) if m > 0 else np.zeros_like(s)
        C = eval_jacobi(k, 2 * m + 2, 0, z)
        dC = 0.5 * (k + 2 * m + 3) * eval_jacobi(k - 1, 2 * m + 3, 1, z) if k > 0 else np.zeros_like(z)
        out[:, n_, 0] = dA * B * S * C / s
        out[:, n_, 1] = A * dB * S * C / s
        # a = x/s and b = y/s change with z at fixed (x, y): da/dz = a / (2 s)
        out[:, n_, 2] = (dA * B * a + A * dB * b) / (2 * s) * S * C + A * B * dS * C + A * B * S * dC
    return out


def sol_points(p=P):
    zg, _ = polys.gauss_legendre(p + 1)
    pts = []
    for k in range(p + 1):
        n = p + 1 - k
        g, _ = polys.gauss_legendre(n)
        s = (1.0 - zg[k]) / 2.0
        for j in range(n):
            for i in range(n):
                pts.append([s * g[i], s * g[j], zg[k]])
    return np.array(pts)


def _tri_face_points():
    """The 15 surface points of a face of the p = 4 tetrahedron as barycentric (s, t)."""
    ids = tet.face_point_ids(0)
    return tet.face_coords(0, tet.SOL_PTS_P4[ids])


def flux_points(p=P):
    """(points [nfp][3], face id [nfp]) in face order."""
    g, _ = polys.gauss_legendre(p + 1)
    pts, face = [], []
    for j in range(p + 1):
        for i in range(p + 1):
            pts.append([g[i], g[j], -1.0])
            face.append(0)
    st = _tri_face_points()
    order = np.lexsort((st[:, 0], st[:, 1]))
    for f in range(1, 5):
        c0, c1, c2 = CORNERS[list(FACES[f])]
        for q in order:
            pts.append(c0 + st[q, 0] * (c1 - c0) + st[q, 1] * (c2 - c0))
            face.append(f)
    return np.array(pts), np.array(face)


def quad_pyr(n=8):
    """Collapsed Gauss rule on the reference pyramid: x = s a, y = s b, dV = s^2 da db dz."""
    g, w = polys.gauss_legendre(n)
    A, B, Z = np.meshgrid(g, g, g, indexing="ij")
    WA, WB, WZ = np.meshgrid(w, w, w, indexing="ij")
    s = (1.0 - Z) / 2.0
    pts = np.stack([s * A, s * B, Z], axis=-1).reshape(-1, 3)
    return pts, (WA * WB * WZ * s * s).ravel()


@lru_cache(maxsize=None)
def pyr_ops(p=P):
    """Operator set of the p = 4 pyramid (same fields as the hex and tet sets)."""
    from .elements import PYR, ElementOps
    if p != P:
        raise ValueError("pyramids are built at p = 4 (the order of the tetrahedra they join)")
    sol = sol_points(p)
    fpts, fface = flux_points(p)
    nsp, nfp = sol.shape[0], fpts.shape[0]
    Vs = basis(sol, p)
    Vinv = np.linalg.inv(Vs)
    lag = lambda x: basis(x, p) @ Vinv
    interp = lag(fpts)
    G = basis_grad(sol, p)
    deriv = np.stack([G[:, :, d] @ Vinv for d in range(3)])
    qp, qw = quad_pyr(p + 4)
    Lq = lag(qp)
    M = Lq.T @ (qw[:, None] * Lq)
    weights = Lq.T @ qw
    E = np.zeros((nsp, nfp))
    g, gw = polys.gauss_legendre(p + 3)
    for f in range(5):
        cols = np.nonzero(fface == f)[0]
        if f == 0:
            # base: tensor Lagrange on the Gauss points of the face, dS = dx dy
            X, Y = np.meshgrid(g, g, indexing="ij")
            W = np.outer(gw, gw).ravel()
            xq = np.stack([X.ravel(), Y.ravel(), -np.ones(X.size)], axis=1)
            gf, _ = polys.gauss_legendre(p + 1)
            Lx = polys.lagrange_matrix(gf, xq[:, 0])
            Ly = polys.lagrange_matrix(gf, xq[:, 1])
            phi = (Ly[:, :, None] * Lx[:, None, :]).reshape(len(W), -1)   # flux point i + (p+1) j
            E[:, cols] = lag(xq).T @ (W[:, None] * phi)
        else:
            c0, c1, c2 = CORNERS[list(FACES[f])]
            tq, tw = tet.quad_tri(p + 3)
            xq = c0 + tq[:, :1] * (c1 - c0) + tq[:, 1:] * (c2 - c0)
            st = np.array([np.linalg.lstsq(np.stack([c1 - c0, c2 - c0], 1), x - c0, rcond=None)[0]
                           for x in fpts[cols]])
            Cf = np.linalg.inv(tet.tri_monomials(st, p))
            phi = tet.tri_monomials(tq, p) @ Cf
            W = tw * 2.0 * face_area(f)
            E[:, cols] = lag(xq).T @ (W[:, None] * phi)
    lift = np.linalg.solve(M, E)
    normals = np.array([face_normal(f) for f in fface])
    degs = np.array([max(i, j) + k for i, j, k in modes(p)])
    return ElementOps(PYR, p, sol, fpts, fface, normals, interp, deriv, lift, weights, 5, 0, Vs, degs)
