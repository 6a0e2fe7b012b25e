"""Reference tetrahedron and its p = 4 point set, for the oracle (FP64).

The reference tetrahedron has corners (-1,-1,-1), (1,-1,-1), (-1,-1,1), (-1,1,-1)
(Fig. mesh b,c), i.e. {x, y, z >= -1, x + y + z <= -1}.

Solution points: the 35 fourth-order alpha-optimised points printed in Fig. mesh(c),
typed in here in the printed order (which is also the canonical solution-point
order of tetrahedra).  Flux points: per face, the solution points that lie on it
(Fig. mesh(b) shows exactly these 34 surface points, with multiplicities 3 at
corners, 2 on edges and 1 inside faces, 60 in total).

Bases: monomials centred at the centroid, graded by total degree; an orthonormal
basis is obtained from them by a Cholesky factorisation of their exact Gram
matrix, and exact integrals of monomials over the simplex are used throughout.
"""
from __future__ import annotations

import math
from functools import lru_cache

import mpmath
import numpy as np

from . import polys

MP_DPS = 40          # digits of the extended-precision operator construction

A = 0.654653670707977      # printed digits; equals sqrt(3/7)
B = 0.551583572090994
C = 0.103167144181987

# Fig. mesh(c), in printed order.
SOL_PTS_P4 = np.array([
    [-1, -1, -1], [-A, -1, -1], [0, -1, -1], [A, -1, -1], [1, -1, -1],
    [-1, -A, -1], [-B, -B, -1], [C, -B, -1], [A, -A, -1], [-1, 0, -1],
    [-B, C, -1], [0, 0, -1], [-1, A, -1], [-A, A, -1], [-1, 1, -1],
    [-1, -1, -A], [-B, -1, -B], [C, -1, -B], [A, -1, -A], [-1, -B, -B],
    [-0.5, -0.5, -0.5], [C, -B, -B], [-1, C, -B], [-B, C, -B], [-1, A, -A],
    [-1, -1, 0], [-B, -1, C], [0, -1, 0], [-1, -B, C], [-B, -B, C],
    [-1, 0, 0], [-1, -1, A], [-A, -1, A], [-1, -A, A], [-1, -1, 1],
], dtype=np.float64)

CORNERS = np.array([[-1, -1, -1], [1, -1, -1], [-1, -1, 1], [-1, 1, -1]], dtype=np.float64)

# faces: corner indices, outward unit normal
FACES = [
    ((0, 1, 3), np.array([0.0, 0.0, -1.0])),                     # z = -1
    ((0, 1, 2), np.array([0.0, -1.0, 0.0])),                     # y = -1
    ((0, 2, 3), np.array([-1.0, 0.0, 0.0])),                     # x = -1
    ((1, 2, 3), np.array([1.0, 1.0, 1.0]) / math.sqrt(3.0)),     # x + y + z = -1
]

CENTROID = np.array([-0.5, -0.5, -0.5])


def exponents(p: int):
    """(a, b, c) with a + b + c <= p, graded by total degree."""
    out = []
    for d in range(p + 1):
        for c in range(d + 1):
            for b in range(d - c + 1):
                out.append((d - b - c, b, c))
    return out


def on_face(pts, f, tol=1e-12):
    n = FACES[f][1]
    x0 = CORNERS[FACES[f][0][0]]
    return np.abs((pts - x0) @ n) < tol


def face_point_ids(f, pts=SOL_PTS_P4):
    return np.nonzero(on_face(pts, f))[0]


# -------------------------- exact integration ------------------------------------

def _simplex_monomial_integral(a, b, c):
    """Integral of u^a v^b w^c over the unit simplex u, v, w >= 0, u + v + w <= 1."""
    return math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)


def quad_tet(n: int = 8):
    """Collapsed Gauss--Legendre rule on the reference tet (exact to degree 2n-3)."""
    g, w = polys.gauss_legendre(n)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    P, W = [], []
    for i in range(n):
        for j in range(n):
            for k in range(n):
                s3 = g[k]
                s2 = g[j] * (1 - s3)
                s1 = g[i] * (1 - g[j]) * (1 - s3)
                jac = (1 - g[j]) * (1 - s3) ** 2
                P.append([s1, s2, s3])
                W.append(w[i] * w[j] * w[k] * jac)
    uvw = np.array(P)
    # reference tet x = -1 + 2u (unit simplex -> reference tet, volume factor 8)
    return -1.0 + 2.0 * uvw, 8.0 * np.array(W)


def quad_tri(n: int = 8):
    """Collapsed Gauss--Legendre rule on the unit triangle s, t >= 0, s + t <= 1."""
    g, w = polys.gauss_legendre(n)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    P, W = [], []
    for i in range(n):
        for j in range(n):
            t = g[j]
            s = g[i] * (1 - t)
            P.append([s, t])
            W.append(w[i] * w[j] * (1 - t))
    return np.array(P), np.array(W)


# -------------------------- bases -------------------------------------------------

def monomials(pts, p):
    x = np.atleast_2d(pts) - CENTROID
    ex = exponents(p)
    return np.stack([x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c for a, b, c in ex], axis=1)


def monomial_grads(pts, p):
    """[n_pts][n_mono][3] gradients of the centred monomials."""
    x = np.atleast_2d(pts) - CENTROID
    ex = exponents(p)
    out = np.zeros((x.shape[0], len(ex), 3))
    for m, (a, b, c) in enumerate(ex):
        if a:
            out[:, m, 0] = a * x[:, 0] ** (a - 1) * x[:, 1] ** b * x[:, 2] ** c
        if b:
            out[:, m, 1] = b * x[:, 0] ** a * x[:, 1] ** (b - 1) * x[:, 2] ** c
        if c:
            out[:, m, 2] = c * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** (c - 1)
    return out


@lru_cache(maxsize=None)
def _ortho_transform(p):
    """T with psi = T @ monomials orthonormal on the reference tet (graded)."""
    qp, qw = quad_tet(p + 3)
    Mq = monomials(qp, p)
    G = Mq.T @ (qw[:, None] * Mq)
    T = np.linalg.inv(np.linalg.cholesky(G))
    # one refinement pass (Cholesky of the residual Gram matrix; stays lower
    # triangular, so the degree grading of the modes is kept)
    Q = Mq @ T.T
    G2 = Q.T @ (qw[:, None] * Q)
    return np.linalg.inv(np.linalg.cholesky(G2)) @ T


def ortho_basis(pts, p):
    """[n_pts][n_modes] orthonormal basis values (modes graded by total degree)."""
    return monomials(pts, p) @ _ortho_transform(p).T


def ortho_degrees(p):
    return np.array([sum(e) for e in exponents(p)])


def lagrange_coeffs(nodes, p):
    """Coefficients C with l_j(x) = monomials(x) @ C[:, j]."""
    return np.linalg.inv(monomials(nodes, p))


def lagrange(nodes, x, p):
    return monomials(x, p) @ lagrange_coeffs(nodes, p)


def lagrange_grad(nodes, x, p):
    """[n_x][n_nodes][3] gradients of the Lagrange basis on `nodes`."""
    Cm = lagrange_coeffs(nodes, p)
    return np.einsum("xmd,mj->xjd", monomial_grads(x, p), Cm)


def face_param(f):
    """Face f as x = X0 + s (X1 - X0) + t (X2 - X0) and its area element |dx/ds x dx/dt|."""
    i0, i1, i2 = FACES[f][0]
    X0, X1, X2 = CORNERS[i0], CORNERS[i1], CORNERS[i2]
    e1, e2 = X1 - X0, X2 - X0
    return X0, e1, e2, float(np.linalg.norm(np.cross(e1, e2)))


def face_coords(f, pts):
    """(s, t) coordinates of points lying on face f."""
    X0, e1, e2, _ = face_param(f)
    Mt = np.stack([e1, e2], axis=1)
    st, *_ = np.linalg.lstsq(Mt, (np.atleast_2d(pts) - X0).T, rcond=None)
    return st.T


def tri_monomials(st, p):
    st = np.atleast_2d(st)
    return np.stack([st[:, 0] ** a * st[:, 1] ** (d - a) for d in range(p + 1) for a in range(d + 1)], axis=1)


# ---------------------- extended-precision construction (mpmath) -------------------
# The tetrahedral operators are assembled in MP_DPS-digit arithmetic from the same
# definitions (monomial Lagrange coefficients, Gauss rules, mass and face matrices)
# and rounded to FP64 once, so the oracle's operators carry no construction error
# beyond that final rounding.

def mp_gauss_legendre(n):
    """n-point Gauss--Legendre rule on [-1, 1], Newton-refined in mpmath."""
    mp = mpmath.mp
    x0, _ = polys.gauss_legendre(n)
    xs, ws = [], []
    for z in x0:
        z = mp.mpf(float(z))
        for _ in range(60):
            p0, p1 = mp.mpf(1), z
            for k in range(1, n):
                p0, p1 = p1, ((2 * k + 1) * z * p1 - k * p0) / (k + 1)
            dp = n * (z * p1 - p0) / (z * z - 1)
            dz = p1 / dp
            z -= dz
            if abs(dz) < mp.mpf(10) ** (-(MP_DPS - 5)):
                break
        p0, p1 = mp.mpf(1), z
        for k in range(1, n):
            p0, p1 = p1, ((2 * k + 1) * z * p1 - k * p0) / (k + 1)
        dp = n * (z * p1 - p0) / (z * z - 1)
        xs.append(z)
        ws.append(2 / ((1 - z * z) * dp * dp))
    return xs, ws


def mp_mono_row(x, p, deriv=None):
    """Centred monomial values (or one partial derivative) at a point, as mpf list."""
    c = [mpmath.mpf(float(v)) - mpmath.mpf(-0.5) for v in x] if not isinstance(x[0], mpmath.mpf) else \
        [v + mpmath.mpf(0.5) for v in x]
    out = []
    for a, b, cc in exponents(p):
        e = [a, b, cc]
        if deriv is None:
            out.append(c[0] ** a * c[1] ** b * c[2] ** cc)
        else:
            if e[deriv] == 0:
                out.append(mpmath.mpf(0))
                continue
            f = mpmath.mpf(e[deriv])
            for k in range(3):
                f *= c[k] ** (e[k] - 1 if k == deriv else e[k])
            out.append(f)
    return out


def mp_quad_tet(n):
    g, w = mp_gauss_legendre(n)
    g = [(v + 1) / 2 for v in g]
    w = [v / 2 for v in w]
    P, W = [], []
    for i in range(n):
        for j in range(n):
            for k in range(n):
                s3 = g[k]
                s2 = g[j] * (1 - s3)
                s1 = g[i] * (1 - g[j]) * (1 - s3)
                P.append([2 * s1 - 1, 2 * s2 - 1, 2 * s3 - 1])
                W.append(8 * w[i] * w[j] * w[k] * (1 - g[j]) * (1 - s3) ** 2)
    return P, W


def mp_quad_tri(n):
    g, w = mp_gauss_legendre(n)
    g = [(v + 1) / 2 for v in g]
    w = [v / 2 for v in w]
    P, W = [], []
    for i in range(n):
        for j in range(n):
            P.append([g[i] * (1 - g[j]), g[j]])
            W.append(w[i] * w[j] * (1 - g[j]))
    return P, W
