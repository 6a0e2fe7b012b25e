"""Pins of the oracle's element operators and of the tetrahedral point set.

The tet points are checked against the paper's printed coordinates (golden fixture
of Fig. mesh b,c) and against symmetry/unisolvence properties; operators against
exact polynomial reproduction and, for the correction term, against the DG lifting
M^{-1}E assembled by independent quadrature.
"""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import elements, polys, tet

GOLD = os.path.join(os.path.dirname(__file__), "golden", "tet_alpha_opt_p4.txt")


def _golden():
    sol, flux, mult = [], [], []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        k, x, y, z, m = line.split()
        (sol if k == "sol" else flux).append([float(x), float(y), float(z)])
        if k == "flux":
            mult.append(int(m))
    return np.array(sol), np.array(flux), np.array(mult)


def test_tet_points_match_paper():
    sol, flux, mult = _golden()
    assert sol.shape == (35, 3)
    np.testing.assert_array_equal(tet.SOL_PTS_P4, sol)
    ops = elements.tet_ops(4)
    # flux points = surface solution points, each listed once per face it lies on
    assert ops.nfp == 60 == mult.sum()
    for q, m in zip(flux, mult):
        hits = np.nonzero(np.all(np.abs(ops.flux_pts - q) < 1e-15, axis=1))[0]
        assert len(hits) == m
        assert len(set(ops.flux_face[hits])) == m


def test_tet_point_structure():
    P = tet.SOL_PTS_P4
    A = math.sqrt(3 / 7)
    assert abs(tet.A - A) < 1e-15
    n_on = sum(tet.on_face(P, f).astype(int) for f in range(4))
    assert (n_on == 0).sum() == 1 and (n_on == 1).sum() == 12 and (n_on == 2).sum() == 18 and (n_on == 3).sum() == 4
    assert np.allclose(P[n_on == 0], [[-0.5, -0.5, -0.5]])
    # unisolvent for P_4
    assert np.linalg.cond(tet.monomials(P, 4)) < 1e5


def test_tet_points_symmetric_under_vertex_permutations():
    C = tet.CORNERS
    P = tet.SOL_PTS_P4
    bary = np.linalg.solve(np.vstack([C.T, np.ones(4)]), np.vstack([P.T, np.ones(len(P))])).T
    for perm in itertools.permutations(range(4)):
        Q = bary[:, perm] @ C
        d = np.linalg.norm(Q[:, None, :] - P[None, :, :], axis=2).min(axis=1)
        assert d.max() < 2e-15


@pytest.mark.parametrize("etype,p", [(0, 1), (0, 2), (0, 3), (0, 4), (1, 4)])
def test_operators_exact_on_polynomials(etype, p):
    ops = elements.ops_for(etype, p)
    rng = np.random.default_rng(3)
    for _ in range(5):
        if etype == 0:
            # random polynomial in Q_p
            c = rng.normal(size=(p + 1,) * 3)
            f = lambda X: sum(c[a, b, d] * X[:, 0] ** a * X[:, 1] ** b * X[:, 2] ** d
                              for a in range(p + 1) for b in range(p + 1) for d in range(p + 1))
            g = lambda X, ax: sum(c[a, b, d] * [a, b, d][ax] * X[:, 0] ** (a - (ax == 0)) *
                                  X[:, 1] ** (b - (ax == 1)) * X[:, 2] ** (d - (ax == 2))
                                  for a in range(p + 1) for b in range(p + 1) for d in range(p + 1)
                                  if [a, b, d][ax] > 0)
        else:
            ex = tet.exponents(p)
            c = rng.normal(size=len(ex))
            f = lambda X: sum(ci * X[:, 0] ** a * X[:, 1] ** b * X[:, 2] ** d for ci, (a, b, d) in zip(c, ex))
            g = lambda X, ax: sum(ci * [a, b, d][ax] * X[:, 0] ** (a - (ax == 0)) *
                                  X[:, 1] ** (b - (ax == 1)) * X[:, 2] ** (d - (ax == 2))
                                  for ci, (a, b, d) in zip(c, ex) if [a, b, d][ax] > 0)
        u = f(ops.sol_pts)
        np.testing.assert_allclose(ops.interp @ u, f(ops.flux_pts), atol=1e-11 * np.abs(u).max())
        for ax in range(3):
            np.testing.assert_allclose(ops.deriv[ax] @ u, g(ops.sol_pts, ax), atol=1e-10 * np.abs(u).max() * p)
    vol = 8.0 if etype == 0 else 4.0 / 3.0
    assert abs(ops.weights.sum() - vol) < 1e-13


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_hex_radau_lift_equals_dg_lifting(p):
    """The tensor Radau correction equals M^{-1} E assembled by Gauss quadrature."""
    from oracle import nodal_dg
    ops = elements.hex_ops(p)
    M, K, B = nodal_dg._hex_matrices(ops, p + 3)
    np.testing.assert_allclose(np.linalg.solve(M, B), ops.lift, atol=1e-12)


def test_tet_mass_matrix_and_lift():
    ops = elements.tet_ops(4)
    V = ops.modal_V
    qp, qw = tet.quad_tet(7)
    Lq = tet.lagrange(ops.sol_pts, qp, 4)
    M = Lq.T @ (qw[:, None] * Lq)
    np.testing.assert_allclose(M, np.linalg.inv(V @ V.T), atol=1e-13)
    # lift of a face-constant unit normal flux integrates to the face area:
    # sum_z W_z (lift Delta)_z = int_faces Delta dS
    for f in range(4):
        d = (ops.flux_face == f).astype(float)
        area = tet.face_param(f)[3] / 2
        assert abs(ops.weights @ ops.lift @ d - area) < 1e-12
    # hex analogue: face area 4
    h = elements.hex_ops(3)
    for f in range(6):
        assert abs(h.weights @ h.lift @ (h.flux_face == f).astype(float) - 4.0) < 1e-12


@pytest.mark.parametrize("etype,p", [(0, 2), (0, 3), (1, 4)])
def test_modal_basis_orthonormal(etype, p):
    ops = elements.ops_for(etype, p)
    V = ops.modal_V
    # orthonormal in L2 of the reference element: V^T W V = I with exact weights
    # (Gauss weights integrate Q_{2p+1} exactly; tet weights are exact integrals of l_z,
    # which integrate degree-8 products only approximately, so use quadrature there)
    if etype == 0:
        G = V.T @ (ops.weights[:, None] * V)
    else:
        qp, qw = tet.quad_tet(7)
        Q = tet.ortho_basis(qp, 4)
        G = Q.T @ (qw[:, None] * Q)
    np.testing.assert_allclose(G, np.eye(V.shape[1]), atol=1e-13)
