"""Pins of the oracle's curved tetrahedra (Sec. "Curved elements", Fig. fsp).

* The order-q map reproduces its nodes; a tetrahedron whose nodes lie on an affine
  map is that map, with the straight element's metric.
* q = 1: both metrics are the straight element's; q = 2 (x_l grad x_m of degree 3,
  represented by the degree-4 interpolant): the conservative metric is the exact
  metric J G^{-1}; q = 3: the two differ at truncation level.
* Free stream: the conservative metric keeps a uniform state steady (Euler with both
  Riemann solvers, Navier--Stokes) for q = 1..4; the cross-product metric does for
  q <= 3 (degree 2(q-1) <= 4, represented exactly) and does not for q = 4.
* The conservative metric's discrete divergence vanishes at the solution points;
  at every pair of flux points the two sides' unit normals are opposite and their
  area elements |S^T n~| times the reference faces' areas are equal.
* Accuracy: the right-hand side of an entropy wave on curved tetrahedra approaches
  the exact -div f at the rate h^4.
"""
import math

import numpy as np
import pytest

from oracle import curved
from oracle import fr as ofr
from oracle import geometry
from oracle import mesh as omesh
from oracle import tet as otet
from oracle.elements import TET
from paper_2408_16509_amd import inputs

REF_FACE_AREA = np.array([2.0, 2.0, 2.0, 2.0 * math.sqrt(3.0)])


def _uniform(b):
    u = np.zeros((len(b.elems), 5, b.ops.nsp))
    u[:, 0], u[:, 1], u[:, 2], u[:, 3], u[:, 4] = 1.2, 0.3, -0.2, 0.5, 2.5
    return u


def _mesh(q, n=2, **kw):
    kw.setdefault("amp", 0.2)
    return inputs.curved_tet_box((n, n, n), q=q, perturb=0.04, perturb_seed=3, **kw)


def test_geo_nodes_count_and_corners():
    for q in (1, 2, 3, 4):
        g = curved.tet_geo_nodes(q)
        assert g.shape == ((q + 1) * (q + 2) * (q + 3) // 6, 3)
        assert np.all(g >= -1 - 1e-15) and np.all(g.sum(axis=1) <= -1 + 1e-13)
    # the generator's corner nodes are the reference corners
    m = inputs.curved_tet_box((1, 1, 1), q=3, amp=0.0)
    g = curved.tet_geo_nodes(3)
    for c, ref in enumerate(otet.CORNERS):
        idx = int(np.nonzero(np.all(np.abs(g - ref) < 1e-14, axis=1))[0][0])
        assert np.array_equal(m.ho_enodes[:, idx], m.enodes[:, c])


def test_map_nodes_and_affine_case():
    rng = np.random.default_rng(0)
    for q in (2, 3, 4):
        g = curved.tet_geo_nodes(q)
        X = rng.normal(size=(2, len(g), 3))
        assert np.allclose(curved.tet_map_points(q, X, g), X, atol=1e-12)
    corners = otet.CORNERS[None] + 0.2 * rng.normal(size=(3, 4, 3))
    q = 3
    Xq = geometry.map_points(TET, corners, curved.tet_geo_nodes(q))
    pts = otet.SOL_PTS_P4
    assert np.allclose(curved.tet_map_points(q, Xq, pts), geometry.map_points(TET, corners, pts), atol=1e-13)
    J1, S1 = geometry.metric(TET, corners, pts)
    for kind in ("cross", "conservative"):
        J2, S2 = curved.tet_metric(kind, q, Xq, pts)
        assert np.allclose(J1, J2, rtol=1e-12) and np.allclose(S1, S2, atol=1e-12)


def test_q1_is_the_straight_element():
    m = _mesh(1)
    straight = inputs.Mesh(m.xyz, m.etype, m.enodes, m.period)
    b0 = omesh.build(straight, 4)[0]
    for kind in ("conservative", "cross"):
        b = omesh.build(m, 4, kind)[0]
        assert np.abs(b.S - b0.S).max() <= 1e-12 * np.abs(b0.S).max()
        assert np.allclose(b.J, b0.J, rtol=1e-12)
        assert np.allclose(b.xsol, b0.xsol, atol=1e-12)


def test_conservative_is_exact_metric_when_representable():
    m = _mesh(2)
    bc, bx = omesh.build(m, 4, "conservative")[0], omesh.build(m, 4, "cross")[0]
    assert np.abs(bc.S - bx.S).max() <= 1e-12 * np.abs(bx.S).max()
    assert np.abs(bc.snorm - bx.snorm).max() <= 1e-12 * np.abs(bx.snorm).max()
    m3 = _mesh(3)
    b3c, b3x = omesh.build(m3, 4, "conservative")[0], omesh.build(m3, 4, "cross")[0]
    assert np.abs(b3c.S - b3x.S).max() > 1e-4 * np.abs(b3x.S).max()


@pytest.mark.parametrize("q", [1, 2, 3, 4])
def test_free_stream(q):
    m = _mesh(q)
    res = {}
    for kind in ("conservative", "cross"):
        bl = omesh.build(m, 4, kind)
        worst = 0.0
        for system, riemann in ((0, 0), (0, 1), (1, 0)):
            R = ofr.rhs(bl, [_uniform(bl[0])], ofr.Params(system=system, riemann=riemann))[0]
            worst = max(worst, float(np.abs(R).max()))
        res[kind] = worst
    assert res["conservative"] <= 1e-12
    if 2 * (q - 1) > 4:
        assert res["cross"] > 1e-3
    else:
        assert res["cross"] <= 1e-12


@pytest.mark.parametrize("q", [3, 4])
def test_divergence_free_and_watertight(q):
    m = _mesh(q)
    for kind in ("conservative", "cross"):
        b = omesh.build(m, 4, kind)[0]
        div = sum(np.einsum("zy,eyn->ezn", b.ops.deriv[i], b.S[:, :, i, :]) for i in range(3))
        if kind == "conservative" or q <= 3:
            assert np.abs(div).max() <= 1e-12
        else:
            assert np.abs(div).max() > 1e-4
        mag = np.linalg.norm(b.snorm, axis=2)
        nh = b.snorm / mag[..., None]
        assert np.abs(nh + nh[b.nbr_elem, b.nbr_fp]).max() <= 1e-11
        area = mag * REF_FACE_AREA[b.ops.flux_face][None, :]
        assert np.abs(area - area[b.nbr_elem, b.nbr_fp]).max() <= 1e-11 * area.max()


def _entropy_wave(x):
    V = np.array([1.0, 0.5, -0.3])
    ph = x[..., 0] + x[..., 1] + x[..., 2]
    rho = 1 + 0.2 * np.sin(ph)
    u = np.stack([rho, rho * V[0], rho * V[1], rho * V[2], 1.0 / 0.4 + 0.5 * rho * (V @ V)], 1)
    adv = 0.2 * np.cos(ph) * V.sum()
    R = -np.stack([adv, adv * V[0], adv * V[1], adv * V[2], 0.5 * (V @ V) * adv], 1)
    return u, R


@pytest.mark.parametrize("q", [2, 3])
def test_entropy_wave_rate(q):
    errs = []
    for n in (8, 12):
        bl = omesh.build(inputs.curved_tet_box((n, n, n), q=q, amp=0.2), 4)
        u, Rex = _entropy_wave(bl[0].xsol)
        R = ofr.rhs(bl, [u], ofr.Params(system=0, riemann=1))[0]
        errs.append(np.sqrt(np.mean((R - Rex) ** 2) / np.mean(Rex ** 2)))
    assert np.log(errs[0] / errs[1]) / np.log(12 / 8) >= 4 - 0.35
