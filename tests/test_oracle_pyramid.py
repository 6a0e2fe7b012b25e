"""Pins of the oracle's p = 4 pyramid (the element of the hexahedron--tetrahedron
transition, Sec. "Mixed elements and domain decomposition") against what the
mathematics fixes: closed-form volume moments, the dimension and unisolvence of the
rational space, exact reproduction of every polynomial of degree <= 4 and of rational
members, closed-form derivatives, face traces equal to a hexahedron's (Q_4) and a
tetrahedron's (P_4) face spaces, the DG lifting identity, free-stream preservation on
all-pyramid and conforming hexahedron--pyramid--tetrahedron meshes, exact corrected
gradients of polynomials, h-convergence of the right-hand side, and high-order
convergence of a vortex carried from the hexahedra into the pyramid--tetrahedron layer.

The collocated divergence (step 4 of the scheme) leaves the rational space, so on
pyramids the weighted sum of the right-hand side is not exactly zero: the tests pin
that it vanishes for fluxes of degree <= 4 and that the mesh-level defect converges
faster than the scheme's own truncation error.
"""
import math
import os
import sys
import types

import numpy as np
import pytest

import oracle
from oracle import elements, fr, mesh, physics, polys, pyramid, rk
from paper_2408_16509_amd import inputs

OPS = elements.ops_for(elements.PYR, 4)


def _p4_monomials():
    return [(a, b, c) for a in range(5) for b in range(5) for c in range(5) if a + b + c <= 4]


def _rand_inside(n, seed):
    """Seeded points strictly inside the reference pyramid."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(-0.95, 0.95, n)
    s = (1 - z) / 2
    return np.stack([s * rng.uniform(-0.95, 0.95, n), s * rng.uniform(-0.95, 0.95, n), z], axis=1)


def _poly(x, coef):
    return sum(c * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** e for c, (a, b, e) in zip(coef, _p4_monomials()))


def _poly_grad(x, coef):
    g = np.zeros((3, x.shape[0]))
    for c, (a, b, e) in zip(coef, _p4_monomials()):
        X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
        if a:
            g[0] += c * a * X ** (a - 1) * Y ** b * Z ** e
        if b:
            g[1] += c * b * X ** a * Y ** (b - 1) * Z ** e
        if e:
            g[2] += c * e * X ** a * Y ** b * Z ** (e - 1)
    return g


def _pyr_moment(a, b, c):
    """Closed form of the integral of x^a y^b z^c over the reference pyramid: the section
    at height z is the square |x|, |y| <= s = (1 - z)/2, so the x and y integrals give
    2 s^(a+1)/(a+1) and 2 s^(b+1)/(b+1) (zero for odd powers), and the z integral of a
    polynomial is done exactly with numpy's polynomial class."""
    if a % 2 or b % 2:
        return 0.0
    s = np.polynomial.Polynomial([0.5, -0.5])
    integrand = (2 * s ** (a + 1) / (a + 1)) * (2 * s ** (b + 1) / (b + 1)) * np.polynomial.Polynomial([0, 1]) ** c
    anti = integrand.integ()
    return float(anti(1.0) - anti(-1.0))


# ----------------------------------------------------------------- the element
def test_space_dimension_and_unisolvence():
    assert len(pyramid.modes()) == 55 == (4 + 1) * (4 + 2) * (2 * 4 + 3) // 6
    x = OPS.sol_pts
    s = (1 - x[:, 2]) / 2
    assert x.shape == (55, 3)
    assert np.all(np.abs(x[:, :2]) < s[:, None]) and np.all(np.abs(x[:, 2]) < 1)
    assert len(np.unique(np.round(x, 12), axis=0)) == 55
    assert np.linalg.cond(pyramid.basis(x)) < 100


def test_volume_moments_closed_form():
    qp, qw = pyramid.quad_pyr(8)
    for a, b, c in [(0, 0, 0), (0, 0, 1), (2, 0, 0), (2, 2, 0), (0, 2, 3), (4, 2, 2), (1, 0, 0), (6, 0, 2)]:
        exact = _pyr_moment(a, b, c)
        got = qw @ (qp[:, 0] ** a * qp[:, 1] ** b * qp[:, 2] ** c)
        assert abs(got - exact) < 1e-14 * max(1.0, abs(exact)), (a, b, c)
    assert _pyr_moment(0, 0, 0) == pytest.approx(8 / 3, abs=1e-15)
    assert _pyr_moment(0, 0, 1) == pytest.approx(-4 / 3, abs=1e-15)     # centroid at z = -1/2
    assert _pyr_moment(2, 0, 0) == pytest.approx(8 / 15, abs=1e-15)
    # the solution-point weights integrate every polynomial of degree <= 4
    for a, b, c in _p4_monomials():
        x = OPS.sol_pts
        assert abs(OPS.weights @ (x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c) - _pyr_moment(a, b, c)) < 1e-13
    assert np.all(OPS.weights > 0)


def test_reproduces_polynomials_and_rational_members():
    coef = np.random.default_rng(11).normal(size=len(_p4_monomials()))
    y = _rand_inside(200, 12)
    lag = pyramid.basis(y) @ np.linalg.inv(pyramid.basis(OPS.sol_pts))
    np.testing.assert_allclose(lag @ _poly(OPS.sol_pts, coef), _poly(y, coef), atol=1e-12)
    np.testing.assert_allclose(OPS.interp @ _poly(OPS.sol_pts, coef), _poly(OPS.flux_pts, coef), atol=1e-12)
    # with a = x/s, b = y/s the members a^i b^j s^m q(z), m = max(i, j), deg q <= 4 - m,
    # include x y / s, x^2 y^2 / s^2 and x y z^3 / s
    for f in (lambda x: x[:, 0] * x[:, 1] / (1 - x[:, 2]),
              lambda x: (x[:, 0] * x[:, 1]) ** 2 / (1 - x[:, 2]) ** 2 + x[:, 0] * x[:, 1] * x[:, 2] ** 3 / (1 - x[:, 2])):
        np.testing.assert_allclose(lag @ f(OPS.sol_pts), f(y), atol=1e-12)
    # a degree-5 polynomial does not
    f5 = lambda x: x[:, 2] ** 5
    assert np.abs(lag @ f5(OPS.sol_pts) - f5(y)).max() > 1e-4


def test_derivatives_closed_form():
    coef = np.random.default_rng(13).normal(size=len(_p4_monomials()))
    x = OPS.sol_pts
    g = _poly_grad(x, coef)
    for i in range(3):
        np.testing.assert_allclose(OPS.deriv[i] @ _poly(x, coef), g[i], atol=1e-11)
    # x y / s with s = (1 - z)/2: gradient (y / s, x / s, x y / (2 s^2))
    s = (1 - x[:, 2]) / 2
    f = x[:, 0] * x[:, 1] / s
    ex = [x[:, 1] / s, x[:, 0] / s, x[:, 0] * x[:, 1] / (2 * s * s)]
    for i in range(3):
        np.testing.assert_allclose(OPS.deriv[i] @ f, ex[i], atol=1e-11)


def test_basis_gradient_by_finite_differences():
    y = _rand_inside(40, 14)
    G = pyramid.basis_grad(y)
    h = 1e-5
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        fd = (8 * (pyramid.basis(y + e) - pyramid.basis(y - e))
              - (pyramid.basis(y + 2 * e) - pyramid.basis(y - 2 * e))) / (12 * h)
        np.testing.assert_allclose(G[:, :, d], fd, atol=2e-7 * np.abs(G).max())


@pytest.mark.parametrize("f", range(5))
def test_face_traces_are_the_neighbours_face_spaces(f):
    """Trace on the base: Q_4 (a hexahedron's face); on a triangle: P_4 (a tetrahedron's
    face).  Each basis function restricted to the face is reproduced exactly by the
    face's own Lagrange interpolation from the face's flux points."""
    cols = np.nonzero(OPS.flux_face == f)[0]
    fp = OPS.flux_pts[cols]
    rng = np.random.default_rng(20 + f)
    if f == 0:
        assert len(cols) == 25
        y = np.column_stack([rng.uniform(-1, 1, 30), rng.uniform(-1, 1, 30), -np.ones(30)])
        g, _ = polys.gauss_legendre(5)
        Lx = polys.lagrange_matrix(g, y[:, 0])
        Ly = polys.lagrange_matrix(g, y[:, 1])
        gx = np.argmin(np.abs(fp[:, 0][:, None] - g[None, :]), axis=1)
        gy = np.argmin(np.abs(fp[:, 1][:, None] - g[None, :]), axis=1)
        phi = Lx[:, gx] * Ly[:, gy]                                      # [30][25]
    else:
        assert len(cols) == 15
        c = pyramid.CORNERS[list(pyramid.FACES[f])]
        st = rng.dirichlet(np.ones(3), 30)[:, 1:]
        y = c[0] + st[:, :1] * (c[1] - c[0]) + st[:, 1:] * (c[2] - c[0])
        stf = np.linalg.lstsq(np.stack([c[1] - c[0], c[2] - c[0]], 1), (fp - c[0]).T, rcond=None)[0].T
        mono = lambda q: np.stack([q[:, 0] ** a * q[:, 1] ** (d - a) for d in range(5) for a in range(d + 1)], 1)
        phi = mono(st) @ np.linalg.inv(mono(stf))
    B = pyramid.basis(y)
    np.testing.assert_allclose(phi @ pyramid.basis(fp), B, atol=1e-11 * np.abs(B).max())


def test_lift_is_the_dg_lifting():
    """Weighted by the quadrature weights, each face's lifting columns sum to the face
    area (4 for the base, sqrt 5 for a triangle); and for every u in the space,
    int u (lift g) dV = int_face u g dS, checked with a finer face rule."""
    fw = OPS.weights @ OPS.lift
    for f in range(5):
        area = 4.0 if f == 0 else math.sqrt(5.0)
        assert fw[OPS.flux_face == f].sum() == pytest.approx(area, rel=1e-13)
    qp, qw = pyramid.quad_pyr(10)
    Vi = np.linalg.inv(pyramid.basis(OPS.sol_pts))
    Lq = pyramid.basis(qp) @ Vi
    u = np.random.default_rng(15).normal(size=55)
    lhs = (qw * (Lq @ u)) @ (Lq @ OPS.lift)                             # [nfp]
    # right side with an independent rule per face: Gauss 9 x 9 on the base, a
    # collapsed rule of 9 points per direction with the corners taken in reverse order
    # on a triangle
    rhs = np.zeros(OPS.nfp)
    g, w = polys.gauss_legendre(9)
    for f in range(5):
        cols = np.nonzero(OPS.flux_face == f)[0]
        fp = OPS.flux_pts[cols]
        if f == 0:
            X, Y = np.meshgrid(g, g, indexing="ij")
            y = np.column_stack([X.ravel(), Y.ravel(), -np.ones(X.size)])
            W = np.outer(w, w).ravel()
            gf, _ = polys.gauss_legendre(5)
            gx = np.argmin(np.abs(fp[:, 0][:, None] - gf[None, :]), axis=1)
            gy = np.argmin(np.abs(fp[:, 1][:, None] - gf[None, :]), axis=1)
            phi = polys.lagrange_matrix(gf, y[:, 0])[:, gx] * polys.lagrange_matrix(gf, y[:, 1])[:, gy]
        else:
            c = pyramid.CORNERS[list(pyramid.FACES[f])][::-1]
            a_, b_ = np.meshgrid((g + 1) / 2, (g + 1) / 2, indexing="ij")
            t = b_.ravel()
            s = a_.ravel() * (1 - t)
            W = np.outer(w / 2, w / 2).ravel() * (1 - t) * 2 * (math.sqrt(5.0))
            y = c[0] + s[:, None] * (c[1] - c[0]) + t[:, None] * (c[2] - c[0])
            stq = np.column_stack([s, t])
            stf = np.linalg.lstsq(np.stack([c[1] - c[0], c[2] - c[0]], 1), (fp - c[0]).T, rcond=None)[0].T
            mono = lambda q: np.stack([q[:, 0] ** a * q[:, 1] ** (d - a) for d in range(5) for a in range(d + 1)], 1)
            phi = mono(stq) @ np.linalg.inv(mono(stf))
        uy = (pyramid.basis(y) @ Vi) @ u
        rhs[cols] = (W * uy) @ phi
    np.testing.assert_allclose(lhs, rhs, atol=1e-12 * np.abs(rhs).max())


def test_divergence_conservative_on_polynomial_fluxes_only():
    """w^T deriv_i f equals the boundary integral of n_i f for every f of degree <= 4,
    not for every member of the rational space (the x-derivative of x y^2 / (1 - z)
    lies outside it)."""
    fw = OPS.weights @ OPS.lift
    coef = np.random.default_rng(16).normal(size=len(_p4_monomials()))
    x = OPS.sol_pts
    for i in range(3):
        f = _poly(x, coef)
        bnd = (fw * OPS.normals[:, i]) @ (OPS.interp @ f)
        assert abs(OPS.weights @ (OPS.deriv[i] @ f) - bnd) < 1e-12
    f = x[:, 0] * x[:, 1] ** 2 / (1 - x[:, 2])          # a b^2 s^2, in the space; d/dx = b^2 s is not
    bnd = (fw * OPS.normals[:, 0]) @ (OPS.interp @ f)
    assert abs(OPS.weights @ (OPS.deriv[0] @ f) - bnd) > 1e-6


# ----------------------------------------------------------------- meshes
MESHES = {
    "pyramids": lambda: inputs.pyramid_box((2, 2, 2), apex_perturb=0.15, perturb_seed=3, permute_seed=4),
    "transition": lambda: inputs.transition_box((4, 2, 2), apex_perturb=0.15, perturb_seed=3, permute_seed=4),
    "transition_kuhn": lambda: inputs.transition_box((5, 2, 2), n_hex=2),
    "pyramids_rotated": lambda: inputs.pyramid_box((2, 2, 2), apex_perturb=0.15, perturb_seed=3, rotate_seed=5),
}


def test_transition_box_structure():
    m = inputs.transition_box((5, 2, 2), n_hex=2)
    # 2 hexahedral columns, 2 transition columns (1 pyramid + 10 tets), 1 Kuhn column
    assert m.n_of(elements.HEX) == 8 and m.n_of(elements.PYR) == 8 and m.n_of(elements.TET) == 80 + 24
    bl = mesh.build(m, 4)
    by = {b.etype: (i, b) for i, b in enumerate(bl)}
    ip, P = by[elements.PYR]
    ih, _ = by[elements.HEX]
    base = P.ops.flux_face == 0
    assert np.all(P.nbr_type[:, base] == ih)                   # every base meets a hexahedron
    assert np.all(P.nbr_type[:, ~base] != ih)                  # every triangle a tet or a pyramid
    vol = sum(np.einsum("s,es->", b.ops.weights, b.J) for b in bl)
    assert vol == pytest.approx((2 * math.pi) ** 3, rel=1e-12)


@pytest.mark.parametrize("kind", list(MESHES))
@pytest.mark.parametrize("system", [0, 1])
def test_free_stream(kind, system):
    bl = mesh.build(MESHES[kind](), 4)
    const = np.array([1.1, 0.3, -0.2, 0.4, 3.0])
    u = [np.broadcast_to(const[None, :, None], (len(b.elems), 5, b.ops.nsp)).copy() for b in bl]
    R = fr.rhs(bl, u, fr.Params(system=system))
    assert max(np.abs(r).max() for r in R) < 1e-12 * 6.0 * 25


def _smooth(x):
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    return inputs.prim_to_cons(1 + 0.2 * np.sin(X) * np.cos(Y) * np.sin(Z + 0.3), 0.3 * np.cos(X + 0.1),
                               0.2 * np.sin(Y - Z), 0.25 * np.cos(Z) * np.sin(X), 1 + 0.1 * np.cos(X + Y))


def _minus_div_exact(x, h=1e-4):
    """-div f(u) of the smooth state by sixth-order central differences of the exact flux."""
    out = 0.0
    for d in range(3):
        for c, k in [(-1 / 60, -3), (3 / 20, -2), (-3 / 4, -1), (3 / 4, 1), (-3 / 20, 2), (1 / 60, 3)]:
            xx = x.copy()
            xx[..., d] += k * h
            out = out - c * physics.euler_flux(_smooth(xx), 1.4)[:, d] / h
    return out


def _rhs_error(m):
    bl = mesh.build(m, 4)
    R = fr.rhs(bl, [np.moveaxis(_smooth(b.xsol), 0, 1).copy() for b in bl], fr.Params())
    e2 = vol = 0.0
    tot, scl = 0.0, 0.0
    for b, r in zip(bl, R):
        wj = b.ops.weights[None, :] * b.J
        e2 += np.einsum("es,evs->", wj, (r - np.moveaxis(_minus_div_exact(b.xsol), 0, 1)) ** 2)
        vol += wj.sum()
        tot = tot + np.einsum("es,evs->v", wj, r)
        scl = scl + np.einsum("es,evs->v", wj, np.abs(r))
    return math.sqrt(e2 / vol), float(np.abs(tot / scl).max())


@pytest.mark.parametrize("kind,rate", [("pyramids", 3.6), ("transition", 3.4)])
def test_rhs_converges_and_conservation_defect_vanishes(kind, rate):
    """Measured between n = 3 and 6: RHS rates 3.9 (pyramids) and 3.7 (transition), the
    design rate p for a right-hand side; the relative conservation defect 2.7e-7 -> 1.4e-9
    and 1.7e-8 -> 7.6e-11 (rate >= 7)."""
    mk = {"pyramids": lambda n: inputs.pyramid_box((n, n, n), apex_perturb=0.15, perturb_seed=3),
          "transition": lambda n: inputs.transition_box((2 * n, n, n), apex_perturb=0.15, perturb_seed=3)}[kind]
    e1, d1 = _rhs_error(mk(3))
    e2, d2 = _rhs_error(mk(6))
    assert math.log2(e1 / e2) >= rate
    assert d1 < 1e-6 and math.log2(d1 / d2) >= 6.0


def _vortex_errors(n, L=8.0, t_end=0.5):
    """L2 density error per element type of Shu's isentropic vortex advected for t_end
    across an n x n x 1 transition box of side 2L (HLLC, RK4)."""
    h = 2 * L / n
    m = inputs.transition_box((n, n, 1), n_hex=n // 2, lo=(-L, -L, -h / 2), hi=(L, L, h / 2))
    bl = mesh.build(m, 4)
    st = lambda b, t: np.moveaxis(inputs.isentropic_vortex(b.xsol[..., 0], b.xsol[..., 1], b.xsol[..., 2],
                                                           t=t, period=2 * L), 0, 1).copy()
    ns = int(np.ceil(t_end / (0.4 * h / (2.5 * 25))))
    u = rk.rk4(lambda s: fr.rhs(bl, s, fr.Params(riemann=1)), [st(b, 0.0) for b in bl], t_end / ns, ns)
    out = {}
    for b, ub in zip(bl, u):
        w = b.ops.weights[None, :] * b.J
        out[b.etype] = math.sqrt(np.einsum("es,es->", w, (ub[:, 0] - st(b, t_end)[:, 0]) ** 2) / w.sum())
    return out


def test_vortex_through_the_transition_converges():
    """The vortex starts centred on the face between the hexahedra and the pyramid layer
    and moves at unit speed into the transition cells; between n = 12 and 16 each type's
    error falls at the scheme's high order (measured: hexahedra 5.1, tetrahedra 4.5,
    pyramids 5.5; design order p + 1 = 5)."""
    e1, e2 = _vortex_errors(12), _vortex_errors(16)
    for t in (elements.HEX, elements.TET, elements.PYR):
        assert math.log(e1[t] / e2[t]) / math.log(16 / 12) >= 4.0, (t, e1[t], e2[t])


@pytest.mark.parametrize("kind", ["pyramids", "transition"])
def test_corrected_gradient_exact_for_polynomials(kind):
    """A continuous global polynomial of degree <= 2 in x has no interface jumps away from
    the periodic wrap, so the corrected gradient of interior elements is the analytic one
    (on every element type of the mesh)."""
    n = 5
    m = (inputs.pyramid_box((n, 2, 2), apex_perturb=0.15, perturb_seed=5) if kind == "pyramids"
         else inputs.transition_box((n, 2, 2), n_hex=2, apex_perturb=0.15, perturb_seed=5))
    bl = mesh.build(m, 4)
    c = np.array([[1.0, 0.1, 0.02], [0.3, -0.05, 0.01], [0.2, 0.04, -0.03], [-0.1, 0.02, 0.0], [2.5, 0.1, 0.05]])
    us = [np.stack([cv[0] + cv[1] * b.xsol[..., 0] + cv[2] * b.xsol[..., 0] ** 2 for cv in c], axis=1) for b in bl]
    grads = fr.gradients(bl, us, fr.Params(system=1))
    h = 2 * math.pi / n
    checked = 0
    for b, (g, _) in zip(bl, grads):
        X = b.xsol[..., 0]
        inner = np.all(np.abs(b.X[:, :, 0]) < math.pi - 0.5 * h, axis=1)
        g_ex = np.stack([cv[1] + 2 * cv[2] * X for cv in c], axis=1)
        np.testing.assert_allclose(g[inner][:, :, 0], g_ex[inner], atol=1e-11)
        np.testing.assert_allclose(g[inner][:, :, 1:], 0.0, atol=1e-11)
        checked += int(inner.sum())
    assert checked >= 8


def test_filter_refuses_pyramids():
    from oracle import entropy_filter as ef
    bl = mesh.build(inputs.pyramid_box((2, 2, 2)), 4)
    u = [np.broadcast_to(np.array([1.0, 0, 0, 0, 2.5])[None, :, None], (len(bl[0].elems), 5, 55)).copy()]
    with pytest.raises(NotImplementedError):
        ef.entropy_filter(bl, u, u)


def test_mesh_errors():
    m = inputs.pyramid_box((2, 2, 2))
    m.xyz = m.xyz.copy()
    base = m.enodes[m.etype == elements.PYR][0, :4]
    m.xyz[base[2]] += np.array([0.0, 0.0, 0.05])            # base no longer a parallelogram
    with pytest.raises(mesh.MeshError, match="parallelogram"):
        mesh.build(m, 4)
    with pytest.raises(mesh.MeshError, match="conform"):        # p = 3 hexahedra against p = 4 bases
        mesh.build(inputs.transition_box((4, 2, 2)), 3)
    with pytest.raises(ValueError):
        inputs.transition_box((3, 2, 2), n_hex=2)
    with pytest.raises(ValueError):
        pyramid.pyr_ops(3)


# ----------------------------------------------------------------- planted mistakes
SRC = os.path.join(os.path.dirname(oracle.__file__), "pyramid.py")
MUTATIONS = {
    "z chain term of a, b dropped": ("(dA * B * a + A * dB * b) / (2 * s) * S * C + ", ""),
    "Jacobi weight 2m": ("eval_jacobi(k, 2 * m + 2, 0, z)\n        out.append", "eval_jacobi(k, 2 * m, 0, z)\n        out.append"),
    "triangle area element halved": ("W = tw * 2.0 * face_area(f)", "W = tw * face_area(f)"),
    "layer scale dropped": ("pts.append([s * g[i], s * g[j], zg[k]])", "pts.append([0.9 * g[i], 0.9 * g[j], zg[k]])"),
}


def _mutant(old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, old
    mod = types.ModuleType("oracle._pyr_mutant")
    mod.__package__ = "oracle"
    sys.modules[mod.__name__] = mod
    try:
        exec(compile(src.replace(old, new), SRC + " (mutated)", "exec"), mod.__dict__)
    finally:
        del sys.modules[mod.__name__]
    return mod


def _pins_hold(pm):
    """The closed-form pins above, on a (possibly mutated) pyramid module."""
    ops = pm.pyr_ops.__wrapped__(4)
    coef = np.random.default_rng(13).normal(size=len(_p4_monomials()))
    x = ops.sol_pts
    ok = all(np.allclose(ops.deriv[i] @ _poly(x, coef), _poly_grad(x, coef)[i], atol=1e-10) for i in range(3))
    fw = ops.weights @ ops.lift
    ok &= all(abs(fw[ops.flux_face == f].sum() - (4.0 if f == 0 else math.sqrt(5.0))) < 1e-12 for f in range(5))
    s = (1 - x[:, 2]) / 2
    ok &= bool(np.allclose(ops.deriv[2] @ (x[:, 0] * x[:, 1] / s), x[:, 0] * x[:, 1] / (2 * s * s), atol=1e-10))
    ok &= bool(np.all(np.abs(x[:, :2]) < s[:, None]))
    return ok


def test_pins_hold_on_the_oracle():
    assert _pins_hold(pyramid)


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_pins_catch_planted_mistake(name):
    assert not _pins_hold(_mutant(*MUTATIONS[name]))
