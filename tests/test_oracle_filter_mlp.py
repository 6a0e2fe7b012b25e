"""Pins of the oracle's entropy filter and MLP.

Filter: sigma_0 = 1 keeps element means; zeta = 0 is the identity; the hex filter is
the tensor product of 1-D filters; the tet filter damps polynomial states shell by
shell in closed form; after filtering every check point satisfies the
bounds; untouched elements stay bit-identical; the bisection result is minimal on
the dyadic grid; the warm-started search returns the plain result.
MLP: analytic gradient vs central differences; Adam's first step in closed form;
training lowers the loss.
"""
import numpy as np
import pytest

from oracle import elements, entropy_filter as ef, fr, mesh, mlp, polys, rk
from paper_2408_16509_amd import inputs


@pytest.fixture(scope="module")
def shock_case():
    m = inputs.hex_box((4, 4, 4))
    bl = mesh.build(m, 3)
    b = bl[0]
    x = b.xsol
    ic = np.moveaxis(inputs.shock(x[..., 0], x[..., 1], x[..., 2]), 0, 1).copy()
    fp = ef.FilterParams()
    # the interpolated discontinuous IC is not admissible at the flux points: filter it first
    u0 = ef.entropy_filter(bl, [ic], [ic], fp)[0][0]
    assert ef.admissible(b, u0, ef.smin_neighbourhood(bl, [ic], fp)[0], fp)[0].all()
    prm = fr.Params(riemann=1)
    smin0 = ef.smin_neighbourhood(bl, [u0], fp)
    stage = lambda s: [ef.filter_block(bb, ss, sm, fp)[0] for bb, ss, sm in zip(bl, s, smin0)]
    # one step with the filter on the intermediate stages; the final state is left
    # unfiltered so the test below can filter it
    u1 = rk.rk4_step(lambda s: fr.rhs(bl, stage(s) if s is not None else s, prm), [u0], 2e-2)[0]
    assert np.all(np.isfinite(u1))
    return bl, u0, u1


def test_filter_operator_properties():
    for etype, p in [(0, 3), (0, 4), (1, 4)]:
        ops = elements.ops_for(etype, p)

        class B:
            pass
        b = B()
        b.ops, b.etype = ops, etype
        u = np.random.default_rng(1).normal(size=(3, 5, ops.nsp))
        np.testing.assert_allclose(ef.filtered(b, u, np.zeros(3)), u, atol=1e-13)
        uf = ef.filtered(b, u, np.array([0.5, 3.0, 40.0]))
        np.testing.assert_allclose(uf @ ops.weights, u @ ops.weights, atol=1e-13)
        if etype == 0:
            x, _ = polys.gauss_legendre(p + 1)
            V1 = np.stack([polys.legendre(k, x) for k in range(p + 1)], axis=1)
            z = 3.0
            F1 = V1 @ np.diag(np.exp(-z * np.arange(p + 1) ** 2 / p ** 2)) @ np.linalg.inv(V1)
            F = np.kron(np.kron(F1, F1), F1)
            np.testing.assert_allclose(ef.filtered(b, u[:1], np.array([z]))[0], u[0] @ F.T, atol=1e-13)


def test_tet_filter_shells_closed_form():
    """The tetrahedral filter damps each total-degree shell by exp(-zeta (d/p)^2),
    whatever orthonormal basis spans it: a state of degree <= 1 becomes its mean plus
    exp(-zeta/p^2) times the rest; a state of degree <= 2 is A + exp(-zeta/p^2) B +
    exp(-4 zeta/p^2) C for fixed fields A, B, C (fitted at three strengths, checked at
    a fourth), with A its mean."""
    ops = elements.ops_for(1, 4)

    class B:
        pass
    b = B()
    b.ops, b.etype = ops, 1
    X = ops.sol_pts
    w = ops.weights / ops.weights.sum()
    lin = 0.3 + 1.2 * X[:, 0] - 0.7 * X[:, 1] + 0.4 * X[:, 2]
    mean = lin @ w
    for z in (0.5, 3.0, 40.0):
        got = ef.filtered(b, np.tile(lin, (1, 5, 1)), np.array([z]))[0]
        np.testing.assert_allclose(got, np.tile(mean + np.exp(-z / 16) * (lin - mean), (5, 1)), atol=1e-12)
    quad = lin + 0.5 * X[:, 0] * X[:, 1] - 0.8 * X[:, 2] ** 2 + 0.2 * X[:, 1]
    fz = lambda z: ef.filtered(b, np.tile(quad, (1, 1, 1)), np.array([z]))[0, 0]
    zs = (0.0, 2.0, 7.0)
    M = np.array([[1.0, np.exp(-z / 16), np.exp(-z / 4)] for z in zs])
    ABC = np.linalg.solve(M, np.stack([fz(z) for z in zs]))
    z4 = 13.0
    np.testing.assert_allclose(fz(z4), np.array([1.0, np.exp(-z4 / 16), np.exp(-z4 / 4)]) @ ABC, atol=1e-11)
    np.testing.assert_allclose(ABC[0], np.full(ops.nsp, quad @ w), atol=1e-12)


def test_filter_bounds_minimality_and_warm_start(shock_case):
    bl, u0, u1 = shock_case
    fp = ef.FilterParams()
    b = bl[0]
    smin = ef.smin_neighbourhood(bl, [u0], fp)[0]
    un, k, ev = ef.filter_block(b, u1, smin, fp)
    troubled = np.nonzero(k != 0)[0]
    assert troubled.size >= 3
    # untouched elements are bit-identical
    assert np.array_equal(un[k == 0], u1[k == 0])
    # bounds hold (no fallback expected in this case)
    assert np.all(k >= 0)
    ok, _ = ef.admissible(b, un, smin, fp)
    assert ok.all()
    # means unchanged
    np.testing.assert_allclose(un @ b.ops.weights, u1 @ b.ops.weights, rtol=1e-14, atol=1e-14)
    # minimality on the dyadic grid
    kk = k[troubled]
    g_prev = ef._G(b, u1[troubled], smin[troubled], kk - 1, fp)
    assert not g_prev.any()
    # warm start from a noisy prediction gives the same k
    rng = np.random.default_rng(3)
    khat = np.where(k > 0, k * 2.0 ** rng.uniform(-2, 2, size=k.size), 1.0)
    un2, k2, ev2 = ef.filter_block(b, u1, smin, fp, khat=khat)
    assert np.array_equal(k2, k) and np.array_equal(un2, un)
    # and with an exact prediction it needs fewer evaluations
    _, k3, ev3 = ef.filter_block(b, u1, smin, fp, khat=np.maximum(k, 1).astype(float))
    assert np.array_equal(k3, k)
    assert ev3[troubled].sum() < ev[troubled].sum()


def test_features_shape_and_finiteness(shock_case):
    bl, u0, u1 = shock_case
    fp = ef.FilterParams()
    smin = ef.smin_neighbourhood(bl, [u0], fp)[0]
    F = ef.features(bl[0], u1, smin, fp)
    assert F.shape == (u1.shape[0], 16) and np.all(np.isfinite(F))


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(7)
    w = mlp.glorot_init(43) + 0.05 * rng.normal(size=mlp.N_PARAMS)
    X = rng.normal(size=(32, 16))
    y = rng.normal(size=32)
    loss, g = mlp.loss_and_grad(w, X, y)
    h = 1e-6
    idx = rng.choice(mlp.N_PARAMS, size=60, replace=False)
    idx = np.concatenate([idx, [mlp.N_PARAMS - 1, 0, 1024, 1088, 5248]])
    for i in idx:
        e = np.zeros_like(w)
        e[i] = h
        fd = (mlp.loss_and_grad(w + e, X, y)[0] - mlp.loss_and_grad(w - e, X, y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9


def test_adam_first_step_closed_form():
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.1, -3.0, 0.0])
    w1, m, v = mlp.adam_step(w, g, np.zeros(3), np.zeros(3), 1, lr=1e-3)
    np.testing.assert_allclose(w1, w - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_training_reduces_loss():
    rng = np.random.default_rng(9)
    X = rng.normal(size=(2048, 16))
    y = np.tanh(X[:, 0] - 0.5 * X[:, 3]) * 0.5 + 0.1 * X[:, 7]
    w0 = mlp.glorot_init(43)
    l0 = np.mean((mlp.forward(w0, X) - y) ** 2)
    w, hist = mlp.train(w0, X, y, steps=400)
    l1 = np.mean((mlp.forward(w, X) - y) ** 2)
    assert l1 < 0.2 * l0


def test_smin_neighbourhood_takes_a_neighbours_lower_entropy():
    """4 x 1 x 1 periodic cells with constant states rho = 1, p = (3, 1, 4, 2): s = p.  Each
    cell's face neighbours are the two x-adjacent cells (the y and z faces pair a cell with
    itself), so the bounds are min(s_e, s_e-1, s_e+1) = (1, 1, 1, 2): cells 0 and 2 take
    their bound from a neighbour."""
    m = inputs.hex_box((4, 1, 1))
    for p in (2, 3):
        bl = mesh.build(m, p)
        b = bl[0]
        order = np.argsort(b.X[:, :, 0].mean(axis=1))          # cells by x
        pres = np.empty(4)
        pres[order] = [3.0, 1.0, 4.0, 2.0]
        u = np.zeros((4, 5, b.ops.nsp))
        u[:, 0] = 1.0
        u[:, 4] = (pres / 0.4)[:, None]
        smin = ef.smin_neighbourhood(bl, [u], ef.FilterParams())[0]
        np.testing.assert_allclose(smin[order], [1.0, 1.0, 1.0, 2.0], rtol=1e-14)


def test_features_closed_form_hex():
    """A p = 3 hexahedron at rest with uniform pressure pb and density rb + a psi(xi_1), psi
    the orthonormal degree-(1,0,0) Legendre mode sqrt(3/8) xi_1 (orthonormal on [-1, 1]^3,
    so the mean mode's coefficient is rb sqrt(8)):
      f0 = log10(a^2 / (8 rb^2)), every other shell energy of rho, E and p is zero (-30, the floor);
      f9 = -a sqrt(3/8) / rb (minimum density on the face xi_1 = -1), f10 = 0, f13 = a sqrt(3/8) / rb;
      the entropy p rho^-gamma is lowest on the face xi_1 = +1 (s_+) and next lowest on the
      solution-point plane nearest to it (s_1); with the bound s_min set so that
      s_min (1 - eps_s) lies half-way between them, exactly the (p+1)^2 flux points of that face
      violate: f12 = 16 / 160, f11 = (s_+ - s_min) / s_min, f14 = log10(pb rb^-gamma / s_min);
      f15 = 0.  A second element moving uniformly at v_x = V: f15 = V / sqrt(gamma pb / rb),
      and zero-shell features everywhere else."""
    p, g = 3, 1.4
    ops = elements.ops_for(0, p)

    class B:
        pass
    b = B()
    b.ops, b.etype = ops, 0
    rb, a, pb, V = 1.3, 0.05, 0.8, 0.4
    xi1 = ops.sol_pts[:, 0]
    psi = np.sqrt(3.0 / 8.0) * xi1
    u = np.zeros((2, 5, ops.nsp))
    u[0, 0] = rb + a * psi
    u[0, 4] = pb / (g - 1)
    u[1, 0] = rb
    u[1, 1] = rb * V
    u[1, 4] = pb / (g - 1) + 0.5 * rb * V * V
    x, _ = polys.gauss_legendre(p + 1)
    s_plus = pb * (rb + a * np.sqrt(3.0 / 8.0)) ** -g
    s_one = pb * (rb + a * np.sqrt(3.0 / 8.0) * x.max()) ** -g
    fp = ef.FilterParams()
    smin0 = 0.5 * (s_plus + s_one) / (1 - fp.eps_s)
    smin = np.array([smin0, 0.5 * pb * rb ** -g])
    F = ef.features(b, u, smin, fp)
    want = np.full(16, -30.0)
    want[0] = np.log10(a * a / (8 * rb * rb))
    want[9], want[10], want[13] = -a * np.sqrt(3.0 / 8.0) / rb, 0.0, a * np.sqrt(3.0 / 8.0) / rb
    want[11] = (s_plus - smin0) / smin0
    want[12] = (p + 1) ** 2 / (ops.nsp + ops.nfp)
    want[14] = np.log10(pb * rb ** -g / smin0)
    want[15] = 0.0
    np.testing.assert_allclose(F[0], want, rtol=1e-9, atol=1e-12)
    want1 = np.full(16, -30.0)
    want1[9:14] = [0.0, 0.0, (pb * rb ** -g - smin[1]) / smin[1], 0.0, 0.0]
    want1[14] = np.log10(pb * rb ** -g / smin[1])
    want1[15] = V / np.sqrt(g * pb / rb)
    np.testing.assert_allclose(F[1], want1, rtol=1e-9, atol=1e-12)
