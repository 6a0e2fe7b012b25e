"""Pins of the oracle's 1-D machinery against closed forms and DG identities."""
import math

import numpy as np
import pytest

from oracle import polys


CLOSED_GL = {
    3: [-math.sqrt(3 / 5), 0.0, math.sqrt(3 / 5)],
    4: sorted([s * math.sqrt(3 / 7 + t * 2 / 7 * math.sqrt(6 / 5)) for s in (-1, 1) for t in (-1, 1)]),
    5: sorted([0.0] + [s * math.sqrt(5 + t * 2 * math.sqrt(10 / 7)) / 3 for s in (-1, 1) for t in (-1, 1)]),
}


@pytest.mark.parametrize("n", [3, 4, 5])
def test_gauss_legendre_closed_forms(n):
    x, w = polys.gauss_legendre(n)
    np.testing.assert_allclose(np.sort(x), CLOSED_GL[n], atol=1e-15)
    assert abs(w.sum() - 2.0) < 1e-15
    for d in range(2 * n):          # exact up to degree 2n-1
        exact = 0.0 if d % 2 else 2.0 / (d + 1)
        assert abs((w * x ** d).sum() - exact) < 1e-14


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_lagrange_exact_on_polynomials(p):
    x, _ = polys.gauss_legendre(p + 1)
    y = np.linspace(-1, 1, 7)
    L = polys.lagrange_matrix(x, y)
    D = polys.lagrange_deriv_matrix(x, y)
    assert np.allclose(polys.lagrange_matrix(x, x), np.eye(p + 1), atol=1e-15)
    for d in range(p + 1):
        np.testing.assert_allclose(L @ x ** d, y ** d, atol=1e-13)
        np.testing.assert_allclose(D @ x ** d, d * y ** max(d - 1, 0) if d else 0 * y, atol=1e-12)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_radau_endpoints(p):
    assert abs(polys.radau_right(p, 1.0) - 1) < 1e-15 and abs(polys.radau_right(p, -1.0)) < 1e-15
    assert abs(polys.radau_left(p, -1.0) - 1) < 1e-15 and abs(polys.radau_left(p, 1.0)) < 1e-15
    # mirror symmetry g_L(x) = g_R(-x)
    y = np.linspace(-1, 1, 9)
    np.testing.assert_allclose(polys.radau_left(p, y), polys.radau_right(p, -y), atol=1e-14)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_dg_lifting_identity(p):
    """For Gauss points the DG correction derivatives are the lifting l_a(+-1)/w_a."""
    x, w = polys.gauss_legendre(p + 1)
    lR = polys.lagrange_matrix(x, [1.0])[0]
    lL = polys.lagrange_matrix(x, [-1.0])[0]
    np.testing.assert_allclose(polys.radau_right_deriv(p, x), lR / w, atol=1e-13)
    np.testing.assert_allclose(polys.radau_left_deriv(p, x), -lL / w, atol=1e-13)
