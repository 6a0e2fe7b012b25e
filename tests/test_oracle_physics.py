"""Pins of the oracle's Riemann solvers and viscous flux (consistency, symmetry, exact cases)."""
import numpy as np
import pytest

from oracle import physics
from paper_2408_16509_amd import inputs

G = 1.4


def _states(n, seed):
    return inputs.random_state((n,), seed, vel=2.0, amp=0.5)


def _normals(n, seed):
    v = np.random.default_rng(seed).normal(size=(3, n))
    return v / np.linalg.norm(v, axis=0)


@pytest.mark.parametrize("kind", [0, 1])
def test_consistency(kind):
    u = _states(200, 1)
    n = _normals(200, 2)
    F = physics.riemann(kind, u, u, n, G)
    ref = physics.normal_flux(u, n, G)
    if kind == 0:
        assert np.array_equal(F, ref)
    else:
        np.testing.assert_allclose(F, ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("kind", [0, 1])
def test_antisymmetry_and_rotation(kind):
    uL, uR = _states(300, 3), _states(300, 4)
    n = _normals(300, 5)
    F = physics.riemann(kind, uL, uR, n, G)
    F2 = physics.riemann(kind, uR, uL, -n, G)
    np.testing.assert_allclose(F, -F2, rtol=1e-13, atol=1e-12)
    # rigid rotation of velocities and normal
    th = 0.7
    Q = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1.0]])
    rot = lambda u: np.concatenate([u[:1], Q @ u[1:4], u[4:]])
    Fr = physics.riemann(kind, rot(uL), rot(uR), Q @ n, G)
    np.testing.assert_allclose(Fr, rot(F), rtol=1e-12, atol=1e-12)


def test_hllc_supersonic_upwind_and_contact():
    # supersonic to the right: flux is the left flux
    uL = inputs.prim_to_cons(np.array([1.0]), np.array([5.0]), np.array([0.0]), np.array([0.0]), np.array([1.0]))
    uR = inputs.prim_to_cons(np.array([0.5]), np.array([4.0]), np.array([0.3]), np.array([0.0]), np.array([0.8]))
    n = np.array([[1.0], [0.0], [0.0]])
    assert np.array_equal(physics.hllc(uL, uR, n, G), physics.normal_flux(uL, n, G))
    # stationary contact: same p, zero velocity, different density -> exact flux (0, p n, 0)
    uL = inputs.prim_to_cons(np.array([1.0]), *[np.zeros(1)] * 3, np.array([2.0]))
    uR = inputs.prim_to_cons(np.array([0.1]), *[np.zeros(1)] * 3, np.array([2.0]))
    F = physics.hllc(uL, uR, n, G)
    np.testing.assert_allclose(F[:, 0], [0, 2.0, 0, 0, 0], atol=1e-14)
    # Rusanov diffuses the contact (density flux nonzero)
    assert abs(physics.rusanov(uL, uR, n, G)[0, 0]) > 1e-2


def test_shock_rankine_hugoniot():
    (_, _), (r2, p2, u2) = inputs.shock_states(1.4, 3.0)
    assert abs(r2 - 27 / 7) < 1e-15 and abs(p2 - 31 / 3) < 1e-14
    # mass and momentum fluxes balance in the shock frame (shock speed Ms*c1)
    s = 3.0 * np.sqrt(1.4)
    assert abs(1.0 * (0 - s) - r2 * (u2 - s)) < 1e-13
    assert abs((1.0 * s * s + 1.0) - (r2 * (u2 - s) ** 2 + p2)) < 1e-12


def test_viscous_flux_couette():
    """v = (a y, 0, 0), constant rho, p: tau_xy = mu a, heat flux from a linear p."""
    mu, pr = 0.01, 0.71
    y = np.linspace(-1, 1, 5)
    a, b = 0.3, 0.2
    rho = np.ones_like(y)
    p = 1.0 + b * y
    u = inputs.prim_to_cons(rho, a * y, 0 * y, 0 * y, p)
    grad = np.zeros((5, 3, 5))
    grad[1, 1] = a                                    # d(rho u)/dy
    grad[4, 1] = b / 0.4 + a * a * y                  # dE/dy
    fv = physics.viscous_flux(u, grad, G, mu, pr)
    np.testing.assert_allclose(fv[1, 1], mu * a)      # tau_xy
    np.testing.assert_allclose(fv[2, 0], mu * a)      # tau_yx
    np.testing.assert_allclose(fv[0], 0.0)
    # energy flux along y: tau_xy u + kappa de/dy, e = p/(0.4 rho), de/dy = b/0.4
    np.testing.assert_allclose(fv[4, 1], mu * a * a * y + mu * G / pr * b / 0.4, rtol=1e-13)
