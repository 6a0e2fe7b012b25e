"""Pins of the oracle's embedded Runge--Kutta pair and step-size controller.

The tableau satisfies the order conditions of order 3 (weights b) and 2 (embedded b^)
exactly up to the rounding of its published rationals, and the linear fourth-order
condition b A^2 c = 1/24 as well; so on u' = lambda u the step's error against exp falls
by 2^5 per halving of dt, on u' = -u^2 the global error by 2^3 (order 3), and the
embedded estimate by 2^3; the controller lands on t_end, rejects an oversized first
step, and its final error follows the tolerance.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import rk_adaptive as ra


def _conds(w):
    A, c = ra.butcher(), ra.nodes()
    Ac = [sum(A[i][j] * c[j] for j in range(4)) for i in range(4)]
    return [sum(w) - 1, sum(w[i] * c[i] for i in range(4)) - Fr(1, 2),
            sum(w[i] * c[i] ** 2 for i in range(4)) - Fr(1, 3), sum(w[i] * Ac[i] for i in range(4)) - Fr(1, 6)]


def test_order_conditions_and_low_storage_structure():
    assert all(abs(float(x)) < 1e-20 for x in _conds(ra.B))           # third order
    A, c = ra.butcher(), ra.nodes()
    Ac = [sum(A[i][j] * c[j] for j in range(4)) for i in range(4)]
    AAc = [sum(A[i][j] * Ac[j] for j in range(4)) for i in range(4)]
    assert abs(float(sum(ra.B[i] * AAc[i] for i in range(4)) - Fr(1, 24))) < 1e-20   # linear 4th
    cb = _conds(ra.BHAT)
    assert all(abs(float(x)) < 1e-20 for x in cb[:2])                 # second order ...
    assert max(abs(float(x)) for x in cb[2:]) > 1e-3                   # ... and not third
    A = ra.butcher()
    for i in range(4):                                                  # explicit, 2R+ pattern
        assert all(A[i][j] == 0 for j in range(i, 4))
        assert all(A[i][j] == ra.B[j] for j in range(i - 1))


def test_local_error_orders_linear_and_nonlinear():
    lam = -1.3 + 0.4j
    errs, ests = [], []
    for dt in (0.2, 0.1, 0.05):
        un, e = ra.step(lambda s: [lam * s[0]], [np.array([1.0 + 0j])], dt)
        errs.append(abs(un[0][0] - np.exp(lam * dt)))
        ests.append(abs(e[0][0]))
    assert all(26.0 < errs[i] / errs[i + 1] < 38.0 for i in range(2))       # ~2^5
    assert all(6.5 < ests[i] / ests[i + 1] < 9.5 for i in range(2))         # ~2^3
    # u' = -u^2, u(0) = 1: u = 1 / (1 + t); global error to t = 1 falls by ~2^3 per halving
    gerr = []
    for n in (20, 40, 80):
        u = [np.array([1.0])]
        for _ in range(n):
            u, _ = ra.step(lambda s: [-s[0] ** 2], u, 1.0 / n)
        gerr.append(abs(u[0][0] - 0.5))
    assert all(7.0 < gerr[i] / gerr[i + 1] < 10.0 for i in range(2))


def test_controller_lands_on_t_end_rejects_and_follows_tolerance():
    f = lambda s: [-s[0] ** 2]
    finals = []
    for tol in (1e-6, 1e-8):
        ctl = ra.Controller(atol=tol, rtol=tol)
        u, st = ra.integrate(f, [np.array([1.0])], 2.0, 1.0, ctl)
        assert st.t == 2.0
        assert not st.steps[0][2]                          # dt0 = 1 is far too large: rejected
        assert st.rejected >= 1 and st.accepted >= 5
        assert st.n_rhs == 4 * (st.accepted + st.rejected)
        finals.append(abs(u[0][0] - 1.0 / 3.0))
    assert finals[0] < 30 * 1e-6 and finals[1] < 30 * 1e-8
    assert 10.0 < finals[0] / finals[1] < 1000.0


def test_norm_and_factor_edge_cases():
    ctl = ra.Controller()
    z = [np.zeros(3)]
    assert ra.error_norm(z, z, z, ctl) == 0.0 and ra.factor(0.0, ctl) == ctl.fac_max
    assert ra.factor(float("nan"), ctl) == ctl.fac_min and ra.factor(1e9, ctl) == ctl.fac_min
    # norm exactly 1 at e = atol + rtol max(|u0|, |u1|) in every value
    u0, u1 = [np.array([2.0, -3.0])], [np.array([1.0, 4.0])]
    e = [ctl.atol + ctl.rtol * np.array([2.0, 4.0])]
    assert ra.error_norm(e, u0, u1, ctl) == pytest.approx(1.0, rel=1e-15)
    assert ra.factor(1.0, ctl) == pytest.approx(ctl.safety, rel=1e-15)
