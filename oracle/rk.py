"""Classical four-stage Runge--Kutta (oracle, FP64).

The paper leaves the integrator as "a suitable explicit time integration scheme"
and lists RK4 among the available ones; the classical Butcher tableau is used:
    k1 = R(u_n), k2 = R(u_n + dt/2 k1), k3 = R(u_n + dt/2 k2), k4 = R(u_n + dt k3)
    u_{n+1} = u_n + dt/6 (k1 + 2 k2 + 2 k3 + k4)
"""
from __future__ import annotations


def rk4_step(rhs, u, dt, stage_post=None):
    """One step for a state given as a list of arrays; rhs maps such a list to its R.

    stage_post (optional) is applied to the intermediate stage states u_n + c dt k
    before their R is evaluated, and to the new state (the entropy filter hook).
    """
    sp = stage_post or (lambda s: s)
    k1 = rhs(u)
    k2 = rhs(sp([a + 0.5 * dt * k for a, k in zip(u, k1)]))
    k3 = rhs(sp([a + 0.5 * dt * k for a, k in zip(u, k2)]))
    k4 = rhs(sp([a + dt * k for a, k in zip(u, k3)]))
    return sp([a + dt / 6.0 * (q1 + 2 * q2 + 2 * q3 + q4) for a, q1, q2, q3, q4 in zip(u, k1, k2, k3, k4)])


def rk4(rhs, u, dt, n_steps, post=None):
    for _ in range(n_steps):
        u = rk4_step(rhs, u, dt)
        if post is not None:
            u = post(u)
    return u
