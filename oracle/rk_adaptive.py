"""Adaptive time stepping with an embedded Runge--Kutta pair (oracle, FP64).

The paper (Sec. "Adaptive time stepping") states that low-storage Runge--Kutta
schemes with embedded pairs give a cheap estimate of the error of each step, which,
once normalised, decides whether the step is accepted and sets the next step size
(larger after accepted steps, smaller after rejected ones).  It names no scheme,
norm or controller; the reading used here:

  scheme     the four-stage, third-order pair with a second-order embedded solution in
             the low-storage "2R+" form of Kennedy, Carpenter & Lewis (Appl. Numer. Math.
             35, 2000), RK3(2)4[2R+]C: a Butcher tableau whose entries below the
             subdiagonal repeat the weights (a_ij = b_j for j < i - 1), so two state
             registers carry the step; written out here in plain Butcher form
  error      e = u_{n+1} - u^_{n+1} = dt sum_i (b_i - b^_i) k_i
  norm       RMS over every value of e / (atol + rtol max(|u_n|, |u_{n+1}|))
  accept     norm <= 1
  new step   dt <- dt min(fac_max, max(fac_min, safety norm^(-1/3)))  (elementary
             controller, exponent 1 / (order of the embedded solution + 1)); a
             non-finite norm rejects with fac_min
  last step  shortened to land on t_end

This module is test infrastructure; only tests/ and the bench's CPU leg use it.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction as Fr

import numpy as np

# RK3(2)4[2R+]C: subdiagonal a_{i+1,i}, weights b, embedded weights b^ (published rationals)
A_SUB = (Fr(11847461282814, 36547543011857), Fr(3943225443063, 7078155732230),
         Fr(-346793006927, 4029903576067))
B = (Fr(1017324711453, 9774461848756), Fr(8237718856693, 13685301971492),
     Fr(57731312506979, 19404895981398), Fr(-101169746363290, 37734290219643))
BHAT = (Fr(15763415370699, 46270243929542), Fr(514528521746, 5659431552419),
        Fr(27030193851939, 9429696342944), Fr(-69544964788955, 30262026368149))
ORDER, EMBEDDED_ORDER, STAGES = 3, 2, 4


def butcher():
    """Full Butcher matrix A [4][4] (exact rationals) of the 2R+ scheme."""
    A = [[Fr(0)] * STAGES for _ in range(STAGES)]
    for i in range(1, STAGES):
        for j in range(i - 1):
            A[i][j] = B[j]
        A[i][i - 1] = A_SUB[i - 1]
    return A


def nodes():
    return [sum(r) for r in butcher()]


@dataclass
class Controller:
    atol: float = 1e-6
    rtol: float = 1e-6
    safety: float = 0.9
    fac_min: float = 0.3
    fac_max: float = 2.5


def step(rhs, u, dt):
    """One step in Butcher form for a state given as a list of arrays.  Returns
    (u_{n+1}, e) with e = u_{n+1} - u^_{n+1}."""
    A = [[float(x) for x in r] for r in butcher()]
    k = []
    for i in range(STAGES):
        s = [a + dt * sum(A[i][j] * k[j][q] for j in range(i)) if i else a for q, a in enumerate(u)]
        k.append(rhs(s))
    un = [a + dt * sum(float(B[i]) * k[i][q] for i in range(STAGES)) for q, a in enumerate(u)]
    e = [dt * sum(float(B[i] - BHAT[i]) * k[i][q] for i in range(STAGES)) for q in range(len(u))]
    return un, e


def error_norm(e, u0, u1, ctl: Controller):
    num, cnt = 0.0, 0
    for ee, a, b in zip(e, u0, u1):
        sc = ctl.atol + ctl.rtol * np.maximum(np.abs(a), np.abs(b))
        num += float(np.sum((ee / sc) ** 2))
        cnt += ee.size
    return float(np.sqrt(num / cnt))


def factor(norm, ctl: Controller):
    if not np.isfinite(norm):
        return ctl.fac_min
    if norm == 0.0:
        return ctl.fac_max
    return min(ctl.fac_max, max(ctl.fac_min, ctl.safety * norm ** (-1.0 / (EMBEDDED_ORDER + 1))))


@dataclass
class Stats:
    accepted: int = 0
    rejected: int = 0
    n_rhs: int = 0
    t: float = 0.0
    dt_next: float = 0.0
    steps: list = field(default_factory=list)      # (dt, norm, accepted) per attempt


def integrate(rhs, u, t_end, dt0, ctl: Controller = Controller(), max_steps=100000):
    """Advance u from t = 0 to t_end (or until max_steps attempts)."""
    st = Stats()
    t, dt = 0.0, dt0
    while t < t_end and st.accepted + st.rejected < max_steps:
        last = dt >= t_end - t
        h = t_end - t if last else dt
        un, e = step(rhs, u, h)
        st.n_rhs += STAGES
        nrm = error_norm(e, u, un, ctl)
        ok = bool(nrm <= 1.0)
        st.steps.append((h, nrm, ok))
        if ok:
            u, t = un, (t_end if last else t + h)
            st.accepted += 1
        else:
            st.rejected += 1
        dt = h * factor(nrm, ctl)
    st.t, st.dt_next = t, dt
    return u, st
