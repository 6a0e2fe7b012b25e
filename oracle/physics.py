"""Compressible Euler / Navier--Stokes physics for the oracle (FP64).

State u = (rho, rho v_x, rho v_y, rho v_z, E) on the leading axis (length 5).
p = (gamma - 1)(E - rho |v|^2 / 2);  f_j = (rho v_j, rho v v_j + p e_j, (E + p) v_j).

Common interface fluxes (the paper's 𝔉 is "e.g. an appropriate Riemann solver";
these are the readings used):
  * Rusanov:  F = (f_L + f_R).n / 2 - lambda (u_R - u_L) / 2,
              lambda = max(|v_L.n| + c_L, |v_R.n| + c_R),  c = sqrt(gamma p / rho)
  * HLLC (Toro), Davis wave-speed estimates; a contact exactly at S* = 0 takes the
    left star state.
Viscous terms (constant mu, Prandtl number Pr): Newtonian stress
tau = mu (grad v + grad v^T - 2/3 div v I) and heat flux q = -(mu gamma / Pr) grad e,
e = p / ((gamma - 1) rho); viscous flux f_v,j = (0, tau_.j, tau_.j . v - q_j).
"""
from __future__ import annotations

import numpy as np


def pressure(u, gamma):
    rho = u[0]
    return (gamma - 1.0) * (u[4] - 0.5 * (u[1] ** 2 + u[2] ** 2 + u[3] ** 2) / rho)


def euler_flux(u, gamma):
    """Physical flux [5][3][...]: f[v, j] is the flux of variable v in direction j."""
    rho = u[0]
    vel = u[1:4] / rho
    p = pressure(u, gamma)
    f = np.empty((5, 3) + u.shape[1:])
    for j in range(3):
        f[0, j] = u[1 + j]
        for i in range(3):
            f[1 + i, j] = u[1 + i] * vel[j]
        f[1 + j, j] += p
        f[4, j] = (u[4] + p) * vel[j]
    return f


def normal_flux(u, n, gamma):
    """f(u).n with n [3][...] (unit or not)."""
    f = euler_flux(u, gamma)
    return f[:, 0] * n[0] + f[:, 1] * n[1] + f[:, 2] * n[2]


def rusanov(uL, uR, n, gamma):
    fL = normal_flux(uL, n, gamma)
    fR = normal_flux(uR, n, gamma)
    cL = np.sqrt(gamma * pressure(uL, gamma) / uL[0])
    cR = np.sqrt(gamma * pressure(uR, gamma) / uR[0])
    vnL = np.einsum("j...,j...->...", uL[1:4] / uL[0], n)
    vnR = np.einsum("j...,j...->...", uR[1:4] / uR[0], n)
    lam = np.maximum(np.abs(vnL) + cL, np.abs(vnR) + cR)
    return 0.5 * (fL + fR) - 0.5 * lam * (uR - uL)


def hllc(uL, uR, n, gamma):
    rL, rR = uL[0], uR[0]
    vL, vR = uL[1:4] / rL, uR[1:4] / rR
    pL, pR = pressure(uL, gamma), pressure(uR, gamma)
    cL, cR = np.sqrt(gamma * pL / rL), np.sqrt(gamma * pR / rR)
    vnL = np.einsum("j...,j...->...", vL, n)
    vnR = np.einsum("j...,j...->...", vR, n)
    SL = np.minimum(vnL - cL, vnR - cR)
    SR = np.maximum(vnL + cL, vnR + cR)
    Ss = (pR - pL + rL * vnL * (SL - vnL) - rR * vnR * (SR - vnR)) / (rL * (SL - vnL) - rR * (SR - vnR))
    fL = normal_flux(uL, n, gamma)
    fR = normal_flux(uR, n, gamma)

    def star(r, v, vn, p, E, S):
        fac = r * (S - vn) / (S - Ss)
        us = np.empty((5,) + np.shape(r))
        us[0] = fac
        for i in range(3):
            us[1 + i] = fac * (v[i] + (Ss - vn) * n[i])
        us[4] = fac * (E / r + (Ss - vn) * (Ss + p / (r * (S - vn))))
        return us

    usL = star(rL, vL, vnL, pL, uL[4], SL)
    usR = star(rR, vR, vnR, pR, uR[4], SR)
    FsL = fL + SL * (usL - uL)
    FsR = fR + SR * (usR - uR)
    return np.where(0 <= SL, fL, np.where(0 <= Ss, FsL, np.where(0 < SR, FsR, fR)))


def riemann(kind, uL, uR, n, gamma):
    for u in (uL, uR):
        if not (np.all(u[0] > 0) and np.all(pressure(u, gamma) > 0)):
            raise FloatingPointError("non-positive density or pressure at a flux point")
    if kind == 0:
        return rusanov(uL, uR, n, gamma)
    if kind == 1:
        return hllc(uL, uR, n, gamma)
    raise ValueError("unknown Riemann solver")


def viscous_flux(u, grad, gamma, mu, prandtl):
    """Viscous flux [5][3][...] from u [5][...] and conservative gradients grad [5][3][...]."""
    rho = u[0]
    vel = u[1:4] / rho
    p = pressure(u, gamma)
    e = p / ((gamma - 1.0) * rho)
    gv = np.empty((3, 3) + u.shape[1:])            # gv[i, j] = d v_i / d x_j
    for i in range(3):
        gv[i] = (grad[1 + i] - vel[i] * grad[0]) / rho
    # grad e = (grad E - (E/rho) grad rho - (rho v).grad v) / rho
    ge = (grad[4] - (u[4] / rho) * grad[0] - np.einsum("i...,ij...->j...", u[1:4], gv)) / rho
    div = gv[0, 0] + gv[1, 1] + gv[2, 2]
    tau = mu * (gv + np.swapaxes(gv, 0, 1))
    for i in range(3):
        tau[i, i] -= 2.0 / 3.0 * mu * div
    kappa = mu * gamma / prandtl
    fv = np.zeros((5, 3) + u.shape[1:])
    for j in range(3):
        for i in range(3):
            fv[1 + i, j] = tau[i, j]
        fv[4, j] = np.einsum("i...,i...->...", tau[:, j], vel) + kappa * ge[j]
    return fv
