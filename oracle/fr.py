"""The Flux Reconstruction right-hand side, written out step by step (oracle, FP64).

Follows Sec. "Flux Reconstruction" literally, per element type block, with dense
operators (elements.py) and metric terms from geometry.py:

  1. u_f = interp u                                              (eq:disu)
  2. F^C_sigma = |S^T n~| 𝔉(u_sigma, u'_sigma, n^)               (eq:comm_flux)
     n^ = S^T n~ / |S^T n~| is the outward physical unit normal; the length
     |S^T n~| turns the physical normal flux into the transformed one (reading of
     the paper's silent scaling between the two).
  3. f~_zeta = S_zeta f(u_zeta); f~perp_sigma = n~_sigma . interp f~   (second eq:disu)
  4. div_zeta = sum_i deriv_i f~_i + lift (F^C - f~perp)          (eq:FRfinal; the
     printed jump term is read as "common minus discontinuous normal flux")
     R_zeta = - div_zeta / J_zeta                                (transformed equation)

Navier--Stokes (the paper names the equations; the viscous discretisation is the
LDG reading): common solution u^ = (u_L + u_R)/2 + beta (u_L - u_R), corrected
reference gradient  grad~u = sum_i deriv_i u e_i + lift (n~ (u^ - u_f)), physical
gradient grad u = G^{-T} grad~u at solution points, interpolated to flux points;
flux f = f_inv - f_v; common flux along the left side's normal
    𝔉 = 𝔉_inv(u_L, u_R, n^_L) - [ (f_vL + f_vR)/2 - beta (f_vL - f_vR) ] . n^_L
        + tau (u_L - u_R),
entering the left element as +|S|𝔉 and the right element as -|S|𝔉.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import physics

EULER = 0
NAVIER_STOKES = 1


@dataclass
class Params:
    system: int = EULER
    riemann: int = 0            # 0 Rusanov, 1 HLLC
    gamma: float = 1.4
    mu: float = 1.0 / 1600.0
    prandtl: float = 0.71
    ldg_beta: float = 0.5
    ldg_tau: float = 0.1


def _apply(op, x):
    """Apply op [a][b] along the last axis of x [..., b] -> [..., a]."""
    x = np.ascontiguousarray(x)
    return (x.reshape(-1, x.shape[-1]) @ op.T).reshape(x.shape[:-1] + (op.shape[0],))


def transform_flux(S, f):
    """f~_i = sum_j S_ij f_j: S [n][nsp][3][3], f [5][3][n][nsp] -> [5][3][n][nsp]."""
    out = np.zeros_like(f)
    for i in range(3):
        for j in range(3):
            out[:, i] += S[None, :, :, i, j] * f[:, j]
    return out


def gather(blocks, vals, b):
    """Values at the paired flux points: vals[bi] is [n_bi][C][nfp_bi] -> [n_b][C][nfp_b]."""
    C = vals[0].shape[1]
    out = np.empty((len(b.elems), C, b.ops.nfp))
    ot = np.moveaxis(out, 1, 2)                     # [n][nfp][C] view
    for tb in range(len(blocks)):
        mask = b.nbr_type == tb
        if np.any(mask):
            ot[mask] = vals[tb][b.nbr_elem[mask], :, b.nbr_fp[mask]]
    return out


def _left_right(b, own, nbr):
    """(u_L, u_R) [C][n][nfp] from own/neighbour values [n][C][nfp]."""
    L = b.is_left[:, None, :]
    uL = np.where(L, own, nbr)
    uR = np.where(L, nbr, own)
    return np.moveaxis(uL, 1, 0), np.moveaxis(uR, 1, 0)


def gradients(blocks, u_list, prm: Params):
    """Corrected physical gradients: per block (grad_sol [n][5][3][nsp], grad_fp [n][5][3][nfp])."""
    uf = [_apply(b.ops.interp, u) for b, u in zip(blocks, u_list)]
    out = []
    for bi, (b, u) in enumerate(zip(blocks, u_list)):
        ufn = gather(blocks, uf, b)
        uL, uR = _left_right(b, uf[bi], ufn)
        uhat = 0.5 * (uL + uR) + prm.ldg_beta * (uL - uR)          # [5][n][nfp]
        jump = np.moveaxis(uhat, 0, 1) - uf[bi]                     # [n][5][nfp]
        gt = np.empty(u.shape[:2] + (3, u.shape[2]))                # [n][5][3][nsp]
        for i in range(3):
            gt[:, :, i, :] = _apply(b.ops.deriv[i], u) + _apply(b.ops.lift, jump * b.ops.normals[:, i])
        # grad_j = sum_i (G^{-1})_{ij} gt_i = sum_i S_ij / J gt_i
        Ginv = b.S / b.J[..., None, None]                          # [n][nsp][3][3]
        g = np.zeros_like(gt)
        for j in range(3):
            for i in range(3):
                g[:, :, j, :] += Ginv[:, None, :, i, j] * gt[:, :, i, :]
        gf = _apply(b.ops.interp, g)
        out.append((g, gf))
    return out


def common_flux(blocks, bi, uf, gfs, prm: Params):
    """Transformed common normal flux |S^T n~| * (+-𝔉) at the flux points of block bi: [5][n][nfp]."""
    b = blocks[bi]
    gam = prm.gamma
    ufn = gather(blocks, uf, b)
    uL, uR = _left_right(b, uf[bi], ufn)
    mag = np.linalg.norm(b.snorm, axis=2)                      # [n][nfp]
    nhat = np.moveaxis(b.snorm / mag[..., None], 2, 0)         # [3][n][nfp]
    sgn = np.where(b.is_left, 1.0, -1.0)
    nL = nhat * sgn
    F = physics.riemann(prm.riemann, uL, uR, nL, gam)
    if gfs is not None:
        gf_nbr = gather(blocks, gfs, b)
        gL, gR = _left_right(b, gfs[bi], gf_nbr)                # [15][n][nfp]
        gL = gL.reshape((5, 3) + gL.shape[1:])
        gR = gR.reshape((5, 3) + gR.shape[1:])
        fvL = physics.viscous_flux(uL, gL, gam, prm.mu, prm.prandtl)
        fvR = physics.viscous_flux(uR, gR, gam, prm.mu, prm.prandtl)
        beta = prm.ldg_beta
        fvc = 0.5 * (fvL + fvR) - beta * (fvL - fvR)
        F = F - np.einsum("vj...,j...->v...", fvc, nL) + prm.ldg_tau * (uL - uR)
    return mag * sgn * F


def rhs(blocks, u_list, prm: Params):
    """R = du/dt per block, each [n][5][nsp]."""
    gam = prm.gamma
    uf = [_apply(b.ops.interp, u) for b, u in zip(blocks, u_list)]
    ns = prm.system == NAVIER_STOKES
    if ns:
        grads = gradients(blocks, u_list, prm)
        gfs = [g[1].reshape(g[1].shape[0], 15, -1) for g in grads]
    out = []
    for bi, (b, u) in enumerate(zip(blocks, u_list)):
        ops = b.ops
        ut = np.moveaxis(u, 1, 0)                                  # [5][n][nsp]
        f = physics.euler_flux(ut, gam)                            # [5][3][n][nsp]
        if ns:
            g = np.moveaxis(grads[bi][0], (1, 2), (0, 1))          # [5][3][n][nsp]
            f = f - physics.viscous_flux(ut, g, gam, prm.mu, prm.prandtl)
        # step 3: transformed flux at solution points and its normal trace
        ftil = transform_flux(b.S, f)                              # [5][3][n][nsp]
        ftf = _apply(ops.interp, ftil)                             # [5][3][n][nfp]
        fperp = sum(ops.normals[:, i] * ftf[:, i] for i in range(3))   # [5][n][nfp]
        # step 2: common normal flux along the left side's outward normal
        Fc = common_flux(blocks, bi, uf, gfs if ns else None, prm)   # [5][n][nfp]
        # step 4: corrected divergence
        div = sum(_apply(ops.deriv[i], ftil[:, i]) for i in range(3))
        div = div + _apply(ops.lift, Fc - fperp)                   # [5][n][nsp]
        out.append(np.moveaxis(-div / b.J[None], 0, 1).copy())
    return out
