"""Entropy-bounded modal filter (oracle, FP64).

The paper (Sec. "Numerical Stability", entropy filtering; modal filtering) states
only that a modal filter is applied selectively to elements violating positivity
of density or pressure or a minimum-entropy condition, with the strength chosen
iteratively per element so as to filter as little as possible.  The details below
are the reading used (all constants are parameters):

  modes      u^ = V^{-1} u with V the orthonormal modal Vandermonde at the solution
             points (tensor Legendre for hexahedra, orthonormal P_p basis for tets)
  filter     u^_k <- sigma_k(zeta) u^_k,
             hex: sigma_ijk = exp(-zeta (i^2 + j^2 + k^2) / p^2)
             tet: sigma_k   = exp(-zeta (deg_k / p)^2)
             sigma_0 = 1, so the element mean is kept exactly (conservative)
  checks     at the solution points and the flux points (interpolated):
             rho >= eps_rho,  p >= eps_p,  s >= s_min,e - eps_s |s_min,e|,
             s = p rho^-gamma, s_min,e = min of s over the check points of e and of
             its face neighbours, evaluated on the state at the start of the step
  search     G(k) = "checks hold at zeta = k zeta_max / 2^n", zeta_max = 40 p^2, n = 20:
             G(0) -> element untouched; not G(2^n) -> zeta = zeta_max (fallback);
             else bisection on integers lo = 0, hi = 2^n keeping G(lo) false and
             G(hi) true; result zeta = hi zeta_max / 2^n.
  warm start a predicted k^ gives the bracket [floor(k^/2), ceil(2 k^)]; its ends are
             tested and the search continues in the bracket that keeps "G(lo) false,
             G(hi) true", so for a G monotone in k the result equals the plain one.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .elements import HEX, PYR
from .fr import gather


@dataclass
class FilterParams:
    gamma: float = 1.4
    eps_rho: float = 1e-8
    eps_p: float = 1e-8
    eps_s: float = 1e-4
    zeta_max_coef: float = 40.0     # zeta_max = coef * p^2
    n_bits: int = 20


def order_of(b):
    return b.ops.order


def sigma_exponent(b):
    """Per-mode exponent e_k with sigma_k = exp(-zeta e_k)."""
    if b.etype == PYR:
        # the filter's modal form is read for hexahedra and tetrahedra only; the pyramid's
        # basis is not normalised and no reading of its modal grading is pinned
        raise NotImplementedError("the entropy filter has no pyramid form")
    p = order_of(b)
    if b.etype == HEX:
        d = b.ops.modal_deg
        return (d ** 2).sum(axis=1) / float(p * p)
    return (b.ops.modal_deg / float(p)) ** 2


def entropy(rho, p, gamma):
    with np.errstate(divide="ignore", invalid="ignore"):
        s = p * np.power(np.where(rho > 0, rho, np.nan), -gamma)
    return np.where(np.isfinite(s), s, -np.inf)


def check_values(b, u, gamma):
    """(rho, p, s) at the check points [n][nsp + nfp] of states u [n][5][nsp]."""
    uf = u @ b.ops.interp.T
    w = np.concatenate([u, uf], axis=2)
    rho = w[:, 0]
    p = (gamma - 1.0) * (w[:, 4] - 0.5 * (w[:, 1] ** 2 + w[:, 2] ** 2 + w[:, 3] ** 2) / rho)
    return rho, p, entropy(rho, p, gamma)


def smin_neighbourhood(blocks, u_prev, fp: FilterParams):
    """s_min over each element and its face neighbours, per block [n]."""
    own = []
    for b, u in zip(blocks, u_prev):
        _, _, s = check_values(b, u, fp.gamma)
        own.append(s.min(axis=1))
    out = []
    for b, s_own in zip(blocks, own):
        m = s_own.copy()
        for tb in range(len(blocks)):
            mask = b.nbr_type == tb
            nb = np.where(mask, b.nbr_elem, -1)
            for f in range(b.ops.nfp):
                sel = nb[:, f] >= 0
                m[sel] = np.minimum(m[sel], own[tb][nb[sel, f]])
        out.append(m)
    return out


def admissible(b, u, smin, fp: FilterParams):
    rho, p, s = check_values(b, u, fp.gamma)
    ok = (rho >= fp.eps_rho) & (p >= fp.eps_p) & (s >= (smin - fp.eps_s * np.abs(smin))[:, None])
    return ok.all(axis=1), ok


def filtered(b, u, zeta):
    """u_F(zeta) = V diag(sigma(zeta)) V^{-1} u for states u [n][5][nsp], zeta [n]."""
    V = b.ops.modal_V
    uh = u @ np.linalg.inv(V).T                       # modal coefficients [n][5][nm]
    sig = np.exp(-zeta[:, None] * sigma_exponent(b)[None, :])
    return (uh * sig[:, None, :]) @ V.T


def _G(b, u, smin, k, fp):
    zmax = fp.zeta_max_coef * order_of(b) ** 2
    zeta = k.astype(np.float64) * (zmax / 2.0 ** fp.n_bits)
    return admissible(b, filtered(b, u, zeta), smin, fp)[0]


def filter_block(b, u, smin, fp: FilterParams, khat=None):
    """Filter one block.  Returns (u_new, k [n] int64 (0 = untouched, -1 = fallback), n_evals [n])."""
    n = u.shape[0]
    N = 2 ** fp.n_bits
    evals = np.ones(n, dtype=np.int64)
    ok0 = admissible(b, u, smin, fp)[0]
    k = np.zeros(n, dtype=np.int64)
    bad = np.nonzero(~ok0)[0]
    if bad.size:
        ub, sb = u[bad], smin[bad]
        lo = np.zeros(bad.size, dtype=np.int64)
        hi = np.full(bad.size, N, dtype=np.int64)
        active = np.ones(bad.size, bool)
        fallback = np.zeros(bad.size, bool)
        ev = np.zeros(bad.size, dtype=np.int64)
        if khat is None:
            gN = _G(b, ub, sb, hi, fp)
            ev += 1
            fallback = ~gN
            active &= gN
        else:
            kh = np.clip(np.asarray(khat, dtype=np.float64)[bad], 1.0, float(N))
            blo = np.floor(kh / 2).astype(np.int64)
            bhi = np.minimum(np.ceil(2 * kh).astype(np.int64), N)
            g_hi = _G(b, ub, sb, bhi, fp)
            ev += 1
            # G(bhi) true: try the lower end
            need_lo = g_hi & (blo > 0)
            g_lo = np.zeros(bad.size, bool)
            if np.any(need_lo):
                g_lo[need_lo] = _G(b, ub[need_lo], sb[need_lo], blo[need_lo], fp)
                ev[need_lo] += 1
            # bracket selection
            hi = np.where(g_hi, np.where(g_lo, blo, bhi), N)
            lo = np.where(g_hi, np.where(g_lo, 0, blo), bhi)
            # G(bhi) false: the top end decides fallback
            top = ~g_hi & (bhi < N)
            if np.any(top):
                gt = _G(b, ub[top], sb[top], np.full(int(top.sum()), N), fp)
                ev[top] += 1
                fb = np.zeros(bad.size, bool)
                fb[top] = ~gt
                fallback |= fb
            fallback |= ~g_hi & (bhi >= N)
            active &= ~fallback
        while True:
            run = active & (hi - lo > 1)
            if not np.any(run):
                break
            mid = (lo + hi) // 2
            g = np.zeros(bad.size, bool)
            g[run] = _G(b, ub[run], sb[run], mid[run], fp)
            ev[run] += 1
            hi = np.where(run & g, mid, hi)
            lo = np.where(run & ~g, mid, lo)
        kk = np.where(fallback, -1, hi)
        k[bad] = kk
        evals[bad] += ev
    zmax = fp.zeta_max_coef * order_of(b) ** 2
    zeta = np.where(k < 0, zmax, k * (zmax / 2.0 ** fp.n_bits))
    u_new = u.copy()
    sel = k != 0
    if np.any(sel):
        u_new[sel] = filtered(b, u[sel], zeta[sel])
    return u_new, k, evals


def entropy_filter(blocks, u, u_prev, fp: FilterParams = FilterParams(), khat=None):
    """Filter all blocks; returns (u_new list, k list, evals list)."""
    if any(b.etype == PYR for b in blocks):
        raise NotImplementedError("the entropy filter has no pyramid form")
    smin = smin_neighbourhood(blocks, u_prev, fp)
    res = [filter_block(b, ub, sm, fp, None if khat is None else khat[i])
           for i, (b, ub, sm) in enumerate(zip(blocks, u, smin))]
    return [r[0] for r in res], [r[1] for r in res], [r[2] for r in res]


# ------------------------------ MLP features ---------------------------------------

def features(b, u, smin, fp: FilterParams):
    """16 per-element features (FP64) of states u [n][5][nsp]."""
    if b.etype == PYR:
        raise NotImplementedError("the entropy filter has no pyramid form")
    g = fp.gamma
    V = b.ops.modal_V
    Vi = np.linalg.inv(V)
    rho, p, s = check_values(b, u, g)
    W = b.ops.weights / b.ops.weights.sum()
    mean = u @ W                                             # [n][5]
    rb, Eb = mean[:, 0], mean[:, 4]
    vb = mean[:, 1:4] / rb[:, None]
    pb = (g - 1.0) * (Eb - 0.5 * rb * (vb ** 2).sum(axis=1))
    cb = np.sqrt(g * np.maximum(pb, 1e-300) / rb)
    sb = np.maximum(pb, 1e-300) * rb ** (-g)
    p_sol = p[:, :u.shape[2]]
    fields = [u[:, 0], u[:, 4], p_sol]
    if b.etype == HEX:
        shell = b.ops.modal_deg.max(axis=1)
    else:
        shell = b.ops.modal_deg
    F = np.zeros((u.shape[0], 16))
    for fi, q in enumerate(fields):
        c = q @ Vi.T
        e0 = c[:, 0] ** 2 + 1e-300
        for m in range(3):
            sel = (shell == m + 1) if m < 2 else (shell >= 3)
            F[:, 3 * fi + m] = np.log10(np.maximum((c[:, sel] ** 2).sum(axis=1) / e0, 1e-30))
    F[:, 9] = rho.min(axis=1) / rb - 1.0
    F[:, 10] = p.min(axis=1) / pb - 1.0
    sm = np.where(np.isfinite(s), s, -1e30).min(axis=1)
    F[:, 11] = np.clip((sm - smin) / np.maximum(np.abs(smin), 1e-300), -10.0, 10.0)
    ok = admissible(b, u, smin, fp)[1]
    F[:, 12] = 1.0 - ok.mean(axis=1)
    F[:, 13] = np.abs(rho - rb[:, None]).max(axis=1) / rb
    F[:, 14] = np.log10(np.maximum(sb / np.maximum(smin, 1e-300), 1e-30))
    F[:, 15] = np.sqrt((vb ** 2).sum(axis=1)) / cb
    return F
