"""Evaluate the oracle on a neighbourhood of sampled elements of a large mesh.

The FR right-hand side of an element depends only on the states of the elements within
a few face-neighbour rings of it: Euler on the element and its face neighbours (one
ring: their traces enter the common fluxes), Navier--Stokes on two rings (the
neighbours' gradients, which enter the viscous common flux, use their own neighbours'
traces), and every further right-hand side or entropy-filter application inside an RK
step adds one more ring (the filter's entropy bound reads the face neighbours).  So the
oracle's values at sampled elements of a mesh too large for it follow from its own
functions applied to the type blocks cut down to the sampled elements' rings: the same
arithmetic on fewer elements.  Flux points whose partner lies outside the kept set are
paired with themselves, which keeps the outermost ring's values finite (they are
wrong, and never reach the samples).

Only the oracle's data structures are sliced here; no arithmetic of the method is done.
"""
from __future__ import annotations

import dataclasses

import numpy as np


def rings(blocks, seeds, k):
    """Per block, sorted local indices of the elements within k face-neighbour rings of
    seeds (a list with one index array per block)."""
    keep = [np.unique(np.asarray(s, dtype=np.int64)) for s in seeds]
    for _ in range(k):
        new = [set(map(int, kb)) for kb in keep]
        for bi, b in enumerate(blocks):
            if keep[bi].size == 0:
                continue
            nt = b.nbr_type[keep[bi]].ravel()
            ne = b.nbr_elem[keep[bi]].ravel()
            for tb in range(len(blocks)):
                new[tb].update(map(int, np.unique(ne[nt == tb])))
        keep = [np.array(sorted(s), dtype=np.int64) for s in new]
    return keep


def restrict(blocks, keep):
    """Type blocks holding only the kept elements (keep: one sorted index array per block),
    neighbour indices renumbered; flux points paired outside the kept set are paired with
    themselves."""
    remap = []
    for b, kb in zip(blocks, keep):
        m = np.full(len(b.elems), -1, dtype=np.int64)
        m[kb] = np.arange(kb.size)
        remap.append(m)
    out = []
    for bi, (b, kb) in enumerate(zip(blocks, keep)):
        nt, ne, nf = b.nbr_type[kb], b.nbr_elem[kb], b.nbr_fp[kb]
        new_e = np.empty_like(ne)
        for tb in range(len(blocks)):
            sel = nt == tb
            new_e[sel] = remap[tb][ne[sel]]
        outside = new_e < 0
        own = np.broadcast_to(np.arange(kb.size)[:, None], ne.shape)
        own_fp = np.broadcast_to(np.arange(ne.shape[1])[None, :], ne.shape)
        nt2 = np.where(outside, bi, nt)
        ne2 = np.where(outside, own, new_e)
        nf2 = np.where(outside, own_fp, nf)
        out.append(dataclasses.replace(
            b, elems=b.elems[kb], X=b.X[kb], J=b.J[kb], S=b.S[kb], Jf=b.Jf[kb], Sf=b.Sf[kb], snorm=b.snorm[kb],
            nbr_type=nt2, nbr_elem=ne2, nbr_fp=nf2, is_left=b.is_left[kb], xsol=b.xsol[kb]))
    return out
