"""Oracle connectivity: periodic face matching, flux-point pairing, left/right sides.

The tessellation is conforming (Sec. "Flux Reconstruction": non-overlapping
conforming elements; flux points of adjoining elements conform).  Faces are
matched by their centroids reduced modulo the box periods; flux points of a
matched pair are paired by coordinates after removing the periodic translation
between the two face centroids (not a per-point wrap, which would be ambiguous for
face corners of a one-cell-wide periodic box).  An
unpaired face, a non-matching flux point or J <= 0 is a mesh error.

Left/right side of a face (needed only by the LDG viscous terms, whose common
values are one-sided): the side whose outward unit normal at the face centroid has
its dominant component (first component within a relative 1e-6 of the largest
magnitude) positive.  This is a reading; the paper is silent on viscous details.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import curved, geometry
from .elements import HEX, PYR, TET, ops_for

HEX_FACE_CORNERS = [(0, 3, 4, 7), (1, 2, 5, 6), (0, 1, 4, 5), (2, 3, 6, 7), (0, 1, 2, 3), (4, 5, 6, 7)]
TET_FACE_CORNERS = [(0, 1, 3), (0, 1, 2), (0, 2, 3), (1, 2, 3)]
PYR_FACE_CORNERS = [(0, 1, 2, 3), (0, 1, 4), (1, 2, 4), (2, 3, 4), (3, 0, 4)]
N_CORNERS = {HEX: 8, TET: 4, PYR: 5}


class MeshError(ValueError):
    pass


@dataclass
class TypeBlock:
    etype: int
    elems: np.ndarray          # global element ids of this type (mesh order)
    ops: object
    X: np.ndarray              # [n][nc][3] corners
    J: np.ndarray              # [n][nsp]
    S: np.ndarray              # [n][nsp][3][3]
    Jf: np.ndarray             # [n][nfp] J at flux points
    Sf: np.ndarray             # [n][nfp][3][3] S at flux points
    snorm: np.ndarray          # [n][nfp][3]  S^T n~ at flux points
    nbr_type: np.ndarray       # [n][nfp] type block index of the paired flux point
    nbr_elem: np.ndarray       # [n][nfp] local element index in that block
    nbr_fp: np.ndarray         # [n][nfp] flux point index in that element
    is_left: np.ndarray        # [n][nfp] bool
    xsol: np.ndarray           # [n][nsp][3] physical solution points


def _corners(etype):
    return {HEX: HEX_FACE_CORNERS, TET: TET_FACE_CORNERS, PYR: PYR_FACE_CORNERS}[etype]


def _wrap(d, period):
    out = d.copy()
    for a in range(3):
        if period[a] > 0:
            out[..., a] -= period[a] * np.round(out[..., a] / period[a])
    return out


def _keys(c, period, scale):
    """Integer keys [n][3] of points c [n][3] reduced modulo the periods."""
    k = np.empty(c.shape, dtype=np.int64)
    for a in range(3):
        if period[a] > 0:
            n = int(round(period[a] / scale))
            k[:, a] = np.rint(np.mod(c[:, a], period[a]) / scale).astype(np.int64) % n
        else:
            k[:, a] = np.rint(c[:, a] / scale).astype(np.int64)
    return k


def build(mesh, order: int, metric: str = "conservative"):
    """Connectivity and geometry of `mesh` at polynomial order `order` (tets, pyramids: 4).

    Curved meshes (mesh.ho_enodes set, hexahedra or tetrahedra of geometry order
    mesh.geo_order, one type per mesh): metric terms, J and solution points come from
    the high-order map (curved.py, `metric` "conservative" or "cross"); faces are
    matched, flux points paired and left/right sides chosen from the corners as for
    straight elements."""
    period = np.asarray(mesh.period, dtype=np.float64)
    types = [t for t in (HEX, TET, PYR) if np.any(mesh.etype == t)]
    ho = getattr(mesh, "ho_enodes", None)
    if ho is not None and len(types) != 1:
        raise MeshError("curved meshes hold one element type")
    blocks = []
    for t in types:
        elems = np.nonzero(mesh.etype == t)[0]
        ops = ops_for(t, order if t == HEX else 4)
        nc = N_CORNERS[t]
        X = mesh.xyz[mesh.enodes[elems, :nc]]
        if t == PYR:
            if ho is not None:
                raise MeshError("pyramids are straight-sided")
            skew = np.linalg.norm(X[:, 2] - X[:, 1] - X[:, 3] + X[:, 0], axis=1)
            if np.any(skew > 1e-10 * np.ptp(mesh.xyz, axis=0).max()):
                raise MeshError("pyramid base is not a parallelogram (the map must be affine)")
        if ho is None:
            J, S = geometry.metric(t, X, ops.sol_pts)
            Jf, Sf = geometry.metric(t, X, ops.flux_pts)
            xsol = geometry.map_points(t, X, ops.sol_pts)
        else:
            q = int(mesh.geo_order)
            Xh = mesh.xyz[ho[elems]]
            if t == HEX:
                J, S = curved.metric(metric, q, order, Xh, ops.sol_pts)
                Jf, Sf = curved.metric(metric, q, order, Xh, ops.flux_pts)
                xsol = curved.map_points(q, Xh, ops.sol_pts)
            else:
                J, S = curved.tet_metric(metric, q, Xh, ops.sol_pts)
                Jf, Sf = curved.tet_metric(metric, q, Xh, ops.flux_pts)
                xsol = curved.tet_map_points(q, Xh, ops.sol_pts)
        if np.any(J <= 0) or np.any(Jf <= 0):
            raise MeshError("element with J <= 0")
        snorm = np.einsum("epij,pi->epj", Sf, ops.normals)
        n, nfp = len(elems), ops.nfp
        blocks.append(TypeBlock(t, elems, ops, X, J, S, Jf, Sf, snorm,
                                np.full((n, nfp), -1), np.full((n, nfp), -1),
                                np.full((n, nfp), -1), np.zeros((n, nfp), bool), xsol))
    # ---- face matching (vectorised) ------------------------------------------------
    span = np.ptp(mesh.xyz, axis=0).max()
    scale = 1e-8 * max(span, 1e-300)
    recs = []                                   # (block, elem, face, key0, key1, key2)
    for bi, b in enumerate(blocks):
        fc = _corners(b.etype)
        for f, corners in enumerate(fc):
            cen = b.X[:, list(corners), :].mean(axis=1)          # [n][3]
            keys = _keys(cen, period, scale)
            n = len(b.elems)
            recs.append(np.column_stack([np.full(n, bi), np.arange(n), np.full(n, f), keys]))
    recs = np.concatenate(recs).astype(np.int64)
    order = np.lexsort((recs[:, 5], recs[:, 4], recs[:, 3]))
    recs = recs[order]
    same = np.all(recs[1:, 3:] == recs[:-1, 3:], axis=1)
    # every key must occur exactly twice
    run_start = np.concatenate([[True], ~same])
    starts = np.nonzero(run_start)[0]
    lengths = np.diff(np.concatenate([starts, [len(recs)]]))
    if np.any(lengths != 2):
        raise MeshError(f"{int(np.sum(lengths != 2))} faces without exactly one partner")
    pa, pb = recs[starts], recs[starts + 1]
    combos = np.unique(np.column_stack([pa[:, 0], pa[:, 2], pb[:, 0], pb[:, 2]]), axis=0)
    for ba, fa, bb, fb in combos:
        sel = (pa[:, 0] == ba) & (pa[:, 2] == fa) & (pb[:, 0] == bb) & (pb[:, 2] == fb)
        ea, eb = pa[sel, 1], pb[sel, 1]
        A, B = blocks[ba], blocks[bb]
        ia = np.nonzero(A.ops.flux_face == fa)[0]
        ib = np.nonzero(B.ops.flux_face == fb)[0]
        if len(_corners(A.etype)[fa]) != len(_corners(B.etype)[fb]):
            raise MeshError("matched faces of different kinds")
        xa = geometry.map_points(A.etype, A.X[ea], A.ops.flux_pts[ia])     # [m][q][3]
        xb = geometry.map_points(B.etype, B.X[eb], B.ops.flux_pts[ib])
        # the periodic translation between the two faces, from their centroids
        ca = A.X[ea][:, list(_corners(A.etype)[fa]), :].mean(axis=1)
        cb = B.X[eb][:, list(_corners(B.etype)[fb]), :].mean(axis=1)
        shift = (ca - cb) - _wrap(ca - cb, period)                        # [m][3]
        d = xa[:, :, None, :] - xb[:, None, :, :] - shift[:, None, None, :]
        dist = np.linalg.norm(d, axis=3)                                   # [m][q][q]
        match = np.argmin(dist, axis=2)                                    # [m][q]
        best = np.take_along_axis(dist, match[:, :, None], axis=2)[..., 0]
        if np.any(best > 1e-8 * span) or np.any(np.sort(match, axis=1) != np.arange(len(ia))):
            raise MeshError("flux points of matched faces do not conform")
        # left/right from side A's outward normal at the face centroid
        fc_ref = A.ops.flux_pts[ia].mean(axis=0)
        nref = A.ops.normals[ia[0]]
        sn = geometry.scaled_normals(A.etype, A.X[ea], fc_ref[None, :], nref[None, :])[:, 0]
        nhat = sn / np.linalg.norm(sn, axis=1, keepdims=True)
        mag = np.abs(nhat)
        first = np.argmax(mag >= (1 - 1e-6) * mag.max(axis=1, keepdims=True), axis=1)
        a_left = nhat[np.arange(len(ea)), first] > 0
        sb = ib[match]                                                      # [m][q]
        sa = np.broadcast_to(ia, sb.shape)
        EA = np.broadcast_to(ea[:, None], sb.shape)
        EB = np.broadcast_to(eb[:, None], sb.shape)
        A.nbr_type[EA, sa], A.nbr_elem[EA, sa], A.nbr_fp[EA, sa] = bb, EB, sb
        B.nbr_type[EB, sb], B.nbr_elem[EB, sb], B.nbr_fp[EB, sb] = ba, EA, sa
        AL = np.broadcast_to(a_left[:, None], sb.shape)
        A.is_left[EA, sa] = AL
        B.is_left[EB, sb] = ~AL
    for b in blocks:
        if np.any(b.nbr_fp < 0):
            raise MeshError("unpaired flux point")
    return blocks
