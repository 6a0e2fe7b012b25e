"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the oracle's tests.

This module holds no arithmetic of the Flux Reconstruction method itself: it only
builds meshes (vertex coordinates and element connectivity of periodic boxes),
draws seeded random numbers, and evaluates initial-condition formulas at
coordinates the caller supplies.

Meshes
    * ``hex_box``: a structured periodic grid of 8-node hexahedra on a box, with
      optional seeded vertex perturbation (periodic images move identically) and a
      seeded permutation of the element order.
    * ``kuhn_split``: each hexahedral cell cut into 6 tetrahedra sharing the cell's
      main diagonal, which stays conforming between neighbouring cells.
    * ``curved_hex_box``: the structured periodic grid with every element curved:
      a lattice of (n q + 1)^3 nodes per box moved by a smooth periodic displacement,
      each element described by its (q+1)^3 nodes (geometry order q).
    * ``curved_tet_box``: the same curved lattice with every cell Kuhn-split, each
      tetrahedron described by its (q+1)(q+2)(q+3)/6 lattice nodes.
    * ``pyramid_box``: every cell cut into 6 pyramids, one per cell face, sharing an
      apex near the cell centre (seeded apex displacement); the bases stay exact
      parallelograms, so every pyramid is affine.
    * ``transition_box``: a conforming hexahedron--pyramid--tetrahedron box.  Along x,
      a slab of hexahedral cells, then a transition cell (a pyramid on the face shared
      with the hexahedra, its apex near the cell centre, and the other five faces'
      pyramids each cut into 2 tetrahedra), Kuhn-split cells, and a second transition
      cell facing the periodic image of the first hexahedral column.  Every cell face
      not covered by a pyramid is cut along the diagonal joining its lowest and highest
      corners, the diagonal the Kuhn split uses, so all faces conform.

Node orders
    Hexahedra use the VTK corner order, reference corners
    (-1,-1,-1) (1,-1,-1) (1,1,-1) (-1,1,-1) (-1,-1,1) (1,-1,1) (1,1,1) (-1,1,1).
    Tetrahedra list their 4 corners in the order of the reference tetrahedron
    printed with the paper's tetrahedral point sets (Fig. mesh b,c):
    (-1,-1,-1) (1,-1,-1) (-1,-1,1) (-1,1,-1).
    Pyramids list the 4 base corners in cyclic order, then the apex, matching the
    reference pyramid (-1,-1,-1) (1,-1,-1) (1,1,-1) (-1,1,-1) (0,0,1).
    Curved hexahedra of geometry order q list (q+1)^3 nodes in tensor order: node
    i + (q+1)(j + (q+1)k) sits at reference point (-1 + 2i/q, -1 + 2j/q, -1 + 2k/q).
    Curved tetrahedra of geometry order q list the nodes (i, j, k), i + j + k <= q, k
    outermost, then j, then i, at reference point (-1 + 2i/q, -1 + 2j/q, -1 + 2k/q).

Initial conditions (evaluated at caller-given physical points)
    * Taylor--Green vortex (Sec. "Accuracy", TGV initial-condition equations),
      with the reference pressure chosen from the Mach number, p0 = 1/(gamma Ma^2).
    * Planar Mach-3 shock at a seeded orientation over seeded density noise.
    * Isentropic vortex (Shu) for convergence tests.
    * Seeded random smooth/perturbed states for parity tests.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

HEX = 0
TET = 1
PYR = 2
N_CORNERS = {HEX: 8, TET: 4, PYR: 5}

# Reference corners of the two element types (documented above).
HEX_REF_CORNERS = np.array(
    [[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
     [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], dtype=np.float64)
TET_REF_CORNERS = np.array(
    [[-1, -1, -1], [1, -1, -1], [-1, -1, 1], [-1, 1, -1]], dtype=np.float64)


@dataclass
class Mesh:
    """A mixed mesh: vertices, element types and corner lists (padded to 8 with -1)."""
    xyz: np.ndarray            # [n_vert][3] float64
    etype: np.ndarray          # [n_elem] int32 (HEX, TET or PYR)
    enodes: np.ndarray         # [n_elem][8] int64, tets use the first 4, pyramids 5
    period: np.ndarray         # [3] float64 box lengths (0 = not periodic)
    meta: dict = field(default_factory=dict)
    geo_order: int = 1         # curved meshes: geometry order q of ho_enodes
    ho_enodes: np.ndarray = None   # curved meshes (one element type): [n_elem][nodes] int64, see above

    @property
    def n_elem(self) -> int:
        return int(self.etype.shape[0])

    def n_of(self, t: int) -> int:
        return int(np.count_nonzero(self.etype == t))

    def corners(self, idx) -> np.ndarray:
        """Corner coordinates [len(idx)][n_corner][3] of elements `idx` (one type)."""
        idx = np.asarray(idx)
        t = int(self.etype[idx[0]]) if idx.size else HEX
        return self.xyz[self.enodes[idx, :N_CORNERS[t]]]


def _grid_vertices(n, lo, hi, perturb, seed):
    nx, ny, nz = n
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    h = (hi - lo) / np.array([nx, ny, nz], dtype=np.float64)
    # canonical (periodic) vertex lattice [k][j][i][3]
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    canon = np.stack([lo[0] + ii * h[0], lo[1] + jj * h[1], lo[2] + kk * h[2]], axis=-1)
    if perturb:
        rng = np.random.default_rng(seed)
        canon = canon + rng.uniform(-perturb, perturb, size=canon.shape) * h
    # full lattice with periodic images on the upper faces
    K, J, I = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    xyz = canon[K % nz, J % ny, I % nx].copy()
    xyz[..., 0] += (I // nx) * (hi[0] - lo[0])
    xyz[..., 1] += (J // ny) * (hi[1] - lo[1])
    xyz[..., 2] += (K // nz) * (hi[2] - lo[2])
    return xyz.reshape(-1, 3), h


def _vid(i, j, k, n):
    nx, ny, _ = n
    return (k * (ny + 1) + j) * (nx + 1) + i


def hex_box(n=(4, 4, 4), lo=(-math.pi,) * 3, hi=(math.pi,) * 3, perturb=0.0,
            perturb_seed=None, permute_seed=None) -> Mesh:
    """Periodic box of nx*ny*nz hexahedra (VTK corner order).

    perturb: each canonical vertex coordinate moves by U(-perturb, perturb) * h,
    drawn with numpy PCG64(perturb_seed) in C order of the canonical lattice
    [k][j][i][3]; periodic images move identically.
    permute_seed: if given, element order is PCG64(permute_seed).permutation.
    """
    n = tuple(int(v) for v in n)
    xyz, h = _grid_vertices(n, lo, hi, perturb, perturb_seed)
    nx, ny, nz = n
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    corners = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0),
               (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]
    en = np.stack([_vid(i + a, j + b, k + c, n) for a, b, c in corners], axis=1).astype(np.int64)
    if permute_seed is not None:
        perm = np.random.default_rng(permute_seed).permutation(en.shape[0])
        en = en[perm]
    etype = np.full(en.shape[0], HEX, dtype=np.int32)
    period = np.asarray(hi, dtype=np.float64) - np.asarray(lo, dtype=np.float64)
    return Mesh(xyz, etype, en, period, {"n": n, "h": h, "kind": "hex_box"})


def _curved_lattice(n, q, amp, lo, hi, perturb, perturb_seed):
    """Nodes of the curved lattice shared by the curved boxes: (n_a q + 1) per direction,
    evenly spaced, moved by the periodic displacement and the optional jitter described
    in curved_hex_box.  Returns (xyz [n_nodes][3], nodes per direction, box lengths)."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    L = hi - lo
    m = [v * q + 1 for v in n]
    K, J, I = np.meshgrid(np.arange(m[2]), np.arange(m[1]), np.arange(m[0]), indexing="ij")
    x = lo[0] + I * (L[0] / (n[0] * q))
    y = lo[1] + J * (L[1] / (n[1] * q))
    z = lo[2] + K * (L[2] / (n[2] * q))
    sx, sy, sz = (2 * np.pi * (x - lo[0]) / L[0], 2 * np.pi * (y - lo[1]) / L[1], 2 * np.pi * (z - lo[2]) / L[2])
    xyz = np.stack([x + amp * L[0] / (2 * np.pi) * np.sin(sy) * np.sin(sz),
                    y + amp * L[1] / (2 * np.pi) * np.sin(sx) * np.sin(sz),
                    z + amp * L[2] / (2 * np.pi) * np.sin(sx) * np.sin(sy)], axis=-1)
    if perturb:
        hn = L / (np.asarray(n, dtype=np.float64) * q)
        jit = np.random.default_rng(perturb_seed).uniform(-perturb, perturb, size=(m[2] - 1, m[1] - 1, m[0] - 1, 3))
        xyz = xyz + jit[K % (m[2] - 1), J % (m[1] - 1), I % (m[0] - 1)] * hn
    return xyz.reshape(-1, 3), m, L


def curved_hex_box(n=(4, 4, 4), q=2, amp=0.15, lo=(-math.pi,) * 3, hi=(math.pi,) * 3,
                   perturb=0.0, perturb_seed=None, permute_seed=None) -> Mesh:
    """Periodic box of nx*ny*nz hexahedra of geometry order q, all curved.

    A lattice of (n_a q + 1) nodes per direction, evenly spaced, is moved by the
    periodic displacement (s_a = 2 pi (x_a - lo_a) / L_a, L the box lengths)
        dx = amp L_x / (2 pi) sin(s_y) sin(s_z),  dy = amp L_y / (2 pi) sin(s_x) sin(s_z),
        dz = amp L_z / (2 pi) sin(s_x) sin(s_y),
    whose gradient entries stay within amp (for equal box lengths), so the map
    stays invertible for amp well below 1.  Element (i, j, k) takes lattice nodes
    (i q + a, j q + b, k q + c), a, b, c = 0..q, in tensor order (ho_enodes); its
    8 corners, in VTK order, are the lattice nodes with a, b, c in {0, q}
    (enodes).  Nodes on the upper box faces are separate vertices from their
    periodic images on the lower faces and carry the same displacement.
    perturb: each node of the periodic lattice (n_a q nodes per direction) then moves
    by U(-perturb, perturb) times the node spacing per coordinate, drawn with numpy
    PCG64(perturb_seed) in C order of that lattice [k][j][i][3]; images move alike.
    permute_seed: if given, element order is PCG64(permute_seed).permutation.
    """
    n = tuple(int(v) for v in n)
    q = int(q)
    xyz, m, L = _curved_lattice(n, q, amp, lo, hi, perturb, perturb_seed)

    def vid(i, j, k):
        return (k * m[1] + j) * m[0] + i

    kk, jj, ii = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    ii, jj, kk = ii.ravel() * q, jj.ravel() * q, kk.ravel() * q
    ho = np.stack([vid(ii + a, jj + b, kk + c)
                   for c in range(q + 1) for b in range(q + 1) for a in range(q + 1)], axis=1).astype(np.int64)
    corners = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]
    en = np.stack([ho[:, a * q + (q + 1) * (b * q + (q + 1) * c * q)] for a, b, c in corners], axis=1)
    if permute_seed is not None:
        perm = np.random.default_rng(permute_seed).permutation(en.shape[0])
        en, ho = en[perm], ho[perm]
    etype = np.full(en.shape[0], HEX, dtype=np.int32)
    return Mesh(xyz, etype, en, L.copy(), {"n": n, "kind": "curved_hex_box", "q": q, "amp": amp},
                geo_order=q, ho_enodes=ho)


def _tet_signed_volume(c):
    a = c[..., 1, :] - c[..., 0, :]
    b = c[..., 3, :] - c[..., 0, :]
    d = c[..., 2, :] - c[..., 0, :]
    # reference axes: corner1-corner0 = 2e_x, corner3-corner0 = 2e_y, corner2-corner0 = 2e_z
    return np.einsum("...i,...i->...", a, np.cross(b, d))


def kuhn_split(mesh: Mesh, permute_seed=None) -> Mesh:
    """Cut every hexahedron into 6 tetrahedra around its corner0-corner6 diagonal.

    For each ordering (a, b, c) of the three axes the tetrahedron is the path
    corner0 -> +e_a -> +e_a+e_b -> corner6.  All cells use the same diagonal, so
    the split is conforming between neighbouring cells, including across the
    periodic boundaries.  Corner order is fixed up so the affine map has J > 0.
    """
    # VTK corner index from (dx, dy, dz) bits
    bit = {(0, 0, 0): 0, (1, 0, 0): 1, (1, 1, 0): 2, (0, 1, 0): 3,
           (0, 0, 1): 4, (1, 0, 1): 5, (1, 1, 1): 6, (0, 1, 1): 7}
    tets_local = []
    for perm in itertools.permutations(range(3)):
        p = [0, 0, 0]
        path = [bit[tuple(p)]]
        for ax in perm:
            p[ax] = 1
            path.append(bit[tuple(p)])
        tets_local.append(path)
    tets_local = np.array(tets_local)            # [6][4]
    hexes = mesh.enodes[mesh.etype == HEX, :8]
    tn = hexes[:, tets_local].reshape(-1, 4)     # [6*nh][4]
    vol = _tet_signed_volume(mesh.xyz[tn])
    neg = vol < 0
    tn[neg] = tn[neg][:, [0, 2, 1, 3]]           # swap two corners to flip orientation
    if permute_seed is not None:
        tn = tn[np.random.default_rng(permute_seed).permutation(tn.shape[0])]
    en = np.full((tn.shape[0], 8), -1, dtype=np.int64)
    en[:, :4] = tn
    etype = np.full(tn.shape[0], TET, dtype=np.int32)
    meta = dict(mesh.meta)
    meta["kind"] = "kuhn"
    return Mesh(mesh.xyz.copy(), etype, en, mesh.period.copy(), meta)


def curved_tet_box(n=(3, 3, 3), q=2, amp=0.15, lo=(-math.pi,) * 3, hi=(math.pi,) * 3,
                   perturb=0.0, perturb_seed=None, permute_seed=None) -> Mesh:
    """Periodic box of 6 nx*ny*nz tetrahedra of geometry order q, all curved.

    The lattice, displacement and jitter are those of curved_hex_box; every cell is
    cut into the 6 tetrahedra of kuhn_split (same diagonal, same corner fix-up, the
    orientation taken from the undisplaced cell).  Tetrahedron nodes (ho_enodes,
    (q+1)(q+2)(q+3)/6 of them) are the lattice nodes q C0 + i (C1 - C0) + j (C3 - C0)
    + k (C2 - C0) (C the corners' cell offsets, in the reference corner order) for
    i + j + k <= q, k outermost, then j, then i; node (i, j, k) sits at reference
    point (-1 + 2i/q, -1 + 2j/q, -1 + 2k/q).  Neighbouring tetrahedra share the
    lattice nodes of their common face, so curved faces conform.
    """
    n = tuple(int(v) for v in n)
    q = int(q)
    xyz, m, L = _curved_lattice(n, q, amp, lo, hi, perturb, perturb_seed)
    tets = []
    for perm in itertools.permutations(range(3)):
        P = [np.zeros(3, dtype=np.int64)]
        for ax in perm:
            nxt = P[-1].copy()
            nxt[ax] = 1
            P.append(nxt)
        vol = np.dot(P[1] - P[0], np.cross(P[3] - P[0], P[2] - P[0]))
        if vol < 0:
            P = [P[0], P[2], P[1], P[3]]
        tets.append(P)
    lat = [(i, j, k) for k in range(q + 1) for j in range(q + 1 - k) for i in range(q + 1 - k - j)]
    kk, jj, ii = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    cell = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1) * q          # [ncell][3]
    ho = []
    for P in tets:
        off = np.array([q * P[0] + i * (P[1] - P[0]) + j * (P[3] - P[0]) + k * (P[2] - P[0]) for i, j, k in lat])
        g = cell[:, None, :] + off[None, :, :]                                     # [ncell][nn][3]
        ho.append((g[..., 2] * m[1] + g[..., 1]) * m[0] + g[..., 0])
    ho = np.stack(ho, axis=1).reshape(-1, len(lat)).astype(np.int64)            # cell-major, 6 per cell
    c_ids = [lat.index((0, 0, 0)), lat.index((q, 0, 0)), lat.index((0, 0, q)), lat.index((0, q, 0))]
    if permute_seed is not None:
        ho = ho[np.random.default_rng(permute_seed).permutation(ho.shape[0])]
    en = np.full((ho.shape[0], 8), -1, dtype=np.int64)
    en[:, :4] = ho[:, c_ids]
    etype = np.full(ho.shape[0], TET, dtype=np.int32)
    return Mesh(xyz, etype, en, L.copy(), {"n": n, "kind": "curved_tet_box", "q": q, "amp": amp},
                geo_order=q, ho_enodes=ho)


# VTK corner index of a cell corner from its (dx, dy, dz) offsets
_CELL_BIT = {(0, 0, 0): 0, (1, 0, 0): 1, (1, 1, 0): 2, (0, 1, 0): 3,
             (0, 0, 1): 4, (1, 0, 1): 5, (1, 1, 1): 6, (0, 1, 1): 7}
# cell faces as (axis, side) with their corner offsets in cyclic order
_CELL_FACES = []
for _ax in range(3):
    for _side in (0, 1):
        _u, _v = [a for a in range(3) if a != _ax]
        _cyc = []
        for du, dv in ((0, 0), (1, 0), (1, 1), (0, 1)):
            o = [0, 0, 0]
            o[_ax], o[_u], o[_v] = _side, du, dv
            _cyc.append(_CELL_BIT[tuple(o)])
        _CELL_FACES.append((_ax, _side, _cyc))


def _cell_centres(mesh_xyz, cells, h, perturb, seed):
    """One new vertex per cell (cells [m][8] VTK corners): the centre, moved by
    U(-perturb, perturb) * h per coordinate with PCG64(seed) in cell order."""
    c = mesh_xyz[cells].mean(axis=1)
    if perturb:
        c = c + np.random.default_rng(seed).uniform(-perturb, perturb, size=c.shape) * h
    return c


def _orient_pyr(xyz, pn):
    """Reorder base corners so that (X1 - X0) x (X3 - X0) points at the apex (J > 0)."""
    c = xyz[pn]
    vol = np.einsum("ni,ni->n", np.cross(c[:, 1] - c[:, 0], c[:, 3] - c[:, 0]), c[:, 4] - c[:, 0])
    neg = vol < 0
    pn[neg] = pn[neg][:, [0, 3, 2, 1, 4]]
    return pn


def _orient_tet(xyz, tn):
    vol = _tet_signed_volume(xyz[tn])
    neg = vol < 0
    tn[neg] = tn[neg][:, [0, 2, 1, 3]]
    return tn


def _face_split_tets(cell, face_cyc, apex):
    """The pyramid (apex, cell face) cut into 2 tetrahedra along the face diagonal from
    its lowest to its highest corner: [2][4] vertex ids (orientation not yet fixed)."""
    ids = [cell[k] for k in face_cyc]
    # cyclic corners 0 and 2 are the (0,0) and (1,1) offsets in the face's axes
    lo_, a, hi_, b = ids
    return [[apex, lo_, a, hi_], [apex, lo_, b, hi_]]


def _assemble(xyz, blocks, period, meta, permute_seed):
    en, et = [], []
    for t, nodes in blocks:
        if len(nodes) == 0:
            continue
        e = np.full((len(nodes), 8), -1, dtype=np.int64)
        e[:, :nodes.shape[1]] = nodes
        en.append(e)
        et.append(np.full(len(nodes), t, dtype=np.int32))
    en, et = np.concatenate(en), np.concatenate(et)
    if permute_seed is not None:
        perm = np.random.default_rng(permute_seed).permutation(en.shape[0])
        en, et = en[perm], et[perm]
    return Mesh(xyz, et, en, period, meta)


def pyramid_box(n=(3, 3, 3), lo=(-math.pi,) * 3, hi=(math.pi,) * 3, apex_perturb=0.0,
                perturb_seed=None, permute_seed=None, rotate_seed=None) -> Mesh:
    """Periodic box with each of the nx*ny*nz cells cut into 6 pyramids (one per face).

    The apex of a cell's pyramids is its centre moved by U(-apex_perturb, apex_perturb) * h
    per coordinate, drawn with PCG64(perturb_seed) in C order of the cells [k][j][i];
    the lattice itself is not perturbed, so every base is an exact parallelogram.
    rotate_seed: if given, each pyramid's base corners are shifted cyclically by
    PCG64(rotate_seed).integers(0, 4) places (orientation kept), so that neighbouring
    faces meet in every relative orientation.
    """
    hx = hex_box(n, lo, hi)
    cells = hx.enodes[:, :8]
    cen = _cell_centres(hx.xyz, cells, hx.meta["h"], apex_perturb, perturb_seed)
    xyz = np.concatenate([hx.xyz, cen])
    apex = hx.xyz.shape[0] + np.arange(cells.shape[0])
    pn = np.concatenate([np.column_stack([cells[:, cyc], apex]) for _, _, cyc in _CELL_FACES])
    pn = _orient_pyr(xyz, pn)
    if rotate_seed is not None:
        k = np.random.default_rng(rotate_seed).integers(0, 4, size=pn.shape[0])
        idx = (np.arange(4)[None, :] + k[:, None]) % 4
        pn[:, :4] = np.take_along_axis(pn[:, :4], idx, axis=1)
    return _assemble(xyz, [(PYR, pn)], hx.period.copy(),
                     {"n": tuple(n), "h": hx.meta["h"], "kind": "pyramid_box"}, permute_seed)


def transition_box(n=(4, 2, 2), n_hex=None, lo=(-math.pi,) * 3, hi=(math.pi,) * 3,
                   apex_perturb=0.0, perturb_seed=None, permute_seed=None) -> Mesh:
    """Conforming periodic box of hexahedra, pyramids and tetrahedra (see module notes).

    Cell column i along x: i < n_hex hexahedra (default nx // 2); i = n_hex and
    i = nx - 1 transition cells (1 pyramid on the face toward the hexahedra + 10
    tetrahedra); the columns between them Kuhn-split (6 tetrahedra each).  Requires
    nx >= n_hex + 2.  Apex displacement as in ``pyramid_box``, in cell order
    [k][j][i] over the transition cells only.
    """
    n = tuple(int(v) for v in n)
    nx, ny, nz = n
    n_hex = nx // 2 if n_hex is None else int(n_hex)
    if n_hex < 1 or nx < n_hex + 2:
        raise ValueError("transition_box needs 1 <= n_hex <= nx - 2")
    hx = hex_box(n, lo, hi)
    cells = hx.enodes[:, :8]                       # C order [k][j][i]
    ci = np.arange(cells.shape[0]) % nx
    hexes = cells[ci < n_hex]
    kuhn = kuhn_split(Mesh(hx.xyz, np.full(int(np.sum((ci > n_hex) & (ci < nx - 1))), HEX, np.int32),
                           cells[(ci > n_hex) & (ci < nx - 1)], hx.period))
    tets = [kuhn.enodes[:, :4]] if kuhn.n_elem else []
    trans = np.nonzero((ci == n_hex) | (ci == nx - 1))[0]
    cen = _cell_centres(hx.xyz, cells[trans], hx.meta["h"], apex_perturb, perturb_seed)
    xyz = np.concatenate([hx.xyz, cen])
    pyrs, extra = [], []
    for t_, c in enumerate(trans):
        cell, apex = cells[c], hx.xyz.shape[0] + t_
        base_side = 0 if ci[c] == n_hex else 1       # pyramid on the x face toward the hexahedra
        for ax, side, cyc in _CELL_FACES:
            if ax == 0 and side == base_side:
                pyrs.append([cell[k] for k in cyc] + [apex])
            else:
                extra.extend(_face_split_tets(cell, cyc, apex))
    tets.append(np.array(extra, dtype=np.int64))
    tn = _orient_tet(xyz, np.concatenate(tets).astype(np.int64))
    pn = _orient_pyr(xyz, np.array(pyrs, dtype=np.int64))
    return _assemble(xyz, [(HEX, hexes), (PYR, pn), (TET, tn)], hx.period.copy(),
                     {"n": n, "n_hex": n_hex, "h": hx.meta["h"], "kind": "transition_box"},
                     permute_seed)


def concat(meshes, permute_seed=None) -> Mesh:
    """Several meshes in one element list (they must not share faces)."""
    xyz, en, et = [], [], []
    off = 0
    for m in meshes:
        xyz.append(m.xyz)
        e = m.enodes.copy()
        e[e >= 0] += off
        en.append(e)
        et.append(m.etype)
        off += m.xyz.shape[0]
    en = np.concatenate(en)
    et = np.concatenate(et)
    if permute_seed is not None:
        perm = np.random.default_rng(permute_seed).permutation(en.shape[0])
        en, et = en[perm], et[perm]
    return Mesh(np.concatenate(xyz), et, en, meshes[0].period.copy(), {"kind": "concat"})


# ----------------------------------------------------------------------------------
# Initial conditions.  All take physical coordinates x,y,z (any equal shapes) and
# return conservative variables stacked on a new leading axis of length 5:
# (rho, rho*u, rho*v, rho*w, E).
# ----------------------------------------------------------------------------------

def prim_to_cons(rho, u, v, w, p, gamma=1.4):
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, E])


def tgv(x, y, z, mach=0.1, gamma=1.4):
    """Taylor--Green vortex with unit velocity/length/density scales, p0 = 1/(gamma Ma^2)."""
    p0 = 1.0 / (gamma * mach * mach)
    u = np.sin(x) * np.cos(y) * np.cos(z)
    v = -np.cos(x) * np.sin(y) * np.cos(z)
    w = np.zeros_like(u)
    p = p0 + (np.cos(2 * x) + np.cos(2 * y)) * (2.0 + np.cos(2 * z)) / 16.0
    rho = p / p0
    return prim_to_cons(rho, u, v, w, p, gamma)


SHOCK_MACH = 3.0


def shock_normal(seed=41):
    v = np.random.default_rng(seed).normal(size=3)
    return v / np.linalg.norm(v)


def shock_states(gamma=1.4, ms=SHOCK_MACH):
    """Pre/post states of a normal shock moving into gas at rest (rho=1, p=1)."""
    g = gamma
    r2 = (g + 1) * ms * ms / ((g - 1) * ms * ms + 2)
    p2 = 1.0 + 2 * g / (g + 1) * (ms * ms - 1)
    c1 = math.sqrt(g)
    u2 = ms * c1 * (1.0 - 1.0 / r2)
    return (1.0, 1.0), (r2, p2, u2)


def shock(x, y, z, gamma=1.4, orient_seed=41, noise_seed=42, noise=0.05):
    """Planar Mach-3 shock through the origin at a seeded orientation.

    Upstream (n.x > 0): rho = 1 + noise*U(-1,1) i.i.d. per point (PCG64(noise_seed),
    drawn in the C order of the coordinate arrays), v = 0, p = 1.
    Downstream: Rankine--Hugoniot state moving along n.
    """
    nvec = shock_normal(orient_seed)
    s = nvec[0] * x + nvec[1] * y + nvec[2] * z
    (_, _), (r2, p2, u2) = shock_states(gamma)
    rng = np.random.default_rng(noise_seed)
    rho1 = 1.0 + noise * rng.uniform(-1.0, 1.0, size=np.shape(x))
    pre = s > 0
    rho = np.where(pre, rho1, r2)
    p = np.where(pre, 1.0, p2)
    vel = np.where(pre, 0.0, u2)
    return prim_to_cons(rho, vel * nvec[0], vel * nvec[1], vel * nvec[2], p, gamma)


def isentropic_vortex(x, y, z, t=0.0, eps=5.0, u0=1.0, v0=0.0, gamma=1.4, period=20.0):
    """Shu's isentropic vortex centred at the origin, convected by (u0, v0) for time t.

    The nearest periodic image (period in x and y) of the vortex centre is used.
    """
    xc = u0 * t
    yc = v0 * t
    dx = x - xc
    dy = y - yc
    dx = dx - period * np.round(dx / period)
    dy = dy - period * np.round(dy / period)
    r2 = dx * dx + dy * dy
    f = np.exp(0.5 * (1.0 - r2))
    du = -eps / (2 * math.pi) * f * dy
    dv = eps / (2 * math.pi) * f * dx
    T = 1.0 - (gamma - 1.0) * eps * eps / (8 * gamma * math.pi * math.pi) * f * f
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho ** gamma
    return prim_to_cons(rho, u0 + du, v0 + dv, np.zeros_like(x), p, gamma)


def random_state(shape, seed, rho0=1.0, p0=1.0, vel=0.5, amp=0.1, gamma=1.4):
    """Seeded random positive state: rho, p = base*(1 + amp*U(-1,1)), velocity U(-vel, vel)."""
    rng = np.random.default_rng(seed)
    rho = rho0 * (1.0 + amp * rng.uniform(-1, 1, size=shape))
    u = vel * rng.uniform(-1, 1, size=shape)
    v = vel * rng.uniform(-1, 1, size=shape)
    w = vel * rng.uniform(-1, 1, size=shape)
    p = p0 * (1.0 + amp * rng.uniform(-1, 1, size=shape))
    return prim_to_cons(rho, u, v, w, p, gamma)


# ----------------------------------------------------------------- learned warm start
MLP_SHAPES = ((64, 16), (64,), (64, 64), (64,), (64,), (1,))   # W1 b1 W2 b2 w3 b3, flat in this order


def mlp_glorot(seed=43):
    """Initial MLP parameters (flat FP32, 5,313): Glorot-uniform weights drawn from
    PCG64(seed) in the order W1, W2, w3; zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape, fan in zip(MLP_SHAPES, ((16, 64), None, (64, 64), None, (64, 1), None)):
        if fan is None:
            parts.append(np.zeros(shape))
        else:
            a = math.sqrt(6.0 / (fan[0] + fan[1]))
            parts.append(rng.uniform(-a, a, size=shape))
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def minibatch_rows(n, batch, steps, seed=44):
    """Row ids of `steps` minibatches (flat int32): epochs of PCG64(seed) permutations,
    a batch never straddling two epochs."""
    rng = np.random.default_rng(seed)
    out, perm, pos = [], rng.permutation(n), 0
    for _ in range(steps):
        if pos + batch > n:
            perm, pos = rng.permutation(n), 0
        out.append(perm[pos:pos + batch])
        pos += batch
    return np.concatenate(out).astype(np.int32)
