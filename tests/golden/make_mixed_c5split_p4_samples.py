"""Write mixed_c5split_p4_ns_tgv_samples.txt: the FP64 oracle's right-hand side at
sampled elements of the full-size mixed hexahedral + tetrahedral workload.

Workload (917,504 elements, 43.9 M points): two periodic boxes of 32 x 64 x 64 cells,
every vertex coordinate moved by U(-0.1, 0.1) h (seed 51): box A on [-pi, pi]^3 kept as
131,072 p = 4 hexahedra (125 Gauss--Legendre points each), box B on [3, 3 + 2 pi] x
[-pi, pi]^2 cut into 786,432 p = 4 tetrahedra (6 per cell, the 35 points of Fig. mesh),
the two element lists concatenated and permuted (seed 53); compressible Navier--Stokes
(LDG, beta = 1/2, tau = 0.1, mu = 1/1600, Pr = 0.71) with the Rusanov inviscid flux; the
Taylor--Green vortex at Mach 0.1 as the state.  The boxes share no face, so each is its
own periodic mesh for the oracle.

The oracle is evaluated on the type block cut down to the two face-neighbour rings of the
sampled elements (oracle_subset.py: the same functions on fewer elements), for 32
sampled hexahedra and 32 sampled tetrahedra.  Also stored per element type: the FP64
rounding floor of the samples (relative L2 change of the oracle's values when the state
is perturbed by a relative U(-1, 1) 2^-53).

Element ids are canonical ones of the library's layout: per type block (hexahedra, then
tetrahedra), elements in the order they appear in the permuted mesh.

Usage: python tests/golden/make_mixed_c5split_p4_samples.py   (from the repository root)
"""
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import oracle_subset as osub           # noqa: E402
from oracle import fr as ofr          # noqa: E402
from oracle import mesh as omesh      # noqa: E402
from paper_2408_16509_amd import inputs  # noqa: E402

N, ORDER, MACH = (32, 64, 64), 4, 0.1
PERTURB, PERTURB_SEED, PERMUTE_SEED = 0.1, 51, 53
SAMPLE_SEED, N_SAMPLES = 54, 32
OUT = os.path.join(HERE, "mixed_c5split_p4_ns_tgv_samples.txt")


def boxes():
    lo_b = (3.0, -math.pi, -math.pi)
    hi_b = tuple(v + 2 * math.pi for v in lo_b)
    a = inputs.hex_box(N, perturb=PERTURB, perturb_seed=PERTURB_SEED)
    b = inputs.kuhn_split(inputs.hex_box(N, lo=lo_b, hi=hi_b, perturb=PERTURB, perturb_seed=PERTURB_SEED))
    return a, b


def canonical_to_box(n_a, n_b):
    """For each element type, the box-local index of each canonical element."""
    perm = np.random.default_rng(PERMUTE_SEED).permutation(n_a + n_b)   # as inputs.concat draws it
    hexes = perm[perm < n_a]
    tets = perm[perm >= n_a] - n_a
    return hexes, tets


def sample_block(box_mesh, local_ids):
    bl = omesh.build(box_mesh, ORDER)
    keep = osub.rings(bl, [local_ids], 2)
    sb = osub.restrict(bl, keep)
    del bl
    x = sb[0].xsol
    u = [np.moveaxis(inputs.tgv(x[..., 0], x[..., 1], x[..., 2], mach=MACH), 0, 1).copy()]
    prm = ofr.Params(system=1, riemann=0)
    pos = np.searchsorted(keep[0], local_ids)
    R = ofr.rhs(sb, u, prm)[0][pos].copy()
    rng = np.random.default_rng(0)
    up = [u[0] * (1 + 2.0 ** -53 * rng.uniform(-1, 1, size=u[0].shape))]
    Rp = ofr.rhs(sb, up, prm)[0][pos]
    return R, float(np.linalg.norm(Rp - R) / np.linalg.norm(R)), int(keep[0].size)


def main():
    a, b = boxes()
    hexes, tets = canonical_to_box(a.n_elem, b.n_elem)
    rng = np.random.default_rng(SAMPLE_SEED)
    res = {}
    for name, box, local_of in (("hex", a, hexes), ("tet", b, tets)):
        canon = np.sort(rng.choice(len(local_of), N_SAMPLES, replace=False))
        R, floor, kept = sample_block(box, local_of[canon])
        res[name] = (canon, R, floor)
        print(f"{name}: {N_SAMPLES} samples, {kept} elements evaluated, floor {floor:.3e}", flush=True)
    with open(OUT, "w") as fh:
        fh.write("# FP64 oracle right-hand side at sampled elements; written by make_mixed_c5split_p4_samples.py\n")
        fh.write(f"# two boxes of {N} cells, perturb={PERTURB} seed={PERTURB_SEED}, box B Kuhn-split, "
                 f"concatenated and permuted with seed {PERMUTE_SEED}\n")
        fh.write(f"# order {ORDER}, Navier-Stokes, Rusanov, TGV Mach {MACH} at the solution points\n")
        fh.write("# layout: 'floor <type> <value>' lines, then '<type> <canonical id within the type block>'\n")
        fh.write("# followed by 5 rows (variables) of the element's solution points\n")
        for name in ("hex", "tet"):
            fh.write(f"floor {name} {res[name][2]:.6e}\n")
        for name in ("hex", "tet"):
            canon, R, _ = res[name]
            for i, e in enumerate(canon):
                fh.write(f"{name} {int(e)}\n")
                for v in range(5):
                    fh.write(" ".join(f"{val:.17e}" for val in R[i, v]) + "\n")
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
