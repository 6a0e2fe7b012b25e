"""Write pyr24_p4_ns_tgv_samples.txt: the FP64 oracle's right-hand side at sampled
elements of the full-size pyramid workload.

Workload (82,944 elements, 4.56 M points): 24^3 cells on [-pi, pi]^3, each cut into the 6
pyramids on its faces around an apex at the cell centre moved by U(-0.1, 0.1) h per
coordinate (seed 61), elements permuted (seed 62); p = 4 (55 solution points per pyramid);
compressible Navier--Stokes (LDG, beta = 1/2, tau = 0.1, mu = 1/1600, Pr = 0.71) with the
Rusanov inviscid flux; the Taylor--Green vortex at Mach 0.1 as the state.

The oracle is evaluated on the block cut down to the two face-neighbour rings of 32
sampled elements (oracle_subset.py: the same functions on fewer elements).  Also stored:
the FP64 rounding floor of the samples (relative L2 change of the oracle's values when the
state is perturbed by a relative U(-1, 1) 2^-53).  Element ids are canonical ones: the
order of the elements in the permuted mesh.

Usage: python tests/golden/make_pyr24_p4_samples.py   (from the repository root)
"""
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

N, ORDER, MACH = (24, 24, 24), 4, 0.1
APEX, APEX_SEED, PERMUTE_SEED = 0.1, 61, 62
SAMPLE_SEED, N_SAMPLES = 63, 32
OUT = os.path.join(HERE, "pyr24_p4_ns_tgv_samples.txt")


def main():
    mesh = inputs.pyramid_box(N, apex_perturb=APEX, perturb_seed=APEX_SEED, permute_seed=PERMUTE_SEED)
    canon = np.sort(np.random.default_rng(SAMPLE_SEED).choice(mesh.n_elem, N_SAMPLES, replace=False))
    bl = omesh.build(mesh, ORDER)
    keep = osub.rings(bl, [canon], 2)
    sb = osub.restrict(bl, keep)
    del bl
    x = sb[0].xsol
    u = [np.moveaxis(inputs.tgv(x[..., 0], x[..., 1], x[..., 2], mach=MACH), 0, 1).copy()]
    prm = ofr.Params(system=1, riemann=0)
    pos = np.searchsorted(keep[0], canon)
    R = ofr.rhs(sb, u, prm)[0][pos].copy()
    rng = np.random.default_rng(0)
    up = [u[0] * (1 + 2.0 ** -53 * rng.uniform(-1, 1, size=u[0].shape))]
    floor = float(np.linalg.norm(ofr.rhs(sb, up, prm)[0][pos] - R) / np.linalg.norm(R))
    print(f"{N_SAMPLES} samples, {keep[0].size} elements evaluated, floor {floor:.3e}", flush=True)
    with open(OUT, "w") as fh:
        fh.write("# FP64 oracle right-hand side at sampled elements; written by make_pyr24_p4_samples.py\n")
        fh.write(f"# pyramid box of {N} cells x 6, apex moved by {APEX} h (seed {APEX_SEED}), permuted (seed {PERMUTE_SEED})\n")
        fh.write(f"# order {ORDER}, Navier-Stokes, Rusanov, TGV Mach {MACH} at the solution points\n")
        fh.write("# layout: 'floor <value>', then 'pyr <canonical id>' followed by 5 rows (variables) of 55 values\n")
        fh.write(f"floor {floor:.6e}\n")
        for i, e in enumerate(canon):
            fh.write(f"pyr {int(e)}\n")
            for v in range(5):
                fh.write(" ".join(f"{val:.17e}" for val in R[i, v]) + "\n")
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
