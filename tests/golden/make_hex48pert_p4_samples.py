"""Write hex48pert_p4_ns_tgv_samples.txt: the FP64 oracle's right-hand side at sampled
elements of the full-size perturbed, permuted hexahedral workload.

Workload: periodic [-pi, pi]^3 box of 48^3 hexahedra, every vertex coordinate moved by
U(-0.1, 0.1) h (seed 31), elements in random order (seed 32); p = 4 (125 Gauss--Legendre
points per element); compressible Navier--Stokes (LDG, beta = 1/2, tau = 0.1, mu = 1/1600,
Pr = 0.71) with the Rusanov inviscid flux; Taylor--Green vortex at Mach 0.1 as the state
(Sec. "Taylor--Green vortex": rho = p / p0, p0 = 1 / (gamma Ma^2)).

Only oracle/ and the seeded input generator are used.  The oracle needs about two minutes
and 35 GB of host memory per right-hand side at this size, which is why its values are
stored for a sample of elements.  Also stored: the FP64 rounding floor of those samples
(relative L2 change of the oracle's values when the state is perturbed by a relative
U(-1, 1) 2^-53, the test's tolerance unit).

Usage: python tests/golden/make_hex48pert_p4_samples.py   (from the repository root)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import fr as ofr          # noqa: E402
from oracle import mesh as omesh      # noqa: E402
from paper_2408_16509_amd import inputs  # noqa: E402

N, ORDER, MACH = 48, 4, 0.1
PERTURB, PERTURB_SEED, PERMUTE_SEED = 0.1, 31, 32
SAMPLE_SEED, N_SAMPLES = 33, 24
OUT = os.path.join(HERE, "hex48pert_p4_ns_tgv_samples.txt")


def main():
    mesh = inputs.hex_box((N, N, N), perturb=PERTURB, perturb_seed=PERTURB_SEED, permute_seed=PERMUTE_SEED)
    bl = omesh.build(mesh, ORDER)
    x = bl[0].xsol
    u = [np.moveaxis(inputs.tgv(x[..., 0], x[..., 1], x[..., 2], mach=MACH), 0, 1).copy()]
    prm = ofr.Params(system=1, riemann=0)
    E = u[0].shape[0]
    elems = np.sort(np.random.default_rng(SAMPLE_SEED).choice(E, N_SAMPLES, replace=False))
    R = ofr.rhs(bl, u, prm)[0][elems].copy()
    rng = np.random.default_rng(0)
    up = [u[0] * (1 + 2.0 ** -53 * rng.uniform(-1, 1, size=u[0].shape))]
    Rp = ofr.rhs(bl, up, prm)[0][elems]
    floor = float(np.linalg.norm(Rp - R) / np.linalg.norm(R))
    with open(OUT, "w") as fh:
        fh.write("# FP64 oracle right-hand side at sampled elements; written by make_hex48pert_p4_samples.py\n")
        fh.write(f"# mesh hex_box n={N} perturb={PERTURB} perturb_seed={PERTURB_SEED} permute_seed={PERMUTE_SEED}\n")
        fh.write(f"# order {ORDER}, Navier-Stokes, Rusanov, TGV Mach {MACH} at the solution points\n")
        fh.write("# layout: 'elem <id>' then 5 rows (variables) of the element's solution points\n")
        fh.write(f"floor {floor:.6e}\n")
        for i, e in enumerate(elems):
            fh.write(f"elem {int(e)}\n")
            for v in range(5):
                fh.write(" ".join(f"{val:.17e}" for val in R[i, v]) + "\n")
    print(f"wrote {OUT}: {len(elems)} elements, floor {floor:.3e}")


if __name__ == "__main__":
    main()
