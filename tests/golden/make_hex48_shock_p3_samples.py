"""Write hex48_shock_p3_samples.txt: the FP64 oracle's entropy filter, right-hand side and
one filtered RK4 step at sampled elements of the full-size Mach-3 shock workload.

Workload: periodic [-pi, pi]^3 box of 48^3 straight hexahedra, p = 3 (64 Gauss--Legendre
points each), compressible Euler with the HLLC flux; initial condition a planar Mach-3
shock at the seeded orientation (seed 41) over a density of 1 +- 5 % seeded noise
(seed 42), Rankine--Hugoniot post-shock state.  The interpolated discontinuous state is
not admissible at the flux points, so the plain entropy filter is applied to it first
(entropy bound from the state itself): u0 = filter(IC).  Stored at the samples (24
elements the filter treats and 8 it leaves alone, seed 43):
  * k: the dyadic filter strength index of each sample (0 untouched, -1 fallback);
  * u0, the filtered state;
  * R(u0), the right-hand side (one face-neighbour ring);
  * u1, one RK4 step of dt = 5e-4 from u0 with the plain filter on every stage state and
    on the new state, the entropy bound taken from u0 (evaluated on the samples' five
    face-neighbour rings: four right-hand sides and the filter's bound each reach one ring
    further; oracle_subset.py);
  * the FP64 rounding floor of R(u0) at the samples.
Only oracle/ and the seeded input generator are used.

Usage: python tests/golden/make_hex48_shock_p3_samples.py   (from the repository root)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import oracle_subset as osub              # noqa: E402
from oracle import entropy_filter as ef   # noqa: E402
from oracle import fr as ofr              # noqa: E402
from oracle import mesh as omesh          # noqa: E402
from oracle import rk as ork              # noqa: E402
from paper_2408_16509_amd import inputs   # noqa: E402

N, ORDER, DT = 48, 3, 5e-4
ORIENT_SEED, NOISE_SEED, SAMPLE_SEED = 41, 42, 43
N_TROUBLED, N_PLAIN = 24, 8
OUT = os.path.join(HERE, "hex48_shock_p3_samples.txt")


def main():
    mesh = inputs.hex_box((N, N, N))
    bl = omesh.build(mesh, ORDER)
    x = bl[0].xsol
    ic = np.moveaxis(inputs.shock(x[..., 0], x[..., 1], x[..., 2], orient_seed=ORIENT_SEED,
                                  noise_seed=NOISE_SEED), 0, 1).copy()
    fp = ef.FilterParams()
    un, kk, _ = ef.entropy_filter(bl, [ic], [ic], fp)
    u0, k0 = un[0], kk[0]
    rng = np.random.default_rng(SAMPLE_SEED)
    tr = np.nonzero(k0 != 0)[0]
    ok = np.nonzero(k0 == 0)[0]
    elems = np.sort(np.concatenate([rng.choice(tr, N_TROUBLED, replace=False),
                                    rng.choice(ok, N_PLAIN, replace=False)]))
    print(f"filter on the IC: {tr.size} troubled of {k0.size}", flush=True)
    prm = ofr.Params(system=0, riemann=1)
    # right-hand side and its rounding floor (one ring)
    keep = osub.rings(bl, [elems], 1)
    sb = osub.restrict(bl, keep)
    pos = np.searchsorted(keep[0], elems)
    us = u0[keep[0]]
    R = ofr.rhs(sb, [us], prm)[0][pos].copy()
    up = us * (1 + 2.0 ** -53 * np.random.default_rng(0).uniform(-1, 1, size=us.shape))
    Rp = ofr.rhs(sb, [up], prm)[0][pos]
    floor = float(np.linalg.norm(Rp - R) / np.linalg.norm(R))
    # one filtered RK4 step (five rings)
    keep5 = osub.rings(bl, [elems], 5)
    sb5 = osub.restrict(bl, keep5)
    pos5 = np.searchsorted(keep5[0], elems)
    u05 = [u0[keep5[0]]]
    smin0 = ef.smin_neighbourhood(sb5, u05, fp)
    post = lambda s: [ef.filter_block(b, ss, sm, fp)[0] for b, ss, sm in zip(sb5, s, smin0)]
    u1 = ork.rk4_step(lambda s: ofr.rhs(sb5, s, prm), u05, DT, stage_post=post)[0][pos5]
    print(f"RHS floor {floor:.3e}; {keep5[0].size} elements in the step's neighbourhood", flush=True)
    with open(OUT, "w") as fh:
        fh.write("# FP64 oracle at sampled elements of the 48^3 p=3 Mach-3 shock; written by "
                 "make_hex48_shock_p3_samples.py\n")
        fh.write(f"# hex_box n={N}, order {ORDER}, Euler, HLLC, shock orient_seed={ORIENT_SEED} "
                 f"noise_seed={NOISE_SEED}; u0 = plain entropy filter of the IC; dt {DT}\n")
        fh.write("# layout: 'elem <id> <k>' then 5 rows of u0, 5 rows of R(u0), 5 rows of u1 (one filtered RK4 step)\n")
        fh.write(f"floor {floor:.6e}\n")
        for i, e in enumerate(elems):
            fh.write(f"elem {int(e)} {int(k0[e])}\n")
            for arr in (u0[e], R[i], u1[i]):
                for v in range(5):
                    fh.write(" ".join(f"{val:.17e}" for val in arr[v]) + "\n")
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
