"""The neighbourhood evaluation behind the stored full-size samples (tests/golden/
oracle_subset.py): the oracle's right-hand side on the type blocks cut down to the
sampled elements' face-neighbour rings equals its value on the whole mesh at the samples
(one ring for Euler, two for Navier--Stokes; one ring is not enough for Navier--Stokes,
which shows the ring count matters)."""
import os
import sys

import numpy as np
import pytest

from oracle import fr, mesh
from paper_2408_16509_amd import inputs

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
import oracle_subset as osub  # noqa: E402


@pytest.mark.parametrize("kind", ["hex", "tet"])
def test_rings_reproduce_the_whole_mesh(kind):
    if kind == "hex":
        m, p = inputs.hex_box((6, 6, 6), perturb=0.1, perturb_seed=3, permute_seed=4), 3
    else:
        m, p = inputs.kuhn_split(inputs.hex_box((4, 4, 4), perturb=0.1, perturb_seed=3), permute_seed=4), 4
    bl = mesh.build(m, p)
    u = [np.moveaxis(inputs.random_state(b.xsol.shape[:2], 5), 0, 1).copy() for b in bl]
    samp = np.random.default_rng(1).choice(len(bl[0].elems), 5, replace=False)
    for system, k, exact in ((0, 1, True), (1, 2, True), (1, 1, False)):
        prm = fr.Params(system=system, riemann=1)
        R = fr.rhs(bl, u, prm)[0][samp]
        keep = osub.rings(bl, [samp], k)
        assert keep[0].size < len(bl[0].elems)
        Rs = fr.rhs(osub.restrict(bl, keep), [u[0][keep[0]]], prm)[0][np.searchsorted(keep[0], samp)]
        err = np.abs(Rs - R).max() / np.abs(R).max()
        assert (err <= 1e-14) == exact, (system, k, err)
