"""The oracle's pins catch plausible mistakes: each case plants one mistake in a copy of
the oracle's FR module (on the CPU, never in the product) and checks that the
brute-force nodal DG pin then fails, while the unmodified module passes it.

Planted mistakes: the sign of beta in the LDG common solution, the viscous common flux
taken from the other side, the sign of the LDG penalty, the sign of the viscous flux,
the sign of the correction (jump) term, and the left/right slot of the common flux.
"""
import os
import sys
import types

import numpy as np
import pytest

import oracle
from oracle import fr, mesh, nodal_dg
from paper_2408_16509_amd import inputs

SRC = os.path.join(os.path.dirname(oracle.__file__), "fr.py")

MUTATIONS = {
    "beta sign in the common solution": ("+ prm.ldg_beta * (uL - uR)", "- prm.ldg_beta * (uL - uR)"),
    "viscous common flux from the other side": ("- beta * (fvL - fvR)", "+ beta * (fvL - fvR)"),
    "penalty sign": ("+ prm.ldg_tau * (uL - uR)", "- prm.ldg_tau * (uL - uR)"),
    "viscous flux sign": ("f = f - physics.viscous_flux", "f = f + physics.viscous_flux"),
    "jump sign": ("_apply(ops.lift, Fc - fperp)", "_apply(ops.lift, fperp - Fc)"),
    "common flux slot": ("return mag * sgn * F", "return mag * F"),
}


def _mutant(old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, old
    mod = types.ModuleType("oracle._fr_mutant")
    mod.__package__ = "oracle"
    sys.modules[mod.__name__] = mod          # dataclasses look their module up there
    try:
        exec(compile(src.replace(old, new), SRC + " (mutated)", "exec"), mod.__dict__)
    finally:
        del sys.modules[mod.__name__]
    return mod


def _mismatch(frmod, kind, beta):
    m = inputs.hex_box((2, 1, 1)) if kind == "hex" else inputs.kuhn_split(inputs.hex_box((1, 1, 1)))
    bl = mesh.build(m, 3 if kind == "hex" else 4)
    prm = fr.Params(system=1, riemann=0, mu=0.05, ldg_beta=beta, ldg_tau=0.5)
    u = [np.moveaxis(inputs.random_state(b.xsol.shape[:2], 7), 0, 1).copy() for b in bl]
    a = frmod.rhs(bl, u, frmod.Params(**vars(prm)))[0]
    d = nodal_dg.rhs(bl, u, prm)[0]
    return np.linalg.norm(a - d) / np.linalg.norm(d)


@pytest.mark.parametrize("kind", ["hex", "tet"])
def test_unmodified_oracle_passes(kind):
    assert _mismatch(fr, kind, 0.5) < 1e-13


@pytest.mark.parametrize("name", list(MUTATIONS))
@pytest.mark.parametrize("kind", ["hex", "tet"])
def test_planted_mistake_fails_the_nodal_dg_pin(name, kind):
    mut = _mutant(*MUTATIONS[name])
    for beta in (0.5, 0.3):
        assert _mismatch(mut, kind, beta) > 1e-6, (name, beta)
