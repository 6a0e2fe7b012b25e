"""Shared helpers of the GPU parity tests: build both sides from the same seeded inputs."""
import numpy as np

from oracle import fr as ofr
from oracle import mesh as omesh
from paper_2408_16509_amd import inputs


def oracle_blocks(mesh, order):
    return omesh.build(mesh, order)


def state_for(blocks, kind, seed=1, mach=0.1):
    """Per-block canonical states [n][5][nsp] at the oracle's solution points."""
    out = []
    for i, b in enumerate(blocks):
        x = b.xsol
        if kind == "random":
            s = inputs.random_state(x.shape[:2], seed + i)
        elif kind == "tgv":
            s = inputs.tgv(x[..., 0], x[..., 1], x[..., 2], mach=mach)
        elif kind == "shock":
            s = inputs.shock(x[..., 0], x[..., 1], x[..., 2])
        else:
            raise ValueError(kind)
        out.append(np.moveaxis(s, 0, 1).copy())
    return out


def oracle_params(system=0, riemann=0, **kw):
    return ofr.Params(system=system, riemann=riemann, **kw)


def rel_err(a, b):
    """(global relative L2, per-variable relative L2 [5]) of a vs reference b, [n][5][nsp] blocks."""
    num = sum(np.sum((x - y) ** 2) for x, y in zip(a, b))
    den = sum(np.sum(y ** 2) for y in b)
    pv_num = sum(np.sum((x - y) ** 2, axis=(0, 2)) for x, y in zip(a, b))
    pv_den = sum(np.sum(y ** 2, axis=(0, 2)) for y in b)
    return float(np.sqrt(num / den)), np.sqrt(pv_num / np.maximum(pv_den, 1e-300))


def elem_max_err(a, b):
    """Largest per-element error of a against reference b ([n][5][nsp] blocks): the L2 norm of
    the element's error over its points and variables, divided by the larger of the element's
    own reference norm and the root-mean-square element norm (so that elements whose residual
    happens to be near zero are measured on the field's scale, not their own)."""
    num = np.concatenate([np.sqrt(np.sum((x - y) ** 2, axis=(1, 2))) for x, y in zip(a, b)])
    den = np.concatenate([np.sqrt(np.sum(y ** 2, axis=(1, 2))) for y in b])
    rms = np.sqrt(np.mean(den ** 2))
    return float(np.max(num / np.maximum(den, rms)))


# Per-element bound, as a multiple of the global relative-L2 tolerance: rounding noise spread
# over the field puts each element near the global figure; a wrong element stands far above.
ELEM_FACTOR = 20.0


def oracle_floor(mesh, order, u_blocks, prm, seed=0):
    """The FP64 rounding floor of the RHS for this input: relative L2 change of the
    oracle's RHS when every state value is perturbed by a relative U(-1,1) * 2^-53
    (one rounding of the input).  Any FP64 evaluation rounds intermediates at that
    level, so no implementation can be asked to agree more closely.  For random
    states the floor is ~4e-16; for the low-Mach Taylor--Green vortex it is
    ~1e-12 (4^3, p=3) and grows with resolution, because the O(1/Ma^2) pressure
    and energy enter residuals that are O(1).  Returns (floor, oracle RHS)."""
    bl = omesh.build(mesh, order)
    R = ofr.rhs(bl, u_blocks, prm)
    rng = np.random.default_rng(seed)
    up = [x * (1 + 2.0 ** -53 * rng.uniform(-1, 1, size=x.shape)) for x in u_blocks]
    Rp = ofr.rhs(bl, up, prm)
    return rel_err(Rp, R)[0], R
