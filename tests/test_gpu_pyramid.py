"""GPU parity of p = 4 pyramids (meshes of pyramids with affine bases) against the FP64
oracle, element by element: fr_rhs for Euler (Rusanov, HLLC) and Navier--Stokes (LDG,
beta = 1/2, -1/2, 0.3), FP64 and the FP32 deviation form, fr_rk_step, the solution
points, and the options a pyramid context refuses.

Tolerances: FP64 relative L2 <= max(1e-12, 8 x the oracle's rounding floor for that
input), per variable and per element as in test_gpu_rhs; FP32 deviation form 1e-5 on
well-conditioned states.  The floor measures the response to a one-ulp perturbation of
the input; the pyramid's dense 55-term products have larger operator norms than the
other types' (interpolation Lebesgue constant near 20 at the triangle flux points,
where a tetrahedron's flux points are its solution points), so the rounding of the
intermediate traces and fluxes of two different evaluation orders differs by a few
times that response: measured 4.5x on the low-Mach Taylor--Green vortex (Navier--Stokes),
hence twice the factor 4 of the hexahedral and tetrahedral tests.  States: small
random perturbations of a state at rest (velocity U(-0.1, 0.1), density and pressure
1 +- 2 %: the layered pyramid points interpolate to the triangle flux points with a
Lebesgue constant near 20, so larger point-wise noise can leave the admissible set
there) and the Taylor--Green vortex.
"""
import numpy as np
import pytest

from oracle import fr as ofr
from oracle import rk as ork
from paper_2408_16509_amd import inputs

from helpers import ELEM_FACTOR, elem_max_err, oracle_blocks, oracle_floor, oracle_params, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

UREF_RANDOM = (1.0, 0.0, 0.0, 0.0, 1.0 / 0.4)
FLOOR_FACTOR = 8.0

MESHES = {
    # 48 elements: one ragged 64-element tile
    "pyr222": lambda: inputs.pyramid_box((2, 2, 2)),
    # 108 elements, apexes moved by up to 15 % of a cell, element order permuted
    "pyrpert": lambda: inputs.pyramid_box((3, 3, 2), apex_perturb=0.15, perturb_seed=3, permute_seed=4),
    # the same with every base's corners shifted cyclically at random: faces meet in five
    # relative orientations (two above), which exercises the face-point permutations
    "pyrrot": lambda: inputs.pyramid_box((3, 3, 2), apex_perturb=0.15, perturb_seed=3, permute_seed=4,
                                         rotate_seed=5),
}


def _state(bl, kind, seed=3):
    out = []
    for i, b in enumerate(bl):
        x = b.xsol
        if kind == "random":
            s = inputs.random_state(x.shape[:2], seed + i, vel=0.1, amp=0.02)
        else:
            s = inputs.tgv(x[..., 0], x[..., 1], x[..., 2], mach=0.1)
        out.append(np.moveaxis(s, 0, 1).copy())
    return out


def _split(flat, like):
    out, o = [], 0
    for b in like:
        out.append(flat[o:o + b.size].reshape(b.shape))
        o += b.size
    return out


def _rhs(mesh, u_blocks, **kw):
    from paper_2408_16509_amd import frmi
    ctx = frmi.Context(mesh, order=4, **kw)
    u = ctx.pack(ctx.join_canon(u_blocks))
    r = ctx.new_native()
    ctx.rhs(u, r)
    out = ctx.unpack_rhs(r).cpu().numpy()
    ctx.close()
    return _split(out, u_blocks)


def _check(Rg, Ro, tol):
    g, pv = rel_err(Rg, Ro)
    glob = np.sqrt(sum(np.sum(y ** 2) for y in Ro))
    pv_abs = np.sqrt(sum(np.sum((x - y) ** 2, axis=(0, 2)) for x, y in zip(Rg, Ro)))
    pv_ref = np.sqrt(sum(np.sum(y ** 2, axis=(0, 2)) for y in Ro))
    floor = np.maximum(pv_ref, 1e-3 * glob)
    em = elem_max_err(Rg, Ro)
    print(f"tol {tol:.2e} global rel L2 {g:.3e}  per-var {np.array2string(pv_abs / floor, precision=2)}  "
          f"max per element {em:.2e}", flush=True)
    assert g <= tol
    assert np.all(pv_abs <= 10 * tol * floor)
    assert em <= ELEM_FACTOR * tol


def test_solution_points_follow_the_reference_order():
    from paper_2408_16509_amd import frmi
    mesh = MESHES["pyrpert"]()
    bl = oracle_blocks(mesh, 4)
    ctx = frmi.Context(mesh, order=4)
    x = ctx.sol_points().reshape(-1, 55, 3)
    ctx.close()
    assert np.abs(x - bl[0].xsol).max() <= 1e-13


CASES = [
    ("pyr222", 0, 0, "random"),
    ("pyrpert", 0, 0, "random"),
    ("pyrpert", 0, 1, "random"),
    ("pyrpert", 1, 0, "random"),
    ("pyrpert", 1, 1, "random"),
    ("pyr222", 1, 0, "tgv"),
    ("pyrpert", 0, 1, "tgv"),
    ("pyrrot", 0, 1, "random"),
    ("pyrrot", 1, 0, "random"),
    ("pyrrot", 1, 1, "tgv"),
]


@pytest.mark.parametrize("mname,system,riemann,state", CASES)
def test_rhs_parity_fp64(mname, system, riemann, state):
    print(f"case pyramids {mname} system={system} riemann={riemann} state={state}", flush=True)
    mesh = MESHES[mname]()
    bl = oracle_blocks(mesh, 4)
    u = _state(bl, state)
    fl, Ro = oracle_floor(mesh, 4, u, oracle_params(system, riemann))
    Rg = _rhs(mesh, u, system=system, riemann=riemann)
    _check(Rg, Ro, max(1e-12, FLOOR_FACTOR * fl))


@pytest.mark.parametrize("beta", [-0.5, 0.3])
def test_rhs_parity_ldg_beta(beta):
    print(f"case pyramids NS beta={beta}", flush=True)
    mesh = MESHES["pyrpert"]()
    bl = oracle_blocks(mesh, 4)
    u = _state(bl, "random")
    fl, Ro = oracle_floor(mesh, 4, u, oracle_params(1, 0, ldg_beta=beta))
    Rg = _rhs(mesh, u, system=1, riemann=0, ldg_beta=beta)
    _check(Rg, Ro, max(1e-12, FLOOR_FACTOR * fl))


@pytest.mark.parametrize("system,riemann", [(0, 0), (0, 1), (1, 0)])
def test_rhs_parity_fp32(system, riemann):
    from paper_2408_16509_amd import frmi
    print(f"case pyramids fp32 system={system} riemann={riemann}", flush=True)
    mesh = MESHES["pyrpert"]()
    bl = oracle_blocks(mesh, 4)
    u = _state(bl, "random")
    Ro = ofr.rhs(bl, u, oracle_params(system, riemann))
    Rg = _rhs(mesh, u, system=system, riemann=riemann, precision=frmi.FR_FP32, u_ref=UREF_RANDOM)
    g, pv = rel_err(Rg, Ro)
    print(f"fp32 pyramids: global {g:.2e} per-var {np.array2string(pv, precision=2)}", flush=True)
    assert g <= 1e-5


def test_uniform_state_is_steady():
    """Free stream: a uniform state's right-hand side is zero to rounding (FP64), and the
    FP32 deviation form returns exactly zero for its own reference state."""
    from paper_2408_16509_amd import frmi
    mesh = MESHES["pyrpert"]()
    bl = oracle_blocks(mesh, 4)
    const = np.array([1.1, 0.3, -0.2, 0.4, 3.0])
    u = [np.broadcast_to(const[None, :, None], (len(b.elems), 5, 55)).copy() for b in bl]
    for system in (0, 1):
        Rg = _rhs(mesh, u, system=system)
        assert max(np.abs(r).max() for r in Rg) < 1e-12 * 6 * 25
    ref = np.array(UREF_RANDOM)
    u = [np.broadcast_to(ref[None, :, None], (len(b.elems), 5, 55)).copy() for b in bl]
    Rg = _rhs(mesh, u, system=1, precision=frmi.FR_FP32, u_ref=UREF_RANDOM)
    assert max(np.abs(r).max() for r in Rg) == 0.0


def test_rk4_steps_parity():
    """Five RK4 steps (Navier--Stokes, HLLC, dt = 1e-3) through fr_rk_step against the
    oracle's RK4; the change of the state over the steps is compared."""
    from paper_2408_16509_amd import frmi
    mesh = MESHES["pyrpert"]()
    bl = oracle_blocks(mesh, 4)
    u = _state(bl, "random", seed=5)
    prm = oracle_params(1, 1)
    uo = ork.rk4(lambda s: ofr.rhs(bl, s, prm), u, 1e-3, 5)
    ctx = frmi.Context(mesh, order=4, system=1, riemann=1)
    ug = ctx.pack64(ctx.join_canon(u))
    ctx.rk_step(ug, 1e-3, 5)
    got = _split(ctx.unpack64(ug).cpu().numpy(), u)
    ctx.close()
    _check([g - a for g, a in zip(got, u)], [o - a for o, a in zip(uo, u)], 1e-11)


def test_refused_options():
    from paper_2408_16509_amd import frmi
    # pyramids joined to hexahedra and tetrahedra: not supported by the library
    with pytest.raises(frmi.FrError) as ei:
        frmi.Context(inputs.transition_box((4, 1, 1)), order=4)
    assert ei.value.status == 7 and "pyramids only" in str(ei.value)
    with pytest.raises(frmi.FrError) as ei:
        frmi.Context(MESHES["pyr222"](), order=3)
    assert ei.value.status == 7
    with pytest.raises(frmi.FrError) as ei:
        frmi.Context(MESHES["pyr222"](), order=4, precision=frmi.FR_FP32_BF16X3, u_ref=UREF_RANDOM)
    assert ei.value.status == 7
    mesh = MESHES["pyr222"]()
    bl = oracle_blocks(mesh, 4)
    u = _state(bl, "random")
    ctx = frmi.Context(mesh, order=4)
    ug = ctx.pack64(ctx.join_canon(u))
    with pytest.raises(frmi.FrError) as ei:
        ctx.rk_step(ug, 1e-3, 1, filter_mode=0)
    assert ei.value.status == 7 and "pyramid" in str(ei.value)
    with pytest.raises(frmi.FrError) as ei:
        ctx.filter(ug)
    assert ei.value.status == 7
    ctx.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_native_order_does_not_change_results(precision):
    """Input order, Morton renumbering and the automatic choice only move data: the
    canonical right-hand side of a permuted pyramid mesh with rotated bases is bit-identical."""
    from paper_2408_16509_amd import frmi
    mesh = inputs.pyramid_box((4, 3, 3), apex_perturb=0.1, perturb_seed=8, permute_seed=9, rotate_seed=10)
    kw = dict(system=1, order=4, riemann=0)
    if precision:
        kw.update(precision=frmi.FR_FP32, u_ref=UREF_RANDOM)
    out = []
    for order in (1, 2, 0):
        ctx = frmi.Context(mesh, elem_order=order, **kw)
        x = ctx.sol_points().reshape(-1, 55, 3)
        s = inputs.random_state(x.shape[:2], 11, vel=0.1, amp=0.02)
        u = ctx.pack(np.ascontiguousarray(np.moveaxis(s, 0, 1)).ravel())
        r = ctx.new_native()
        ctx.rhs(u, r)
        out.append(ctx.unpack_rhs(r).cpu().numpy())
        ctx.close()
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])
