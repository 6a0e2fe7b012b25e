"""The FP32 deviation form (FP32 kernels on du = u - u_ref, FP64 RK accumulation)
against the FP64 oracle.

Stated bounds per RHS (relative L2 against the FP64 oracle):
  * well-conditioned states (random states around the reference state): 1e-5 overall;
  * the low-Mach (Ma 0.1) Taylor--Green vortex: 1e-3 overall, 1e-4 per momentum
    component and 1e-3 for density and energy.  There the density and energy
    residuals are O(Ma^2) differences of O(1/Ma^2) fluxes and the Rusanov
    dissipation scales with the O(1/Ma) sound speed, which multiplies the FP32
    rounding of the state (measured on 8^3, p = 3: rho 2.5e-4, momentum 3.4e-5,
    energy 4.2e-4).
The deviation form is exact for the reference state itself: R(u_ref) = 0 bit for bit.
"""
import numpy as np
import pytest

from oracle import fr as ofr
from oracle import rk as ork
from paper_2408_16509_amd import inputs

from helpers import oracle_blocks, oracle_params, rel_err, state_for

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

P0 = 1.0 / (1.4 * 0.01)
UREF = (1.0, 0.0, 0.0, 0.0, P0 / 0.4)


def _ctx(mesh, u_ref=UREF, **kw):
    from paper_2408_16509_amd import frmi
    return frmi.Context(mesh, precision=frmi.FR_FP32, u_ref=u_ref, **kw)


def _split(flat, like):
    out, o = [], 0
    for b in like:
        out.append(flat[o:o + b.size].reshape(b.shape))
        o += b.size
    return out


def gpu_rhs32(mesh, u_blocks, **kw):
    ctx = _ctx(mesh, **kw)
    u = ctx.pack(ctx.join_canon(u_blocks))
    assert u.dtype == torch.float32
    r = ctx.new_native()
    ctx.rhs(u, r)
    out = ctx.unpack_rhs(r).cpu().numpy()
    ctx.close()
    return _split(out, u_blocks)


# reference state of the random states (rho0 = 1, p0 = 1, at rest)
UREF_RANDOM = (1.0, 0.0, 0.0, 0.0, 1.0 / 0.4)


@pytest.mark.parametrize("order,system,riemann", [(2, 0, 0), (3, 0, 1), (3, 1, 0), (4, 1, 0)])
def test_fp32_rhs_random(order, system, riemann):
    mesh = inputs.hex_box((3, 3, 2), perturb=0.1, perturb_seed=4)
    bl = oracle_blocks(mesh, order)
    u = state_for(bl, "random", seed=5)
    Ro = ofr.rhs(bl, u, oracle_params(system, riemann))
    Rg = gpu_rhs32(mesh, u, system=system, order=order, riemann=riemann, u_ref=UREF_RANDOM)
    g, pv = rel_err(Rg, Ro)
    print(f"fp32 p={order} sys={system} riemann={riemann}: global {g:.2e} per-var {np.array2string(pv, precision=2)}")
    assert g <= 1e-5


@pytest.mark.parametrize("system", [0, 1])
def test_fp32_rhs_random_tets(system):
    mesh = inputs.kuhn_split(inputs.hex_box((2, 2, 2), perturb=0.1, perturb_seed=6), permute_seed=3)
    bl = oracle_blocks(mesh, 4)
    u = state_for(bl, "random", seed=8)
    Ro = ofr.rhs(bl, u, oracle_params(system, 0))
    Rg = gpu_rhs32(mesh, u, system=system, order=4, u_ref=UREF_RANDOM)
    g, pv = rel_err(Rg, Ro)
    print(f"fp32 tets sys={system}: global {g:.2e} per-var {np.array2string(pv, precision=2)}")
    assert g <= 1e-5


@pytest.mark.parametrize("beta", [-0.5, 0.3])
def test_fp32_rhs_random_tets_ldg_beta(beta):
    """FP32 form, Navier--Stokes on tets with the other one-sided switch and with a
    two-sided weighting (the common fluxes then come from the divergence kernel)."""
    mesh = inputs.kuhn_split(inputs.hex_box((2, 2, 2), perturb=0.1, perturb_seed=6), permute_seed=3)
    bl = oracle_blocks(mesh, 4)
    u = state_for(bl, "random", seed=8)
    Ro = ofr.rhs(bl, u, oracle_params(1, 0, ldg_beta=beta))
    Rg = gpu_rhs32(mesh, u, system=1, order=4, u_ref=UREF_RANDOM, ldg_beta=beta)
    g, pv = rel_err(Rg, Ro)
    print(f"fp32 tets NS beta={beta}: global {g:.2e} per-var {np.array2string(pv, precision=2)}")
    assert g <= 1e-5


@pytest.mark.parametrize("system", [0, 1])
def test_bf16x3_rhs_random_tets(system):
    """FP32 form with the tetrahedral operator products as BF16x3 split products
    (FP32 accumulation).  Stated bound for well-conditioned states: 1e-4 relative L2
    (each product keeps ~16 significant bits of both factors: a relative 2^-16 per
    term, times the cancellation of the contraction)."""
    from paper_2408_16509_amd import frmi
    mesh = inputs.kuhn_split(inputs.hex_box((2, 2, 2), perturb=0.1, perturb_seed=6), permute_seed=3)
    bl = oracle_blocks(mesh, 4)
    u = state_for(bl, "random", seed=8)
    Ro = ofr.rhs(bl, u, oracle_params(system, 0))
    ctx = frmi.Context(mesh, precision=frmi.FR_FP32_BF16X3, u_ref=UREF_RANDOM, system=system, order=4)
    ug = ctx.pack(ctx.join_canon(u))
    r = ctx.new_native()
    ctx.rhs(ug, r)
    Rg = _split(ctx.unpack_rhs(r).cpu().numpy(), u)
    ctx.close()
    g, pv = rel_err(Rg, Ro)
    g32, _ = rel_err(gpu_rhs32(mesh, u, system=system, order=4, u_ref=UREF_RANDOM), Ro)
    print(f"bf16x3 tets sys={system}: global {g:.2e} (fp32 form {g32:.2e}) per-var {np.array2string(pv, precision=2)}")
    assert g <= 1e-4


def test_fp32_reference_state_is_exact():
    mesh = inputs.hex_box((3, 3, 3), perturb=0.1, perturb_seed=2)
    bl = oracle_blocks(mesh, 3)
    u = [np.broadcast_to(np.array(UREF)[None, :, None], (len(b.elems), 5, b.ops.nsp)).copy() for b in bl]
    for system in (0, 1):
        Rg = gpu_rhs32(mesh, u, system=system, order=3)
        assert all(np.all(r == 0) for r in Rg)


@pytest.mark.parametrize("system,order,n", [(0, 2, 4), (1, 3, 8)])
def test_fp32_rhs_tgv_stated_errors(system, order, n):
    mesh = inputs.hex_box((n, n, n))
    bl = oracle_blocks(mesh, order)
    u = state_for(bl, "tgv")
    Ro = ofr.rhs(bl, u, oracle_params(system, 0))
    Rg = gpu_rhs32(mesh, u, system=system, order=order)
    g, pv = rel_err(Rg, Ro)
    print(f"fp32 TGV sys={system} p={order} n={n}: global {g:.2e} per-var {np.array2string(pv, precision=2)}")
    # stated bounds (see module docstring)
    assert g <= 1e-3
    assert np.all(pv[1:4] <= 1e-4) and pv[0] <= 1e-3 and pv[4] <= 1e-3


def test_fp32_rk4_solution_error():
    """10 RK4 steps (dt 1e-3) of the Euler TGV on 4^3, p = 2: FP32 operators with FP64
    accumulation against the FP64 oracle trajectory."""
    mesh = inputs.hex_box((4, 4, 4))
    bl = oracle_blocks(mesh, 2)
    u = state_for(bl, "tgv")
    prm = oracle_params(0, 0)
    uo = ork.rk4(lambda s: ofr.rhs(bl, s, prm), u, 1e-3, 10)
    ctx = _ctx(mesh, system=0, order=2)
    ug = ctx.pack64(ctx.join_canon(u))
    ctx.rk_step(ug, 1e-3, 10)
    got = _split(ctx.unpack64(ug).cpu().numpy(), u)
    du_g = [a - b for a, b in zip(got, u)]
    du_o = [a - b for a, b in zip(uo, u)]
    g, pv = rel_err(du_g, du_o)
    sol = rel_err(got, uo)[0]
    print(f"fp32 RK4 10 steps: increment rel {g:.2e} per-var {np.array2string(pv, precision=2)}; solution rel {sol:.2e}")
    assert sol <= 1e-9
    assert g <= 1e-5


# Stated per-variable bounds (rho, rho u, rho v, rho w, E) of one RHS of the Ma 0.1 NS
# Taylor--Green vortex on p = 4 tetrahedra (4^3 cells, +-10 % perturbed, 6 tets each)
# against the FP64 oracle.  The energy residual cancels terms of size H0 = 250 (and the
# density residual inherits it through the Rusanov dissipation), so the rounding of the
# contractions is amplified there; BF16x3 keeps about 16 significant bits per product
# term (relative 2^-16 ... 2^-17 against FP32's 2^-24), i.e. a few hundred times the
# FP32 error.
TGV_TET_BOUNDS = {
    "fp32": np.array([2e-3, 2e-4, 2e-4, 2e-4, 2e-3]),
    "bf16x3": np.array([0.5, 5e-2, 5e-2, 5e-2, 0.5]),
}


@pytest.mark.parametrize("form", ["fp32", "bf16x3"])
def test_reduced_forms_tgv_tets_stated_bounds(form):
    from paper_2408_16509_amd import frmi
    mesh = inputs.kuhn_split(inputs.hex_box((4, 4, 4), perturb=0.1, perturb_seed=5), permute_seed=9)
    bl = oracle_blocks(mesh, 4)
    u = state_for(bl, "tgv")
    prm = oracle_params(1, 0)
    Ro = ofr.rhs(bl, u, prm)
    prec = frmi.FR_FP32 if form == "fp32" else frmi.FR_FP32_BF16X3
    ctx = frmi.Context(mesh, precision=prec, u_ref=UREF, system=1, order=4)
    ug = ctx.pack(ctx.join_canon(u))
    r = ctx.new_native()
    ctx.rhs(ug, r)
    Rg = _split(ctx.unpack_rhs(r).cpu().numpy(), u)
    g, pv = rel_err(Rg, Ro)
    # the solution after 5 RK4 steps: the FP64 accumulation keeps dt R's rounding small
    uo = ork.rk4(lambda s: ofr.rhs(bl, s, prm), u, 2e-3, 5)
    u64 = ctx.pack64(ctx.join_canon(u))
    ctx.rk_step(u64, 2e-3, 5)
    got = _split(ctx.unpack64(u64).cpu().numpy(), u)
    ctx.close()
    sol = rel_err(got, uo)[0]
    print(f"{form} TGV tets: RHS global {g:.2e} per-var {np.array2string(pv, precision=2)}; "
          f"solution after 5 steps {sol:.2e}", flush=True)
    assert np.all(pv <= TGV_TET_BOUNDS[form])
    # the state after 5 steps carries 5 dt |dR| / |u|: at |R| / |u| ~ 10 and the per-RHS
    # bounds above that is below 5e-8 (FP32) and 1e-6 (BF16x3)
    assert sol <= (5e-8 if form == "fp32" else 1e-6)
