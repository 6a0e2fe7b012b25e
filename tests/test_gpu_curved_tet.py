"""GPU parity on curved tetrahedra (fr_setup_mesh_curved_tet: metric terms stored per
solution point) against the FP64 oracle with the same metric (Sec. "Curved elements",
the tetrahedra of Fig. fsp).

Meshes: seeded curved periodic boxes of geometry order q (smooth periodic displacement
plus node jitter) cut into 6 tetrahedra per cell, 3 x 3 x 2 cells = 108 elements (six
16-element tiles, the seventh ragged), element order permuted.  FP64 tolerance:
relative L2 <= max(1e-12, 4 x floor), over all values and per variable with its own
floor, where floor is the oracle's response to a one-ulp relative perturbation of the
state plus a relative perturbation of its metric terms (S, J, S^T n~) of 35 eps, the
terms of the nodal sums that form them; per element 20x that.
Free stream (uniform state): the conservative metric keeps |R| at rounding level (bound
1e-10); the cross-product metric does not at q = 4 (2(q - 1) = 6 > 4), and there the GPU
and the oracle agree on its values; at q <= 3 both stay at rounding level.
A q = 1 curved context and the straight-element path agree to rounding (the affine map
makes both metrics the straight one).
FP32 and BF16x3 forms: well-conditioned random states within the bounds stated for
straight tetrahedra (1e-5 and 1e-4 relative L2).
"""
import dataclasses

import numpy as np
import pytest

from oracle import fr as ofr
from oracle import mesh as omesh
from oracle import rk as ork
from paper_2408_16509_amd import inputs

from helpers import ELEM_FACTOR, elem_max_err, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

UREF = (1.0, 0.0, 0.0, 0.0, 2.5)


def _mesh(q, n=(3, 3, 2), perturb=0.04):
    return inputs.curved_tet_box(n, q=q, amp=0.2, perturb=perturb, perturb_seed=3, permute_seed=7)


def _state(b, kind, seed=1):
    x = b.xsol
    if kind == "random":
        s = inputs.random_state(x.shape[:2], seed)
    elif kind == "tgv":
        s = inputs.tgv(x[..., 0], x[..., 1], x[..., 2], mach=0.1)
    else:
        s = np.zeros((5,) + x.shape[:2])
        s[0], s[1], s[2], s[3], s[4] = 1.2, 0.3, -0.2, 0.5, 2.5
    return np.moveaxis(s, 0, 1).copy()


def _gpu_rhs(mesh, u, **kw):
    from paper_2408_16509_amd import frmi
    ctx = frmi.Context(mesh, order=4, **kw)
    ug = ctx.pack(u.ravel())
    r = ctx.new_native()
    ctx.rhs(ug, r)
    out = ctx.unpack_rhs(r).cpu().numpy().reshape(u.shape)
    ctx.close()
    return out


def _floor(bl, u, prm):
    R = ofr.rhs(bl, [u], prm)[0]
    rng = np.random.default_rng(0)
    up = u * (1 + 2.0 ** -53 * rng.uniform(-1, 1, size=u.shape))
    f_state = rel_err([ofr.rhs(bl, [up], prm)[0]], [R])
    b = bl[0]
    eps = 35 * 2.0 ** -53
    bp = dataclasses.replace(b, S=b.S * (1 + eps * rng.uniform(-1, 1, size=b.S.shape)),
                             J=b.J * (1 + eps * rng.uniform(-1, 1, size=b.J.shape)),
                             snorm=b.snorm * (1 + eps * rng.uniform(-1, 1, size=b.snorm.shape)))
    f_metric = rel_err([ofr.rhs([bp], [u], prm)[0]], [R])
    return f_state[0] + f_metric[0], f_state[1] + f_metric[1], R


CASES = [
    # (q, system, riemann, beta, metric, state)
    (2, 0, 0, 0.5, "conservative", "random"),
    (3, 0, 1, 0.5, "conservative", "tgv"),
    (4, 0, 1, 0.5, "conservative", "random"),
    (2, 1, 0, 0.5, "conservative", "random"),
    (3, 1, 1, 0.3, "conservative", "tgv"),
    (4, 1, 0, -0.5, "conservative", "random"),
    (4, 1, 0, 0.5, "conservative", "tgv"),
    (3, 0, 0, 0.5, "cross", "random"),
    (4, 1, 0, 0.5, "cross", "random"),
]


@pytest.mark.parametrize("q,system,riemann,beta,metric,state", CASES)
def test_curved_tet_rhs_fp64(q, system, riemann, beta, metric, state):
    from paper_2408_16509_amd import frmi
    m = _mesh(q)
    bl = omesh.build(m, 4, metric)
    u = _state(bl[0], state)
    prm = ofr.Params(system=system, riemann=riemann, ldg_beta=beta)
    floor, pv_floor, Ro = _floor(bl, u, prm)
    Rg = _gpu_rhs(m, u, system=system, riemann=riemann, ldg_beta=beta,
                  hex_metric=frmi.FR_METRIC_CONSERVATIVE if metric == "conservative" else frmi.FR_METRIC_CROSS)
    g, pv = rel_err([Rg], [Ro])
    tol = max(1e-12, 4 * floor)
    pv_tol = np.maximum(1e-12, 4 * pv_floor)
    em = elem_max_err([Rg], [Ro])
    print(f"q={q} sys={system} riemann={riemann} beta={beta} {metric} {state}: rel L2 {g:.2e} (tol {tol:.1e}) "
          f"per-var {np.array2string(pv, precision=2)} (tol {np.array2string(pv_tol, precision=2)}) "
          f"max per element {em:.2e}", flush=True)
    assert g <= tol
    assert np.all(pv <= pv_tol)
    assert em <= ELEM_FACTOR * tol


@pytest.mark.parametrize("q", [2, 3, 4])
def test_curved_tet_free_stream(q):
    from paper_2408_16509_amd import frmi
    m = _mesh(q)
    out = {}
    for metric, code in (("conservative", frmi.FR_METRIC_CONSERVATIVE), ("cross", frmi.FR_METRIC_CROSS)):
        bl = omesh.build(m, 4, metric)
        u = _state(bl[0], "uniform")
        for system in (0, 1):
            Ro = ofr.rhs(bl, [u], ofr.Params(system=system))[0]
            Rg = _gpu_rhs(m, u, system=system, hex_metric=code)
            out[(metric, system)] = (np.abs(Rg).max(), np.abs(Ro).max(), np.abs(Rg - Ro).max())
    print(f"q={q}: " + ", ".join(f"{k}: gpu {v[0]:.1e} oracle {v[1]:.1e}" for k, v in out.items()), flush=True)
    for system in (0, 1):
        assert out[("conservative", system)][0] <= 1e-10
        g, o, d = out[("cross", system)]
        if 2 * (q - 1) > 4:
            assert g > 1e-3 and d <= 1e-10 * o
        else:
            assert g <= 1e-10


@pytest.mark.parametrize("system", [0, 1])
def test_q1_curved_tet_equals_straight_path(system):
    m = _mesh(1)
    straight = inputs.Mesh(m.xyz, m.etype, m.enodes, m.period)
    bl = omesh.build(straight, 4)
    u = _state(bl[0], "random")
    Rc = _gpu_rhs(m, u, system=system)
    Rs = _gpu_rhs(straight, u, system=system)
    g = rel_err([Rc], [Rs])[0]
    print(f"sys={system}: curved tets (q=1) vs straight path {g:.2e}", flush=True)
    assert g <= 1e-12


@pytest.mark.parametrize("system", [0, 1])
@pytest.mark.parametrize("form", ["fp32", "bf16x3"])
def test_curved_tet_reduced_forms(form, system):
    from paper_2408_16509_amd import frmi
    m = _mesh(3)
    bl = omesh.build(m, 4)
    u = _state(bl[0], "random")
    Ro = ofr.rhs(bl, [u], ofr.Params(system=system))[0]
    prec = frmi.FR_FP32 if form == "fp32" else frmi.FR_FP32_BF16X3
    Rg = _gpu_rhs(m, u, system=system, precision=prec, u_ref=UREF)
    g = rel_err([Rg], [Ro])[0]
    print(f"{form} form, curved tets q=3 sys={system}: {g:.2e}", flush=True)
    assert g <= (1e-5 if form == "fp32" else 1e-4)


def test_curved_tet_rk4_steps():
    from paper_2408_16509_amd import frmi
    m = _mesh(4)
    bl = omesh.build(m, 4)
    u = _state(bl[0], "tgv")
    prm = ofr.Params(system=1)
    uo = ork.rk4(lambda s: ofr.rhs(bl, s, prm), [u.copy()], 2e-3, 3)
    ctx = frmi.Context(m, system=1, order=4)
    ug = ctx.pack64(u.ravel())
    ctx.rk_step(ug, 2e-3, 3)
    got = ctx.unpack64(ug).cpu().numpy().reshape(u.shape)
    ctx.close()
    err = np.linalg.norm(got - uo[0]) / np.linalg.norm(uo[0] - u)
    print(f"3 RK4 steps, NS TGV on curved tets q=4: {err:.2e} of the state change", flush=True)
    assert err <= 1e-10


def test_curved_tet_whole_field_fp64():
    """NS TGV (Ma 0.1) on 12^3 cells of the bench's curved-tetrahedron construction (q = 4,
    amplitude 0.1, 10,368 elements, 648 tiles), whole field against the oracle, with the
    rounding floor of this same input (the residual of a resolved low-Mach state is small
    against the terms it cancels, so the floor depends on the resolution)."""
    m = inputs.curved_tet_box((12, 12, 12), q=4, amp=0.1, permute_seed=57)
    bl = omesh.build(m, 4)
    x = bl[0].xsol
    u = np.moveaxis(inputs.tgv(x[..., 0], x[..., 1], x[..., 2], mach=0.1), 0, 1).copy()
    prm = ofr.Params(system=1)
    floor, pv_floor, Ro = _floor(bl, u, prm)
    Rg = _gpu_rhs(m, u, system=1)
    g, pv = rel_err([Rg], [Ro])
    tol, pv_tol = max(1e-12, 4 * floor), np.maximum(1e-12, 4 * pv_floor)
    em = elem_max_err([Rg], [Ro])
    print(f"12^3 x 6 curved tets q=4 NS TGV: rel L2 {g:.2e} (tol {tol:.1e}) per-var "
          f"{np.array2string(pv, precision=2)} (tol {np.array2string(pv_tol, precision=2)}) "
          f"max per element {em:.2e}", flush=True)
    assert g <= tol and np.all(pv <= pv_tol) and em <= ELEM_FACTOR * tol
    # the FP32 form (pair-once common flux) on the same field, per variable within the bounds
    # stated for the Ma 0.1 tetrahedral TGV (the low-Mach residual cancels terms of the
    # enthalpy's size in rho and E)
    from paper_2408_16509_amd import frmi
    p0 = 1.0 / (1.4 * 0.01)
    R32 = _gpu_rhs(m, u, system=1, precision=frmi.FR_FP32, u_ref=(1.0, 0.0, 0.0, 0.0, p0 / 0.4))
    pv32 = rel_err([R32], [Ro])[1]
    print(f"  FP32 form per-var {np.array2string(pv32, precision=2)}", flush=True)
    assert np.all(pv32 <= np.array([5e-2, 2e-3, 2e-3, 2e-3, 5e-2]))


def test_curved_tet_full_size_free_stream():
    """At the bench's full size (32^3 cells, 196,608 curved tetrahedra of order 4, the
    launch configuration it times), a property that holds at any size: a uniform stream
    stays uniform with the conservative metric and does not with the cross-product metric.
    Bounds: FP64 1e-10; FP32 form 2e-3, about 3e-6 of the size of the terms that cancel
    (|f| |S| / J (p+1)^2 ~ 600 on these elements), i.e. tens of FP32 rounding steps; the
    cross-product metric above 1e-8 and 1000x the conservative FP64 value (on 32^3 cells
    of amplitude 0.1 the elements are nearly straight, so its truncation error is small:
    2e-6 measured, against 0.9-2 on the coarse meshes above)."""
    from paper_2408_16509_amd import frmi
    m = inputs.curved_tet_box((32, 32, 32), q=4, amp=0.1, permute_seed=57)
    res = {}
    for name, code, kw in (("conservative", frmi.FR_METRIC_CONSERVATIVE, {}),
                           ("conservative_fp32", frmi.FR_METRIC_CONSERVATIVE,
                            dict(precision=frmi.FR_FP32, u_ref=UREF)),
                           ("cross", frmi.FR_METRIC_CROSS, {})):
        ctx = frmi.Context(m, system=1, order=4, hex_metric=code, **kw)
        n = ctx.layout.n_elem[0]
        canon = np.empty((n, 5, 35))
        canon[:, 0], canon[:, 1], canon[:, 2], canon[:, 3], canon[:, 4] = 1.2, 0.3, -0.2, 0.5, 2.5
        r = ctx.new_native()
        ctx.rhs(ctx.pack(canon.ravel()), r)
        res[name] = float(torch.max(torch.abs(ctx.unpack_rhs(r))).item())
        ctx.close()
    print(f"196,608 curved tets, uniform stream, max |R|: {res}", flush=True)
    assert res["conservative"] <= 1e-10 and res["conservative_fp32"] <= 2e-3
    assert res["cross"] > 1e-8 and res["cross"] > 1e3 * res["conservative"]


def test_curved_tet_filtered_rk_step():
    """One RK4 step of the Mach-3 shock on curved tetrahedra (q = 2) with the plain entropy
    filter on every stage state and the new state (the filter uses no metric terms; its
    stage states come from the curved right-hand side), against the oracle: FP64 within
    1e-10 of the increment, and the filter treats elements in the step."""
    from oracle import entropy_filter as ef
    from paper_2408_16509_amd import frmi
    m = inputs.curved_tet_box((3, 3, 3), q=2, amp=0.15, permute_seed=7)
    bl = omesh.build(m, 4)
    x = bl[0].xsol
    ic = np.moveaxis(inputs.shock(x[..., 0], x[..., 1], x[..., 2]), 0, 1).copy()
    fp = ef.FilterParams()
    u0 = ef.entropy_filter(bl, [ic], [ic], fp)[0][0]
    smin0 = ef.smin_neighbourhood(bl, [u0], fp)
    treated = []

    def post(s):
        out = [ef.filter_block(bb, ss, sm, fp) for bb, ss, sm in zip(bl, s, smin0)]
        treated.append(sum(int((r[1] != 0).sum()) for r in out))
        return [r[0] for r in out]
    uo = ork.rk4_step(lambda s: ofr.rhs(bl, s, ofr.Params(riemann=1)), [u0], 5e-3, stage_post=post)[0]
    assert sum(treated) > 0
    ctx = frmi.Context(m, system=0, order=4, riemann=1)
    ug = ctx.pack64(u0.ravel())
    ctx.rk_step(ug, 5e-3, 1, filter_mode=0)
    got = ctx.unpack64(ug).cpu().numpy().reshape(uo.shape)
    ok = ctx.check(ug)
    ctx.close()
    err = np.linalg.norm(got - uo) / np.linalg.norm(uo - u0)
    print(f"filtered RK4 step on curved tets: {err:.2e} of the increment", flush=True)
    assert err <= 1e-10 and ok
    assert ef.admissible(bl[0], got, smin0[0], fp)[0].all()


def test_curved_tet_adaptive_fp64():
    """Adaptive stepping (embedded pair and controller) on curved tetrahedra: the oracle's
    sequence of accepted and rejected steps, its final time and state."""
    from oracle import rk_adaptive as ra
    from paper_2408_16509_amd import frmi
    m = _mesh(3)
    bl = omesh.build(m, 4)
    x = bl[0].xsol
    u = np.moveaxis(inputs.tgv(x[..., 0], x[..., 1], x[..., 2], mach=0.3), 0, 1).copy()
    uo, so = ra.integrate(lambda s: ofr.rhs(bl, s, ofr.Params()), [u], 0.1, 0.05, ra.Controller(atol=1e-6, rtol=1e-6))
    ctx = frmi.Context(m, system=0, order=4)
    ug = ctx.pack64(u.ravel())
    sg = ctx.rk_adaptive(ug, 0.1, 0.05, atol=1e-6, rtol=1e-6)
    got = ctx.unpack64(ug).cpu().numpy().reshape(u.shape)
    ctx.close()
    err = np.linalg.norm(got - uo[0]) / np.linalg.norm(uo[0] - u)
    print(f"curved tets adaptive: accepted {sg.accepted} (oracle {so.accepted}), rejected {sg.rejected} "
          f"(oracle {so.rejected}), state {err:.2e}", flush=True)
    assert (sg.accepted, sg.rejected) == (so.accepted, so.rejected) and sg.t == so.t == 0.1
    assert abs(sg.dt_next - so.dt_next) <= 1e-9 * so.dt_next
    assert err <= 1e-10


@pytest.mark.parametrize("system", [0, 1])
def test_curved_tet_single_cell(system):
    """The degenerate mesh: one periodic cell (6 curved tetrahedra, q = 3, each face's partner
    in the same cell or across the cell's own periodic boundary), FP64 against the oracle."""
    m = inputs.curved_tet_box((1, 1, 1), q=3, amp=0.1)
    bl = omesh.build(m, 4)
    u = _state(bl[0], "random")
    prm = ofr.Params(system=system, riemann=1)
    floor, pv_floor, Ro = _floor(bl, u, prm)
    Rg = _gpu_rhs(m, u, system=system, riemann=1)
    g, pv = rel_err([Rg], [Ro])
    tol = max(1e-12, 4 * floor)
    print(f"single curved cell sys={system}: rel L2 {g:.2e} (tol {tol:.1e})", flush=True)
    assert g <= tol and np.all(pv <= np.maximum(1e-12, 4 * pv_floor))
