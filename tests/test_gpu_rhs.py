"""GPU parity of fr_rhs / fr_rk_step against the FP64 oracle (element by element).

Tolerance: relative L2 over all points and variables <= max(1e-12, 4 x floor),
where floor is the FP64 rounding floor of the RHS for that input (the oracle's
response to a one-ulp relative perturbation of the state, see helpers);
per variable, 10x that with the variable's norm floored at 1e-3 of the global norm
(the low-Mach density and energy residuals are small differences of large fluxes,
so their relative errors reflect the flux magnitudes, not the kernel); per element,
the error norm over the element's points and variables relative to the larger of its
own norm and the RMS element norm stays within 20x the global tolerance.
"""
import numpy as np
import pytest

from oracle import fr as ofr
from oracle import rk as ork
from paper_2408_16509_amd import inputs

from helpers import ELEM_FACTOR, elem_max_err, oracle_blocks, oracle_floor, oracle_params, rel_err, state_for

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _ctx(mesh, **kw):
    from paper_2408_16509_amd import frmi
    return frmi.Context(mesh, **kw)


def gpu_rhs(mesh, u_blocks, **kw):
    ctx = _ctx(mesh, **kw)
    u = ctx.pack(ctx.join_canon(u_blocks))
    r = ctx.new_native()
    ctx.rhs(u, r)
    out = ctx.unpack_rhs(r).cpu().numpy()
    ctx.close()
    return [b.copy() for b in _split(out, u_blocks)]


def _split(flat, like):
    out, o = [], 0
    for b in like:
        out.append(flat[o:o + b.size].reshape(b.shape))
        o += b.size
    return out


def check(Rg, Ro, tol=1e-12, floor_=0.0):
    tol = max(tol, 4 * floor_)
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


CASES = [
    # (mesh, order, system, riemann, state)
    ("hex332", 1, 0, 0, "random"),
    ("hex332", 2, 0, 0, "random"),
    ("hex332", 3, 0, 1, "random"),
    ("hex332", 4, 0, 0, "random"),
    ("hexpert", 2, 0, 1, "random"),
    ("hexpert", 3, 0, 0, "random"),
    ("hexpert", 4, 0, 1, "random"),
    ("hex111", 2, 0, 0, "random"),
    ("hex211", 3, 0, 1, "random"),
    ("hex332", 2, 1, 0, "random"),
    ("hex332", 3, 1, 1, "random"),
    ("hexpert", 3, 1, 0, "random"),
    ("hexpert", 4, 1, 0, "random"),
    ("hex111", 3, 1, 0, "random"),
    ("hex444", 2, 0, 0, "tgv"),
    ("hex444", 3, 1, 0, "tgv"),
    ("tet1", 4, 0, 0, "random"),
    ("tet1", 4, 0, 1, "random"),
    ("tetpert", 4, 0, 0, "random"),
    ("tetpert", 4, 1, 0, "random"),
    ("tet1", 4, 1, 1, "random"),
    ("tetpert", 4, 0, 1, "tgv"),
    ("mixed", 4, 0, 0, "random"),
    ("mixed", 4, 1, 0, "random"),
]

MESHES = {
    "hex332": lambda: inputs.hex_box((3, 3, 2)),
    "hex444": lambda: inputs.hex_box((4, 4, 4)),
    "hex111": lambda: inputs.hex_box((1, 1, 1)),
    "hex211": lambda: inputs.hex_box((2, 1, 1)),
    "hexpert": lambda: inputs.hex_box((3, 4, 3), perturb=0.1, perturb_seed=31, permute_seed=32),
    "tet1": lambda: inputs.kuhn_split(inputs.hex_box((1, 1, 1))),
    "tetpert": lambda: inputs.kuhn_split(inputs.hex_box((2, 3, 2), perturb=0.1, perturb_seed=51), permute_seed=53),
    # a hex box and a tet box (shifted so no face of one lies on a face of the other) in one context
    "mixed": lambda: inputs.concat([
        inputs.hex_box((2, 2, 2), perturb=0.1, perturb_seed=5),
        inputs.kuhn_split(inputs.hex_box((2, 2, 2), lo=(-3.0, -3.1, -3.2),
                                         hi=(-3.0 + 2 * np.pi, -3.1 + 2 * np.pi, -3.2 + 2 * np.pi))),
    ], permute_seed=7),
}


@pytest.mark.parametrize("mname,order,system,riemann,state", CASES)
def test_rhs_parity_small(mname, order, system, riemann, state):
    print(f"case {mname} p={order} system={system} riemann={riemann} state={state}", flush=True)
    mesh = MESHES[mname]()
    bl = oracle_blocks(mesh, order)
    u = state_for(bl, state, seed=3)
    fl, Ro = oracle_floor(mesh, order, u, oracle_params(system, riemann))
    Rg = gpu_rhs(mesh, u, system=system, order=order, riemann=riemann)
    check(Rg, Ro, floor_=fl)


@pytest.mark.parametrize("mname", ["mixed", "tetpert"])
@pytest.mark.parametrize("beta", [-0.5, 0.3])
def test_rhs_parity_ldg_beta(mname, beta):
    """Navier--Stokes with the other one-sided switch (beta = -1/2: the left side's
    gradient and state) and a two-sided weighting (beta = 0.3: both gradients)."""
    print(f"case {mname} NS beta={beta}", flush=True)
    mesh = MESHES[mname]()
    bl = oracle_blocks(mesh, 4)
    u = state_for(bl, "random", seed=3)
    fl, Ro = oracle_floor(mesh, 4, u, oracle_params(1, 0, ldg_beta=beta))
    Rg = gpu_rhs(mesh, u, system=1, order=4, riemann=0, ldg_beta=beta)
    check(Rg, Ro, floor_=fl)


def test_rhs_parity_config1_and_rk4_10_steps():
    """4^3 straight hexes, p = 2, Euler TGV Ma 0.1, Rusanov: RHS and 10 RK4 steps, dt = 1e-3."""
    mesh = inputs.hex_box((4, 4, 4))
    bl = oracle_blocks(mesh, 2)
    u = state_for(bl, "tgv")
    prm = oracle_params(0, 0)
    fl, Ro = oracle_floor(mesh, 2, u, prm)
    check(gpu_rhs(mesh, u, system=0, order=2, riemann=0), Ro, floor_=fl)
    uo = ork.rk4(lambda s: ofr.rhs(bl, s, prm), u, 1e-3, 10)
    ctx = _ctx(mesh, system=0, order=2, riemann=0)
    ug = ctx.pack64(ctx.join_canon(u))
    ctx.rk_step(ug, 1e-3, 10)
    got = _split(ctx.unpack64(ug).cpu().numpy(), u)
    # compare the change over the 10 steps (the state itself is O(p0))
    du_g = [g - a for g, a in zip(got, u)]
    du_o = [o - a for o, a in zip(uo, u)]
    check(du_g, du_o, tol=1e-11)


def test_rk4_equals_composed_rhs():
    mesh = inputs.hex_box((3, 3, 3), perturb=0.1, perturb_seed=5)
    bl = oracle_blocks(mesh, 3)
    u = state_for(bl, "random", seed=9)
    ctx = _ctx(mesh, system=1, order=3, riemann=0)
    u0 = ctx.pack(ctx.join_canon(u))
    dt = 1e-3
    k = [ctx.new_native() for _ in range(4)]
    st = u0.clone()
    ctx.rhs(u0, k[0])
    st = u0 + 0.5 * dt * k[0]
    ctx.rhs(st, k[1])
    st = u0 + 0.5 * dt * k[1]
    ctx.rhs(st, k[2])
    st = u0 + dt * k[2]
    ctx.rhs(st, k[3])
    ref = u0 + dt / 6 * (k[0] + 2 * k[1] + 2 * k[2] + k[3])
    u1 = u0.clone()
    ctx.rk_step(u1, dt, 1)
    a, b = ctx.unpack(u1), ctx.unpack(ref)
    torch.cuda.synchronize()
    d = (a - b).abs().max().item()
    assert d <= 1e-13 * b.abs().max().item()


def test_check_detects_nonfinite():
    mesh = inputs.hex_box((2, 2, 2))
    bl = oracle_blocks(mesh, 2)
    u = state_for(bl, "random")
    ctx = _ctx(mesh, order=2)
    ug = ctx.pack64(ctx.join_canon(u))
    assert ctx.check(ug)
    ug[5] = float("nan")
    assert not ctx.check(ug)


def test_rhs_parity_config2_full_size():
    """32^3 hexes, p = 3, Navier--Stokes TGV Re 1600 Ma 0.1, LDG, FP64: full-size parity."""
    mesh = inputs.hex_box((32, 32, 32))
    bl = oracle_blocks(mesh, 3)
    u = state_for(bl, "tgv")
    fl, Ro = oracle_floor(mesh, 3, u, oracle_params(1, 0))
    Rg = gpu_rhs(mesh, u, system=1, order=3, riemann=0)
    check(Rg, Ro, floor_=fl)


@pytest.mark.parametrize("precision", [0, 1])
def test_native_order_does_not_change_results(precision):
    """The native element order (input order, Morton renumbering, automatic) only moves
    data: the canonical right-hand side of a permuted mixed hex + tet mesh is bit-identical."""
    from paper_2408_16509_amd import frmi
    mesh = inputs.concat([inputs.hex_box((4, 4, 4), perturb=0.1, perturb_seed=3),
                          inputs.kuhn_split(inputs.hex_box((3, 3, 3), lo=(3.0, -3.0, -3.0),
                                                           hi=(3.0 + 2 * np.pi, -3.0 + 2 * np.pi, -3.0 + 2 * np.pi)))],
                         permute_seed=5)
    kw = dict(system=1, order=4, riemann=0)
    if precision:
        kw.update(precision=frmi.FR_FP32, u_ref=(1.0, 0.0, 0.0, 0.0, 2.5))
    out = []
    for order in (1, 2, 0):
        ctx = _ctx(mesh, elem_order=order, **kw)
        x = ctx.sol_points()
        n = x.shape[0]
        rng = np.random.default_rng(7)
        rho = 1.0 + 0.1 * rng.uniform(-1, 1, n)
        vel = 0.3 * rng.uniform(-1, 1, (3, n))
        p = 1.0 + 0.1 * rng.uniform(-1, 1, n)
        st = np.stack([rho, rho * vel[0], rho * vel[1], rho * vel[2], p / 0.4 + 0.5 * rho * (vel ** 2).sum(0)])
        canon = np.concatenate([np.moveaxis(st[:, o:o + m * s].reshape(5, m, s), 0, 1).ravel()
                                for o, m, s in _blocks_of(ctx)])
        u = ctx.pack(canon)
        r = ctx.new_native()
        ctx.rhs(u, r)
        out.append(ctx.unpack_rhs(r).cpu().numpy())
        ctx.close()
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


def _blocks_of(ctx):
    lay = ctx.layout
    res, o = [], 0
    for i in range(lay.n_types):
        m, s = lay.n_elem[i], lay.n_sp[i]
        res.append((o, m, s))
        o += m * s
    return res


def test_context_on_a_side_stream():
    """A context on a stream other than torch's current one: the binding's own buffers
    (the packed state, the unpacked result) are made on the context's stream, so two RK4
    steps there give the bits they give on the current stream."""
    from paper_2408_16509_amd import frmi
    mesh = inputs.hex_box((16, 16, 16), perturb=0.1, perturb_seed=3)
    bl = oracle_blocks(mesh, 3)
    canon = state_for(bl, "tgv")[0].ravel()
    out = []
    for side in (False, True):
        s = torch.cuda.Stream() if side else None
        ctx = frmi.Context(mesh, stream=None if s is None else s.cuda_stream, system=1, order=3)
        u = ctx.pack64(canon)
        ctx.rk_step(u, 1e-3, 2)
        got = ctx.unpack64(u)
        torch.cuda.synchronize()
        out.append(got.cpu().numpy())
        ctx.close()
    print(f"side stream vs current stream: max |diff| {np.abs(out[0] - out[1]).max():.1e}", flush=True)
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_zero_steps_leave_the_state(precision):
    """fr_rk_step with n_steps = 0 (a degenerate call): the state is left bit for bit, with and
    without the filter."""
    from paper_2408_16509_amd import frmi
    mesh = MESHES["mixed"]()
    bl = oracle_blocks(mesh, 4)
    u0 = state_for(bl, "random", seed=5)
    kw = dict(system=1, order=4)
    if precision == "fp32":
        kw.update(precision=frmi.FR_FP32, u_ref=(1.0, 0.0, 0.0, 0.0, 2.5))
    ctx = _ctx(mesh, **kw)
    for mode in (-1, 0):
        u = ctx.pack64(ctx.join_canon(u0))
        before = u.clone()
        ctx.rk_step(u, 1e-3, 0, filter_mode=mode)
        torch.cuda.synchronize()
        assert torch.equal(u, before)
    ctx.close()
