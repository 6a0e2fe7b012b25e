#!/usr/bin/env python3
"""Throughput of the FR right-hand side on one MI355X.

Default workload (the headline): compressible Navier--Stokes Taylor--Green vortex
(Re 1600, Ma 0.1, Pr 0.71, LDG viscous terms, Rusanov inviscid flux) on the mixed
mesh of p = 4 hexahedra and p = 4 tetrahedra: two periodic 32 x 64 x 64 boxes of
+-10 % perturbed cells, one kept as 131,072 hexahedra (125 points each), the other
cut into 786,432 tetrahedra (35 points each), element order permuted: 917,504
elements, 43,909,120 points.  Two forms are timed: FP32 operators and fluxes on
FP32 deviations with FP64 RK accumulation and the entropy filter on every stage
with the learned warm start (the headline), and FP64 with the plain filter.
A step is one classical RK4 step (4 right-hand sides, stage updates, filter) on
the device-resident state; the metric counts right-hand-side degrees of freedom
(elements x solution points, the paper's DoF) per second:
GDoF/s = 4 * sum_e N_sp(e) * steps / time / 1e9.

Also reported: the dominant kernel against the 8 TB/s HBM peak (bytes of the
algorithmic minimum of the right-hand side, read u and write R once, for the
points that kernel processes; the kernel's own compulsory traffic beside it),
each reduced form's error against the FP64 form per variable, the FP64 CPU
oracle timed on the host on a bounded sample of the same workload, and two more
workloads (the 32^3 p = 3 hexahedral NS TGV, the NS TGV on 82,944 p = 4 pyramids, and
the 48^3 Mach-3 shock with the trained learned filter against the plain one) under
"extra_workloads".  Other
workloads by --config (see CONFIGS): curved hexahedra and tetrahedra, adaptive
stepping, the 48^3 perturbed p = 4 hexahedra, and p = 4 pyramids (ns_tgv_pyr24_p4).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

CONFIGS = {
    # name: mesh cells, order, system, riemann, Mach, dt
    "ns_tgv_hex32_p3": dict(n=(32, 32, 32), order=3, system=1, riemann=0, mach=0.1, dt=4e-4, oracle_ok=True),
    "euler_tgv_hex4_p2": dict(n=(4, 4, 4), order=2, system=0, riemann=0, mach=0.1, dt=1e-3, oracle_ok=True),
    "ns_tgv_hex48pert_p4": dict(n=(48, 48, 48), order=4, system=1, riemann=0, mach=0.1, dt=1.5e-4,
                                perturb=0.1, perturb_seed=31, permute_seed=32),
    # 32x64x64 cells twice, +-10 % perturbed (seed 51): p = 4 hexahedra, and the same
    # cells as 6 p = 4 tetrahedra each (917,504 elements), element order seed 53
    # timed forms: FP32 + learned filter (headline), FP64 + plain filter, and both unfiltered
    "ns_tgv_mixed_c5split_p4": dict(kind="mixed", n=(32, 64, 64), order=4, system=1, riemann=0, mach=0.1,
                                    dt=7.5e-5, perturb=0.1, perturb_seed=51, permute_seed=53,
                                    forms="fp32:learned,fp64:plain",
                                    # the warm-start MLP of the learned form, trained on the plain filter's
                                    # rows from a small mixed-mesh Mach-3 shock (NS, p = 4, both element types)
                                    mlp_train=dict(n=(4, 8, 8), seeds=(101, 102, 103), steps=20, dt=5e-4,
                                                   iters=2000),
                                    # oracle timing sample: the same two boxes at 12 x 12 x 12 cells each
                                    oracle_sample=(12, 12, 12)),
    # Mach-3 shock (orientation seed 41, density noise seed 42), Euler + HLLC, entropy
    # filter on every RK stage: plain bisection vs the learned warm start, the MLP
    # trained on the plain filter's data from held-out draws (seeds 101-108 / 201-208)
    # the NS TGV 32^3 p = 3 workload advanced to t = 8e-3 (20 steps of the RK4 dt) with the
    # adaptive embedded pair (atol = rtol = 1e-6, first step 4e-4), against fixed-dt RK4
    # the NS TGV 32^3 p = 3 workload on cubically curved hexahedra (smooth periodic
    # displacement of amplitude 0.1): metric terms stored per point, conservative form
    "ns_tgv_hex32_p3_curved": dict(kind="curved", n=(32, 32, 32), q=3, amp=0.1, order=3, system=1, riemann=0,
                                   mach=0.1, dt=4e-4, oracle_ok=True),
    # the NS TGV on curved tetrahedra of geometry order 4 (the order where the cross-product
    # metric's degree, 6, exceeds the solution order): 32^3 cells of the same curved lattice
    # (amplitude 0.1), 6 tetrahedra each (196,608 elements, 6.9 M points), element order
    # seed 57, conservative metric; oracle timing sample at 12^3 cells
    "ns_tgv_tet32_q4_curved": dict(kind="curved_tet", n=(32, 32, 32), q=4, amp=0.1, order=4, system=1, riemann=0,
                                   mach=0.1, dt=7.5e-5, permute_seed=57, oracle_sample=(12, 12, 12)),
    # the NS TGV on p = 4 pyramids with affine bases (the transition element): 24^3 cells cut
    # into 6 pyramids each around an apex moved by up to 10 % of a cell (seed 61), 82,944
    # elements, 4.6 M points, element order seed 62; oracle timing sample at 8^3 cells
    "ns_tgv_pyr24_p4": dict(kind="pyramid", n=(24, 24, 24), order=4, system=1, riemann=0, mach=0.1, dt=7.5e-5,
                            apex_perturb=0.1, perturb_seed=61, permute_seed=62, oracle_sample=(8, 8, 8)),
    "ns_tgv_hex32_p3_adaptive": dict(n=(32, 32, 32), order=3, system=1, riemann=0, mach=0.1, dt=4e-4,
                                     adaptive=True, t_end=8e-3, tol=1e-6),
    "euler_shock_hex48_p3": dict(n=(48, 48, 48), order=3, system=0, riemann=1, dt=5e-4, filter=True,
                                 orient_seed=41, noise_seed=42, train_seeds=tuple(range(101, 109)),
                                 train_steps=50, val_seed=109, train_iters=4000),
}


def build_mesh(cfg, inputs):
    if cfg.get("kind") == "mixed":
        # two conforming periodic boxes in one context: hexahedra, and the same cells
        # cut into 6 tetrahedra each (the tet box offset in x so the two never pair)
        n = cfg["n"]
        lo_b = (3.0, -3.141592653589793, -3.141592653589793)
        hi_b = tuple(v + 2 * 3.141592653589793 for v in lo_b)
        a = inputs.hex_box(n, perturb=cfg["perturb"], perturb_seed=cfg["perturb_seed"])
        b = inputs.kuhn_split(inputs.hex_box(n, lo=lo_b, hi=hi_b, perturb=cfg["perturb"],
                                             perturb_seed=cfg["perturb_seed"]))
        return inputs.concat([a, b], permute_seed=cfg["permute_seed"])
    if cfg.get("kind") == "curved":
        return inputs.curved_hex_box(cfg["n"], q=cfg["q"], amp=cfg["amp"], permute_seed=cfg.get("permute_seed"))
    if cfg.get("kind") == "pyramid":
        return inputs.pyramid_box(cfg["n"], apex_perturb=cfg["apex_perturb"], perturb_seed=cfg["perturb_seed"],
                                  permute_seed=cfg.get("permute_seed"))
    if cfg.get("kind") == "curved_tet":
        return inputs.curved_tet_box(cfg["n"], q=cfg["q"], amp=cfg["amp"], permute_seed=cfg.get("permute_seed"))
    return inputs.hex_box(cfg["n"], perturb=cfg.get("perturb", 0.0), perturb_seed=cfg.get("perturb_seed"),
                          permute_seed=cfg.get("permute_seed"))


def kernel_bytes_per_elem(name, nsp, nfp):
    """Compulsory HBM bytes per element of each kernel family (each value touched once).

    d is the word size; geometry is 24 words per hexahedron (the 8 corners) and 10
    per tetrahedron (the affine map), connectivity 2 int32 per face.  NS uses the
    one-sided LDG switch (beta = 1/2): the gradient kernel reads the neighbour's
    solution trace only on faces where the element is the right side and stores
    gradient traces only there (half of the flux points); the face kernel reads one
    gradient trace per flux point pair, i.e. the stored half.  Curved hexahedra ("_cur")
    read stored metric terms instead of the 24 corner words: S rows and 1/J at the
    solution points (10 words each) where a kernel forms fluxes or gradients there,
    row d of S at the flux points (3 words each) where it forms common fluxes (the
    face kernel forms each pair's flux once, from the left side: half of them).  Curved
    tetrahedra read S and J per solution point (10 words) instead of per element, and the
    stored scaled normal (3 words) at each flux point where they form a common flux, with
    the same decomposition as straight ones otherwise."""
    fam = name.rsplit("_p", 1)[0] if "_p" in name else name
    d = 8
    if fam.endswith("_f32"):
        fam, d = fam[:-4], 4
    if fam.endswith("_cur"):
        base = fam[:-4]
        if base.startswith("tet_"):
            words = ({"tet_div_euler": 10 * nsp, "tet_grad": 17 * nsp + 5 * nfp // 2,
                      "tet_div_ns": 22 * nsp + 5 * nfp} if d == 4 else
                     {"tet_div_euler": 10 * nsp, "tet_grad": 20 * nsp, "tet_div_ns": 25 * nsp}).get(base)
            if words is None:
                return None
            # the stored scaled normals where common fluxes are formed: every flux point in
            # the divergence, the formed pairs' (half) in the FP32 gradient
            normals = 3 * nfp if base != "tet_grad" else (3 * nfp // 2 if d == 4 else 0)
            return d * (words + 10 * nsp + normals) + 4 * 2 * 4
        plain = kernel_bytes_per_elem(base + ("_f32" if d == 4 else "") + "_p0", nsp, nfp)
        if plain is None:
            return None
        metric = {"hex_trace": 0, "hex_div_euler": 10 * nsp + 3 * nfp, "hex_grad": 10 * nsp,
                  "hex_face_ns": 3 * nfp // 2, "hex_div_ns": 10 * nsp}.get(base)
        geo = 0 if base == "hex_trace" else 24 * d
        return None if metric is None else plain - geo + d * metric
    hex_geo, hex_conn = 24 * d, 6 * 2 * 4
    tet_gc = 10 * d + 4 * 2 * 4
    pyr_gc = 10 * d + 5 * 2 * 4
    table = {
        "hex_trace": d * 5 * (nsp + nfp),
        "hex_div_euler": d * (5 * nsp + 5 * nfp + 5 * nsp) + hex_geo + hex_conn,
        "hex_grad": d * (5 * nsp + 5 * nfp // 2 + 15 * nsp + 15 * nfp // 2) + hex_geo + hex_conn,
        "hex_face_ns": d * (5 * nfp + 15 * nfp // 2 + 5 * nfp) + hex_geo + hex_conn,
        "hex_div_ns": d * (5 * nsp + 15 * nsp + 5 * nfp + 5 * nsp) + hex_geo,
        "tet_div_euler": d * (5 * nsp + 5 * nsp) + tet_gc,
        "tet_grad": d * (5 * nsp + 15 * nsp) + tet_gc,
        "tet_div_ns": d * (5 * nsp + 15 * nsp + 5 * nsp) + tet_gc,
        # pyramids: traces of u stored for every flux point (read by both sides); with the
        # one-sided switch the gradient traces are stored where the element is the right
        # side (half of the flux points) and read from there by both sides
        "pyr_trace": d * 5 * (nsp + nfp),
        "pyr_div_euler": d * (5 * nsp + 5 * nfp + 5 * nsp) + pyr_gc,
        "pyr_grad": d * (5 * nsp + 5 * nfp + 15 * nsp + 15 * nfp // 2) + pyr_gc,
        "pyr_div_ns": d * (5 * nsp + 15 * nsp + 5 * nfp + 15 * nfp // 2 + 5 * nsp) + pyr_gc,
    }
    if d == 4:
        # FP32 form, one-sided LDG: the gradient kernel stores the transformed viscous flux
        # S_i . f_v (12 values per point) instead of the gradient (15) and the common flux
        # of each flux-point pair once (half of the flux points); the divergence kernel
        # reads both, the common flux for all of its flux points
        table["tet_grad"] = d * (5 * nsp + 12 * nsp + 5 * nfp // 2) + tet_gc
        table["tet_div_ns"] = d * (5 * nsp + 12 * nsp + 5 * nsp + 5 * nfp) + tet_gc
    return table.get(fam)


def _family_hash(kernel, read):
    """Hash of the sources a kernel family is built from: its header, the shared physics,
    and the part of the library that configures and launches that family's kernels (the
    shared launch helpers at the head of the dispatch section and the family's own RHS
    driver; the block loop that calls the drivers is left out).  read(name) returns the
    bytes of a file of csrc/."""
    hdr = {"tet_": ("tet.hpp", "hex.hpp", "physics.hpp"),
           "pyr_": ("pyr.hpp", "hex.hpp", "physics.hpp")}.get(kernel[:4], ("hex.hpp", "physics.hpp"))
    h = hashlib.sha256()
    for f in hdr:
        h.update(read(f))
    lib = read("frmi.hip")
    start = lib.index(b"// ------------------------------------------------------------ hex dispatch")
    tet0 = lib.index(b"// CUR: curved tetrahedra, the metric stored per solution point")
    loop = lib.index(b"template <typename T, bool DEV>\nfr_status rhs_t(")
    pyr0 = lib.find(b"// Pyramids: traces, then")
    tet1 = pyr0 if 0 <= pyr0 < loop else loop
    h.update(lib[start:tet0])
    if kernel.startswith("tet_"):
        h.update(lib[tet0:tet1])
    elif kernel.startswith("pyr_"):
        h.update(lib[pyr0:loop])
    return h.hexdigest()[:16]


def source_hash(kernel=""):
    csrc = os.path.join(ROOT, "paper_2408_16509_amd", "csrc")

    def read(f):
        with open(os.path.join(csrc, f), "rb") as fh:
            return fh.read()
    return _family_hash(kernel, read)


def load_traffic(kernel, workload):
    """Counter-measured HBM bytes per launch from profiles/traffic.json, if taken on this source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            db = json.load(fh)
        rec = db.get(f"{workload}:{kernel}")
        if rec and rec.get("source_hash") == source_hash(kernel):
            return rec.get("bytes_per_launch")
    except Exception:
        return None
    return None


def cpu_baseline(mesh, cfg, u_canon_fn):
    """The FP64 oracle on one full RHS of the same workload (host cores)."""
    import numpy as np
    from oracle import fr as ofr
    from oracle import mesh as omesh
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    bl = omesh.build(mesh, cfg["order"])
    u = [u_canon_fn(bl[0].xsol)]
    prm = ofr.Params(system=cfg["system"], riemann=cfg["riemann"])
    t0 = time.perf_counter()
    R = ofr.rhs(bl, u, prm)
    dt = time.perf_counter() - t0
    dof = bl[0].J.size
    return {"value": dof / dt / 1e9, "unit": "GDoF/s", "cores": int(threads), "kind": "oracle",
            "sample": f"1 FP64 oracle RHS over the full mesh ({dof} points), mesh setup excluded, {dt:.1f} s"}, u, R


FILTER_MODES = {"": -1, "plain": 0, "learned": 1}


def run_form(form, cfg, mesh, ic, args, torch, np, frmi, inputs):
    """Time `args.steps` RK4 steps of one form "<precision>[:plain|:learned]" (the suffix
    turns the entropy filter on every stage state and new state on); per-kernel event
    timing.  The learned filter uses the trained weights in args.mlp_weights."""
    prec, _, fmode = form.partition(":")
    filter_mode = FILTER_MODES[fmode]
    kw = dict(system=cfg["system"], order=cfg["order"], riemann=cfg["riemann"])
    if prec in ("fp32", "bf16x3"):
        p0 = 1.0 / (1.4 * cfg["mach"] ** 2)
        kw.update(precision=frmi.FR_FP32 if prec == "fp32" else frmi.FR_FP32_BF16X3,
                  u_ref=(1.0, 0.0, 0.0, 0.0, p0 / 0.4))
    ctx = frmi.Context(mesh, **kw)
    lay = ctx.layout
    x = ctx.sol_points()
    canon, off, blocks = [], 0, {}
    for i in range(lay.n_types):
        n, s = lay.n_elem[i], lay.n_sp[i]
        canon.append(ic(x[off:off + n * s].reshape(n, s, 3)).ravel())
        off += n * s
        key = {frmi.FR_HEX: "hex", frmi.FR_TET: "tet", frmi.FR_PYR: "pyr"}[int(lay.etype[i])]
        blocks[key] = (int(n), int(s), int(lay.n_fp[i]))
    u0 = ctx.pack64(np.concatenate(canon))
    if filter_mode == 1:
        w = getattr(args, "mlp_weights", None)
        if w is None:
            raise RuntimeError("the learned form needs trained MLP weights")
        ctx.mlp_set_weights(*w)
    u = u0.clone()
    stream = torch.cuda.current_stream()
    # the warm-up and the timed steps each as one call advancing several steps (the FP32
    # deviation of the state then comes from the previous step's last update)
    if args.warmup > 0:
        ctx.rk_step(u, cfg["dt"], args.warmup, filter_mode=filter_mode)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    ev0.record(stream)
    ctx.rk_step(u, cfg["dt"], args.steps, filter_mode=filter_mode)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = ev0.elapsed_time(ev1) / args.steps
    res = {"ctx": ctx, "ms": ms, "wall": wall, "finite": ctx.check(u), "blocks": blocks,
           "u_final": ctx.unpack64(u), "steps_total": args.warmup + args.steps}
    # the right-hand side of the initial state (canonical FP64), for the form-to-form comparison
    r = ctx.new_native()
    ctx.rhs(ctx.pack(ctx.unpack64(u0)), r)
    res["rhs0"] = ctx.unpack_rhs(r)
    if filter_mode >= 0:
        # the filter on the final state (entropy bound from itself): how many elements it treats
        uf = u.clone()
        st = ctx.filter(uf, u, mode=filter_mode, stats=True)
        res["filter"] = {"mode": fmode, "candidates": int(st.n_candidates), "troubled": int(st.n_troubled),
                         "evals": int(st.n_evals)}
    if not args.no_kernel_timing:
        uk = u0.clone()
        ctx.profile(True)
        for _ in range(2):
            ctx.rk_step(uk, cfg["dt"], 1, filter_mode=filter_mode)
        res["times"] = ctx.profile_read()
        ctx.profile(False)
    return res


def run_adaptive_workload(cfg, args, torch, np, frmi, inputs):
    """Adaptive embedded-pair integration to t_end (per form): time to solution, RHS
    throughput, accepted / rejected steps; the same interval with fixed-dt RK4 beside it."""
    mesh = build_mesh(cfg, inputs)
    out_forms, dominant = {}, None
    dof = None
    for form in ("fp32", "fp64"):
        kw = dict(system=cfg["system"], order=cfg["order"], riemann=cfg["riemann"])
        if form == "fp32":
            p0 = 1.0 / (1.4 * cfg["mach"] ** 2)
            kw.update(precision=frmi.FR_FP32, u_ref=(1.0, 0.0, 0.0, 0.0, p0 / 0.4))
        ctx = frmi.Context(mesh, **kw)
        lay = ctx.layout
        E, nsp = lay.n_elem[0], lay.n_sp[0]
        dof = E * nsp
        x = ctx.sol_points().reshape(E, nsp, 3)
        u0 = ctx.pack64(np.moveaxis(inputs.tgv(x[..., 0], x[..., 1], x[..., 2], mach=cfg["mach"]), 0, 1).ravel())
        u = u0.clone()
        ctx.rk_adaptive(u, cfg["t_end"] / 4, cfg["dt"], atol=cfg["tol"], rtol=cfg["tol"])      # warm-up
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        u = u0.clone()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        st = ctx.rk_adaptive(u, cfg["t_end"], cfg["dt"], atol=cfg["tol"], rtol=cfg["tol"])
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_a = ev0.elapsed_time(ev1)
        uf = u.clone()
        n_fixed = int(round(cfg["t_end"] / cfg["dt"]))
        u = u0.clone()
        ev0.record(stream)
        ctx.rk_step(u, cfg["dt"], n_fixed)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_f = ev0.elapsed_time(ev1)
        diff = float(torch.linalg.norm(uf - u) / torch.linalg.norm(u - u0))
        out_forms[form] = {
            "gdof_s": round(dof * st.n_rhs / (ms_a * 1e-3) / 1e9, 4), "time_to_t_end_ms": round(ms_a, 3),
            "accepted": int(st.accepted), "rejected": int(st.rejected), "n_rhs": int(st.n_rhs),
            "mean_dt": cfg["t_end"] / max(int(st.accepted), 1), "dt_next": st.dt_next,
            "fixed_rk4": {"dt": cfg["dt"], "steps": n_fixed, "time_to_t_end_ms": round(ms_f, 3),
                          "gdof_s": round(dof * 4 * n_fixed / (ms_f * 1e-3) / 1e9, 4)},
            "state_change_rel_diff_adaptive_vs_rk4": diff,
        }
        if form == "fp32" and not args.no_kernel_timing:
            ctx.profile(True)
            u = u0.clone()
            ctx.rk_adaptive(u, 2 * cfg["dt"], cfg["dt"], atol=cfg["tol"], rtol=cfg["tol"])
            times = ctx.profile_read()
            ctx.profile(False)
            fam = {k: v for k, v in times.items() if kernel_bytes_per_elem(k, nsp, 96) is not None}
            dom = max(fam, key=lambda k: fam[k][1])
            launches, tot = fam[dom]
            avg = tot / launches
            by = kernel_bytes_per_elem(dom, nsp, 96) * E
            dominant = {"bound": "hbm", "achieved": round(by / (avg * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(by / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                        "traffic": load_traffic(dom, "ns_tgv_hex32_p3"), "kernel": dom,
                        "avg_launch_ms": round(avg, 4), "bytes_per_launch": int(by)}
        ctx.close()
    head = out_forms["fp32"]
    return {
        "metric": "RHS GDoF/s (FP32/learned vs FP64 plain) at stated L2 error; % HBM roofline",
        "value": head["gdof_s"], "unit": "GDoF/s", "n_gpus": 1, "steps": head["accepted"], "warmup": 1,
        "ms_per_step": round(head["time_to_t_end_ms"] / max(head["accepted"], 1), 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.config, "elements": int(dof // 64), "order": cfg["order"], "dof": int(dof),
                   "integrator": "RK3(2)4[2R+] embedded pair, adaptive", "t_end": cfg["t_end"],
                   "atol": cfg["tol"], "rtol": cfg["tol"], "dt0": cfg["dt"], "form": "fp32"},
        "roofline": dominant,
        "forms": out_forms,
    }


def run_filter_workload(cfg, args, torch, np, frmi, inputs):
    """Shock workload with the entropy filter (FP64 form): train the warm-start MLP on
    held-out draws, then time filtered RK4 steps with the plain and the learned search
    on the measured draw; compare the dyadic indices both searches return and count
    constraint evaluations per troubled element."""
    mesh = inputs.hex_box(cfg["n"])
    ctx = frmi.Context(mesh, system=cfg["system"], order=cfg["order"], riemann=cfg["riemann"])
    lay = ctx.layout
    E, nsp, nfp = lay.n_elem[0], lay.n_sp[0], lay.n_fp[0]
    x = ctx.sol_points().reshape(E, nsp, 3)

    def ic(o_seed, n_seed):
        s_ = inputs.shock(x[..., 0], x[..., 1], x[..., 2], orient_seed=o_seed, noise_seed=n_seed)
        u = ctx.pack64(np.moveaxis(s_, 0, 1).copy().ravel())
        ctx.filter(u, u, mode=0)
        return u

    dt = cfg["dt"]
    # training data: the plain filter's (features, dyadic index) rows from held-out draws
    t0 = time.perf_counter()
    xs, ks = [], []
    for sd in cfg["train_seeds"]:
        X, K = ctx.mlp_collect(ic(sd, sd + 100), dt, cfg["train_steps"], cap=4_000_000)
        xs.append(X[K > 0])
        ks.append(K[K > 0])
    X = torch.cat(xs).contiguous()
    y = (torch.log2(torch.cat(ks).double()) / 20.0).float().contiguous()
    Xv, Kv = ctx.mlp_collect(ic(cfg["val_seed"], cfg["val_seed"] + 100), dt, 10, cap=1_000_000)
    Xv, yv = Xv[Kv > 0].contiguous(), (torch.log2(Kv[Kv > 0].double()) / 20.0).float()
    Xn = X.double()
    ctx.mlp_set_weights(inputs.mlp_glorot(43), Xn.mean(0).cpu().numpy(), (Xn.std(0) + 1e-6).cpu().numpy())
    iters = cfg["train_iters"]
    rows = torch.tensor(inputs.minibatch_rows(X.shape[0], 256, iters, 44), device="cuda")
    hist = ctx.mlp_train(X, y, rows, iters, 256).cpu().numpy()
    val = float(((ctx.mlp_forward(Xv) - yv) ** 2).mean()) if Xv.shape[0] else None
    train_s = time.perf_counter() - t0
    # measured draw
    u0 = ic(cfg["orient_seed"], cfg["noise_seed"])
    for _ in range(args.warmup):
        ctx.rk_step(u0, dt, 1, filter_mode=0)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    # the FP32 deviation form about the pre-shock state, same mesh and trained weights
    ctx32 = frmi.Context(mesh, system=cfg["system"], order=cfg["order"], riemann=cfg["riemann"],
                         precision=frmi.FR_FP32, u_ref=(1.0, 0.0, 0.0, 0.0, 1.0 / 0.4))
    ctx32.mlp_set_weights(ctx.mlp_get_weights(), Xn.mean(0).cpu().numpy(), (Xn.std(0) + 1e-6).cpu().numpy())
    runs = {}
    for cx, form in ((ctx, "fp64"), (ctx32, "fp32")):
        for mode, name in ((0, "plain"), (1, "mlp")):
            u = u0.clone()
            torch.cuda.synchronize()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            cx.rk_step(u, dt, args.steps, filter_mode=mode)      # one integrator call for the timed steps
            ev1.record(stream)
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1) / args.steps
            uk = u0.clone()
            cx.profile(True)
            for _ in range(2):
                cx.rk_step(uk, dt, 1, filter_mode=mode)
            times = cx.profile_read()
            cx.profile(False)
            runs[f"{form}_{name}"] = {"ms": ms, "u": u, "times": times, "finite": cx.check(u)}
    ref_u = runs["fp64_plain"]["u"]
    for k_, r_ in runs.items():
        r_["sol_rel_l2_vs_fp64_plain"] = float(torch.linalg.norm(r_["u"] - ref_u) / torch.linalg.norm(ref_u))
    # filter statistics on stage-like states: one unfiltered step from points of the trajectory
    probe = {"plain": [0, 0, 0, 0], "mlp": [0, 0, 0, 0]}
    k_equal, k_total, filt_ms = 0, 0, {"plain": [], "mlp": []}
    u = u0.clone()
    for i in range(5):
        for _ in range(max(1, args.steps // 5)):
            ctx.rk_step(u, dt, 1, filter_mode=0)
        us = u.clone()
        ctx.rk_step(us, dt, 1, filter_mode=-1)
        kk = {}
        for mode, name in ((0, "plain"), (1, "mlp")):
            uu = us.clone()
            k = torch.zeros(E, dtype=torch.int32, device="cuda")
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            ev0.record(stream)
            ctx.filter(uu, u, mode=mode, k=k)
            ev1.record(stream)
            st = ctx.filter(us.clone(), u, mode=mode, stats=True)
            filt_ms[name].append(ev0.elapsed_time(ev1))
            probe[name][0] += st.n_troubled
            probe[name][1] += st.n_evals
            probe[name][2] += st.n_fallback
            probe[name][3] += st.n_candidates
            kk[name] = k
        touched = (kk["plain"] != 0) | (kk["mlp"] != 0)
        k_equal += int(((kk["plain"] == kk["mlp"]) & touched).sum())
        k_total += int(touched.sum())
    dof = E * nsp
    gd = {n: 4 * dof / (r["ms"] * 1e-3) / 1e9 for n, r in runs.items()}
    head = runs["fp32_mlp"]
    out = {
        "metric": "RHS GDoF/s (FP32/learned vs FP64 plain) at stated L2 error; % HBM roofline",
        "value": round(gd["fp32_mlp"], 4), "unit": "GDoF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(head["ms"], 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.config, "elements": int(E), "order": cfg["order"], "points_per_elem": int(nsp),
                   "dof": int(dof), "rhs_per_step": 4,
                   "form": "fp32 deviation form (FP64 stage states, accumulation and filter checks), "
                           "entropy filter on every stage, learned warm start",
                   "state_finite_after": bool(all(r["finite"] for r in runs.values()))},
        "speedup_vs_fp64_plain": round(gd["fp32_mlp"] / gd["fp64_plain"], 4),
        "forms": {},
        "filter": {
            "train_rows": int(X.shape[0]), "train_iters": iters, "train_s": round(train_s, 2),
            "loss_first_last": [float(hist[:20].mean()), float(hist[-20:].mean())], "val_mse": val,
            "k_identical_fraction_troubled": k_equal / max(k_total, 1),
        },
    }
    for n, r in runs.items():
        out["forms"][n] = {
            "gdof_s": round(gd[n], 4), "ms_per_step": round(r["ms"], 4),
            "solution_rel_l2_vs_fp64_plain_after_steps": r["sol_rel_l2_vs_fp64_plain"],
            "kernels_ms_per_step": {k: round(v[1] / 2, 4) for k, v in sorted(r["times"].items())}}
    for n in ("plain", "mlp"):
        tr, ev, fb, cand = probe[n]
        out["filter"][n] = {"troubled_per_call": tr / 5, "candidates_per_call": cand / 5,
                            "evals_per_troubled": round(ev / max(tr, 1), 3),
                            "fallback_per_call": fb / 5, "filter_call_ms": round(float(np.mean(filt_ms[n])), 4)}
    times = head["times"]
    fam = {k: v for k, v in times.items() if kernel_bytes_per_elem(k, nsp, nfp) is not None}
    dom = max(fam, key=lambda k: fam[k][1])
    launches, tot = fam[dom]
    avg_ms = tot / launches
    by = kernel_bytes_per_elem(dom, nsp, nfp) * E
    achieved = by / (avg_ms * 1e-3) / 1e9
    out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": load_traffic(dom, args.config),
                       "kernel": dom, "avg_launch_ms": round(avg_ms, 4), "bytes_per_launch": int(by)}
    return out


def _per_var_err(a, b, blocks, torch):
    """Relative L2 error per conservative variable of canonical arrays (blocks of
    [n][5][nsp], in block order)."""
    num = torch.zeros(5, dtype=torch.float64, device=a.device)
    den = torch.zeros(5, dtype=torch.float64, device=a.device)
    o = 0
    for key in ("hex", "tet", "pyr"):
        if key not in blocks:
            continue
        n, s, _ = blocks[key]
        x = a[o:o + n * 5 * s].view(n, 5, s)
        y = b[o:o + n * 5 * s].view(n, 5, s)
        num += ((x - y) ** 2).sum(dim=(0, 2))
        den += (y ** 2).sum(dim=(0, 2))
        o += n * 5 * s
    return [float(v) for v in torch.sqrt(num / den).cpu()]


M0_BYTES_PER_DOF = {"f64": 80, "f32": 40}      # read u + write R once per RHS (FP64 / FP32 form)
M1_BYTES_PER_DOF = {"f64": 320, "f32": 160}    # NS fused in two phases: the gradient round trip added
ERR_TARGET_PER_RHS = 1e-5


def train_mixed_mlp(cfg, torch, np, frmi, inputs):
    """Warm-start MLP for the mixed workload: the plain filter's (features, dyadic index)
    rows of a few filtered RK4 steps of a Mach-3 shock on a small mixed mesh of the same
    element types, orders and equations (FP64 context), then Adam on the device."""
    tr = cfg["mlp_train"]
    t0 = time.perf_counter()
    small = dict(cfg, n=tr["n"])
    mesh = build_mesh(small, inputs)
    ctx = frmi.Context(mesh, system=cfg["system"], order=cfg["order"], riemann=frmi.FR_HLLC)
    lay = ctx.layout
    x = ctx.sol_points()
    xs, ks = [], []
    for sd in tr["seeds"]:
        canon, off = [], 0
        for i in range(lay.n_types):
            n, sp = lay.n_elem[i], lay.n_sp[i]
            xx = x[off:off + n * sp].reshape(n, sp, 3)
            s_ = inputs.shock(xx[..., 0], xx[..., 1], xx[..., 2], orient_seed=sd, noise_seed=sd + 100)
            canon.append(np.moveaxis(s_, 0, 1).ravel())
            off += n * sp
        u = ctx.pack64(np.concatenate(canon))
        ctx.filter(u, u, mode=0)
        X, K = ctx.mlp_collect(u, tr["dt"], tr["steps"], cap=2_000_000)
        xs.append(X[K > 0])
        ks.append(K[K > 0])
    X = torch.cat(xs).contiguous()
    y = (torch.log2(torch.cat(ks).double()) / 20.0).float().contiguous()
    Xn = X.double()
    mean, std = Xn.mean(0).cpu().numpy(), (Xn.std(0) + 1e-6).cpu().numpy()
    ctx.mlp_set_weights(inputs.mlp_glorot(43), mean, std)
    rows = torch.tensor(inputs.minibatch_rows(X.shape[0], 256, tr["iters"], 44), device="cuda")
    hist = ctx.mlp_train(X, y, rows, tr["iters"], 256).cpu().numpy()
    w = ctx.mlp_get_weights()
    ctx.close()
    info = {"rows": int(X.shape[0]), "iters": tr["iters"], "seconds": round(time.perf_counter() - t0, 2),
            "loss_first_last": [float(hist[:20].mean()), float(hist[-20:].mean())],
            "data": f"Mach-3 shock on two {tr['n'][0]}x{tr['n'][1]}x{tr['n'][2]} boxes (hex p=4, tet p=4), "
                    f"orientation seeds {list(tr['seeds'])}, {tr['steps']} filtered RK4 steps each"}
    return (w, mean, std), info


def oracle_threads():
    try:
        from threadpoolctl import threadpool_info
        return int(max([t.get("num_threads", 1) for t in threadpool_info()] or [1]))
    except Exception:
        return int(os.cpu_count() or 1)


def cpu_baseline_sample(cfg, inputs):
    """The FP64 oracle on a bounded sample of the workload: the same construction (element
    types, orders, perturbation, permutation, equations, initial condition) at the sample's
    cell counts; median of 5 right-hand sides after one untimed, mesh setup excluded."""
    import numpy as np
    from oracle import fr as ofr
    from oracle import mesh as omesh
    small = dict(cfg, n=cfg["oracle_sample"])
    mesh = build_mesh(small, inputs)
    bl = omesh.build(mesh, cfg["order"])
    u = [np.moveaxis(inputs.tgv(b.xsol[..., 0], b.xsol[..., 1], b.xsol[..., 2], mach=cfg["mach"]), 0, 1).copy()
         for b in bl]
    prm = ofr.Params(system=cfg["system"], riemann=cfg["riemann"])
    ofr.rhs(bl, u, prm)
    ts = []
    for _ in range(5):
        t0 = time.perf_counter()
        ofr.rhs(bl, u, prm)
        ts.append(time.perf_counter() - t0)
    t = float(np.median(ts))
    dof = sum(b.J.size for b in bl)
    n = cfg["oracle_sample"]
    kinds = ", ".join(f"{len(b.elems)} {('hexahedra', 'tetrahedra', 'pyramids')[b.etype]}" for b in bl)
    return {"value": dof / t / 1e9, "unit": "GDoF/s", "cores": oracle_threads(), "kind": "oracle",
            "sample": f"FP64 oracle RHS on the workload built at {n[0]}x{n[1]}x{n[2]} cells per box ({kinds}, "
                      f"{dof} points), median of 5 ({t:.2f} s each), mesh setup excluded"}


def roofline_for(times, blocks, form):
    """Dominant kernel (most time per step) of a form: the algorithmic-minimum bytes of the
    right-hand side (read u, write R once: the minimum M0) for the points of the
    element block it processes, per launch, against the HBM peak; the kernel's own
    compulsory bytes (this implementation's decomposition) as separate fields."""
    dtype = "f64" if form.split(":")[0] == "fp64" else "f32"

    def block_of(k):
        return blocks.get(k.split("_", 1)[0])
    fam = {k: v for k, v in times.items() if block_of(k) is not None
           and kernel_bytes_per_elem(k, block_of(k)[1], block_of(k)[2]) is not None}
    dom = max(fam, key=lambda k: fam[k][1])
    launches, tot = fam[dom]
    avg_ms = tot / launches
    n, nsp, nfp = block_of(dom)
    m0 = M0_BYTES_PER_DOF[dtype] * n * nsp
    impl = kernel_bytes_per_elem(dom, nsp, nfp) * n
    ach = m0 / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
            "avg_launch_ms": round(avg_ms, 4), "bytes_per_launch_m0": int(m0),
            "kernel_model_bytes_per_launch": int(impl),
            "kernel_model_achieved_gbs": round(impl / (avg_ms * 1e-3) / 1e9, 1),
            "kernel_model_frac": round(impl / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def run_tgv_workload(name, cfg, forms, args, torch, np, frmi, inputs, with_cpu=True):
    """Time the forms of a Taylor--Green workload; errors of each reduced form against the FP64
    form; dominant-kernel roofline; optionally the oracle on a sample (or the full mesh)."""
    mesh = build_mesh(cfg, inputs)

    def ic(xsol):
        s_ = inputs.tgv(xsol[..., 0], xsol[..., 1], xsol[..., 2], mach=cfg["mach"])
        return np.moveaxis(s_, 0, 1).copy()

    mlp_info = None
    if any(f.endswith(":learned") for f in forms):
        args.mlp_weights, mlp_info = train_mixed_mlp(cfg, torch, np, frmi, inputs)
    runs = {f: run_form(f, cfg, mesh, ic, args, torch, np, frmi, inputs) for f in forms}
    head = runs[forms[0]]
    blocks = head["blocks"]
    E = sum(b[0] for b in blocks.values())
    dof = sum(b[0] * b[1] for b in blocks.values())
    gdofs = {f: 4 * dof / (r["ms"] * 1e-3) / 1e9 for f, r in runs.items()}
    dt0 = forms[0].split(":")[0]
    out = {
        "metric": "RHS GDoF/s (FP32/learned vs FP64 plain) at stated L2 error; % HBM roofline",
        "value": round(gdofs[forms[0]], 4), "unit": "GDoF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(head["ms"], 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp32": "f32", "bf16x3": "f32+bf16x3"}.get(dt0, "f64"),
        "data": "synthetic",
        "config": {"workload": name, "elements": int(E), "order": cfg["order"],
                   "blocks": {k: {"elements": v[0], "points_per_elem": v[1]} for k, v in blocks.items()},
                   "dof": int(dof), "rhs_per_step": 4, "form": forms[0],
                   "rk_accumulation": "f64", "state_finite_after": bool(head["finite"]),
                   "wall_s_timed": round(head["wall"], 3)},
        "forms": {f: {"gdof_s": round(gdofs[f], 4), "ms_per_step": round(runs[f]["ms"], 4),
                      "timed_s": round(runs[f]["ms"] * args.steps * 1e-3, 3)} for f in forms},
    }
    fp64_forms = [f for f in forms if f.split(":")[0] == "fp64"]
    if fp64_forms and forms[0] != fp64_forms[0]:
        out["speedup_vs_" + fp64_forms[0].replace(":", "_")] = round(gdofs[forms[0]] / gdofs[fp64_forms[0]], 4)
    if mlp_info is not None:
        out["mlp_training"] = mlp_info
    for f in forms:
        if "filter" in runs[f]:
            fs = dict(runs[f]["filter"])
            fs["state"] = ("idle: no element of this smooth state fails the checks, so the timed cost is the "
                           "entropy-bound and detection passes" if fs["candidates"] == 0 else "active")
            out["forms"][f]["filter_on_final_state"] = fs
    # each reduced-precision form against the first FP64 form of the same run (the FP64 form
    # is the one the parity tests pin to the oracle): the RHS of the initial state per
    # variable against the 1e-5 target, and the solution after the same number of RK4 steps
    ref = fp64_forms[0] if fp64_forms else None
    if ref is not None:
        r64, u64 = runs[ref]["rhs0"], runs[ref]["u_final"]
        for f in forms:
            if f.split(":")[0] == "fp64":
                continue
            rr, uu = runs[f]["rhs0"], runs[f]["u_final"]
            pv = _per_var_err(rr, r64, runs[f]["blocks"], torch)
            o = out["forms"][f]
            o["rhs_rel_l2_vs_fp64_form"] = float(torch.linalg.norm(rr - r64) / torch.linalg.norm(r64))
            o["rhs_rel_l2_vs_fp64_form_per_var"] = pv
            o["rhs_meets_1e-5_per_var"] = [v <= ERR_TARGET_PER_RHS for v in pv]
            bound = STATED_RHS_BOUND.get((name, f.split(":")[0]))
            if bound is not None:
                o["rhs_stated_bound_per_var"] = bound
                o["rhs_within_stated_bound"] = bool(all(v <= b for v, b in zip(pv, bound)))
            o["solution_rel_l2_vs_fp64_form"] = {
                "against": ref, "steps": runs[f]["steps_total"],
                "value": float(torch.linalg.norm(uu - u64) / torch.linalg.norm(u64))}
    if not args.no_kernel_timing:
        out["roofline"] = roofline_for(head["times"], blocks, forms[0])
        out["roofline"]["traffic"] = load_traffic(out["roofline"]["kernel"], name)
        for f in forms:
            out["forms"][f]["kernels_ms_per_step"] = {k: round(v[1] / 2, 4)
                                                       for k, v in sorted(runs[f]["times"].items())}
            dtype = "f64" if f.startswith("fp64") else "f32"
            rate = 4 * dof / (runs[f]["ms"] * 1e-3) / 1e9
            out["forms"][f]["rhs_m0_fraction"] = round(rate * M0_BYTES_PER_DOF[dtype] / HBM_PEAK_GBS, 4)
            if cfg["system"] == 1:
                out["forms"][f]["rhs_m1_fraction"] = round(rate * M1_BYTES_PER_DOF[dtype] / HBM_PEAK_GBS, 4)
            if f != forms[0]:
                out["forms"][f]["roofline"] = roofline_for(runs[f]["times"], blocks, f)
    if with_cpu and not args.no_cpu_baseline:
        if cfg.get("oracle_sample"):
            out["cpu_baseline"] = cpu_baseline_sample(cfg, inputs)
        elif cfg.get("oracle_ok", False):
            base, uo, Ro = cpu_baseline(mesh, cfg, ic)
            out["cpu_baseline"] = base
            for f in forms:
                ctx = runs[f]["ctx"]
                rg = ctx.new_native()
                ctx.rhs(ctx.pack(uo[0].ravel()), rg)
                got = ctx.unpack_rhs(rg).cpu().numpy().reshape(Ro[0].shape)
                err = np.sqrt(((got - Ro[0]) ** 2).sum(axis=(0, 2)) / (Ro[0] ** 2).sum(axis=(0, 2)))
                out["forms"][f]["rhs_rel_l2_vs_oracle"] = float(np.linalg.norm(got - Ro[0]) / np.linalg.norm(Ro[0]))
                out["forms"][f]["rhs_rel_l2_per_var"] = [float(v) for v in err]
        else:
            out["cpu_baseline"] = None
    for r in runs.values():
        r["ctx"].close()
    return out, mesh


# Stated per-variable bounds (rho, rho u, rho v, rho w, E) of the reduced forms' RHS against
# the FP64 form on the Ma 0.1 Taylor--Green workloads: the low-Mach residual cancels terms
# of size H0 = 250 in the energy (and through it in the density), so rho and E sit far
# above the 1e-5 target while the momentum stays near the arithmetic's own level.
STATED_RHS_BOUND = {
    ("ns_tgv_mixed_c5split_p4", "fp32"): [5e-2, 2e-3, 2e-3, 2e-3, 5e-2],
    ("ns_tgv_mixed_c5split_p4", "bf16x3"): [1.0, 5e-2, 5e-2, 5e-2, 1.0],
    ("ns_tgv_hex32_p3", "fp32"): [5e-3, 5e-4, 5e-4, 5e-4, 5e-3],
    ("ns_tgv_tet32_q4_curved", "fp32"): [5e-2, 2e-3, 2e-3, 2e-3, 5e-2],
    ("ns_tgv_pyr24_p4", "fp32"): [5e-2, 2e-3, 2e-3, 2e-3, 5e-2],
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="ns_tgv_mixed_c5split_p4", choices=sorted(CONFIGS))
    ap.add_argument("--forms", default=None,
                    help="forms to time: fp32, fp64 or bf16x3, each optionally with :plain or :learned "
                         "(entropy filter on); the first is the headline (default: the workload's own)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the extra workloads of the default run (32^3 p=3 hexahedra, pyramids, 48^3 shock)")
    ap.add_argument("--stream-probe", action="store_true",
                    help="only measure the HBM streaming ceiling: read-only, write-only, copy and 2:1 passes "
                         "(hand-written kernels in libfrprobe.so, 1 GiB buffers, several grid sizes)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (scale for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(how the path would shard over GPUs is described, not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.stream_probe:
        import ctypes
        torch.cuda.set_device(0)
        lib = ctypes.CDLL(os.path.join(ROOT, "paper_2408_16509_amd", "libfrprobe.so"))
        lib.frprobe_stream.restype = ctypes.c_int
        lib.frprobe_stream.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
        res = {}
        for grid in (1024, 2048, 4096, 8192, 16384):
            out = (ctypes.c_double * 5)()
            rc = lib.frprobe_stream(1 << 30, 5, grid, out)
            if rc != 0:
                raise RuntimeError(f"stream probe failed with HIP error {rc}")
            res[grid] = {"read_gbs": round(out[0], 1), "write_gbs": round(out[1], 1), "copy_gbs": round(out[2], 1),
                         "read2_write1_gbs": round(out[3], 1)}
        best = {k: max(r[k] for r in res.values()) for k in ("read_gbs", "write_gbs", "copy_gbs", "read2_write1_gbs")}
        print(json.dumps({"stream_probe": {"buffer_bytes": 1 << 30, "by_grid": res, "best": best,
                                           "peak_gbs": HBM_PEAK_GBS}}), flush=True)
        return
    if args.copy_calibration:
        torch.cuda.set_device(0)
        n = 1 << 28
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read": 4 * n, "bytes_written": 4 * n, "launches": 5}}), flush=True)
        return

    from paper_2408_16509_amd import frmi, inputs

    cfg = CONFIGS[args.config]
    torch.cuda.set_device(0)
    if cfg.get("filter"):
        print(json.dumps(run_filter_workload(cfg, args, torch, np, frmi, inputs)), flush=True)
        return
    if cfg.get("adaptive"):
        print(json.dumps(run_adaptive_workload(cfg, args, torch, np, frmi, inputs)), flush=True)
        return
    forms = [f.strip() for f in (args.forms or cfg.get("forms", "fp32,fp64")).split(",") if f.strip()]
    out, mesh = run_tgv_workload(args.config, cfg, forms, args, torch, np, frmi, inputs)
    if cfg.get("kind") in ("curved", "curved_tet"):
        # a uniform stream on the same curved mesh, both metrics (FP64): the conservative
        # metric keeps it (R at rounding level), the cross-product metric does not once its
        # degree exceeds the solution order (Sec. "Curved elements", Fig. fsp)
        fs = {}
        for name, code in (("conservative", frmi.FR_METRIC_CONSERVATIVE), ("cross", frmi.FR_METRIC_CROSS)):
            ctx = frmi.Context(mesh, system=cfg["system"], order=cfg["order"], riemann=cfg["riemann"],
                               hex_metric=code)
            canon = np.empty((ctx.layout.canon_len // 5 // ctx.layout.n_sp[0], 5, ctx.layout.n_sp[0]))
            canon[:, 0], canon[:, 1], canon[:, 2], canon[:, 3], canon[:, 4] = 1.2, 0.3, -0.2, 0.5, 2.5
            r = ctx.new_native()
            ctx.rhs(ctx.pack(canon.ravel()), r)
            fs[name] = float(torch.max(torch.abs(ctx.unpack_rhs(r))).item())
            ctx.close()
        out["free_stream_max_abs_rhs"] = fs
    del mesh
    if args.config == "ns_tgv_mixed_c5split_p4" and not args.no_extras and args.forms is None:
        # the other two headline-adjacent workloads, each with its own forms, as extra keys
        extras = {}
        sub = argparse.Namespace(**vars(args))
        sub.steps, sub.warmup = max(args.steps, 20), min(args.warmup, 3)
        c2 = CONFIGS["ns_tgv_hex32_p3"]
        extras["ns_tgv_hex32_p3"] = run_tgv_workload("ns_tgv_hex32_p3", c2, ["fp32", "fp64"], sub, torch, np,
                                                     frmi, inputs, with_cpu=False)[0]
        extras["ns_tgv_pyr24_p4"] = run_tgv_workload("ns_tgv_pyr24_p4", CONFIGS["ns_tgv_pyr24_p4"], ["fp32", "fp64"],
                                                     sub, torch, np, frmi, inputs, with_cpu=False)[0]
        sub.config = "euler_shock_hex48_p3"          # the workload the traffic records are keyed by
        extras["euler_shock_hex48_p3"] = run_filter_workload(CONFIGS["euler_shock_hex48_p3"], sub, torch, np,
                                                             frmi, inputs)
        for v in extras.values():
            for k in ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data", "unit"):
                v.pop(k, None)
        out["extra_workloads"] = extras
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
