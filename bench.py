#!/usr/bin/env python3
"""Throughput of the FR right-hand side on one MI355X.

Default workload: compressible Navier--Stokes Taylor--Green vortex (Re 1600,
Ma 0.1, Pr 0.71) on a periodic 32^3 mesh of straight hexahedra at p = 3
(64 Gauss--Legendre points per element, 2,097,152 points), LDG viscous terms,
Rusanov inviscid flux, FP64.  A step is one classical RK4 step (4 right-hand
sides + the stage updates) on the device-resident state; the metric counts
right-hand-side degrees of freedom (elements x solution points, the paper's DoF)
per second: GDoF/s = 4 * E * N_sp * steps / time / 1e9.

Also reported: the dominant kernel's achieved bandwidth (algorithmic bytes per
launch / HIP-event-measured launch time on the library's stream) against the
8 TB/s HBM peak, and the FP64 CPU oracle timed on the host on one full RHS.
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
    "ns_tgv_hex32_p3": dict(n=(32, 32, 32), order=3, system=1, riemann=0, mach=0.1, dt=4e-4),
    "euler_tgv_hex4_p2": dict(n=(4, 4, 4), order=2, system=0, riemann=0, mach=0.1, dt=1e-3),
    "ns_tgv_hex48pert_p4": dict(n=(48, 48, 48), order=4, system=1, riemann=0, mach=0.1, dt=1.5e-4,
                                perturb=0.1, perturb_seed=31, permute_seed=32),
}


def kernel_bytes_per_elem(name, nsp, nfp):
    """Compulsory HBM bytes per element of each kernel family (each value touched once).

    d is the word size; geometry is 24 words per hexahedron (the 8 corners) and 10
    per tetrahedron (the affine map), connectivity 2 int32 per face.  NS uses the
    one-sided LDG switch (beta = 1/2): the gradient kernel reads the neighbour's
    solution trace only on faces where the element is the right side and stores
    gradient traces only there (half of the flux points); the face kernel reads one
    gradient trace per flux point pair, i.e. the stored half."""
    fam = name.rsplit("_p", 1)[0] if "_p" in name else name
    d = 8
    if fam.endswith("_f32"):
        fam, d = fam[:-4], 4
    hex_geo, hex_conn = 24 * d, 6 * 2 * 4
    tet_gc = 10 * d + 4 * 2 * 4
    table = {
        "hex_trace": d * 5 * (nsp + nfp),
        "hex_div_euler": d * (5 * nsp + 5 * nfp + 5 * nsp) + hex_geo + hex_conn,
        "hex_grad": d * (5 * nsp + 5 * nfp // 2 + 15 * nsp + 15 * nfp // 2) + hex_geo + hex_conn,
        "hex_face_ns": d * (5 * nfp + 15 * nfp // 2 + 5 * nfp) + hex_geo + hex_conn,
        "hex_div_ns": d * (5 * nsp + 15 * nsp + 5 * nfp + 5 * nsp) + hex_geo,
        "tet_div_euler": d * (5 * nsp + 5 * nsp) + tet_gc,
        "tet_grad": d * (5 * nsp + 15 * nsp) + tet_gc,
        "tet_div_ns": d * (5 * nsp + 15 * nsp + 5 * nsp) + tet_gc,
    }
    return table.get(fam)


def source_hash():
    h = hashlib.sha256()
    for f in ("hex.hpp", "tet.hpp", "physics.hpp", "filter.hpp", "frmi.hip"):
        with open(os.path.join(ROOT, "paper_2408_16509_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload):
    """Counter-measured HBM bytes per launch from profiles/traffic.json, if taken on this source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            db = json.load(fh)
        rec = db.get(f"{workload}:{kernel}")
        if rec and rec.get("source_hash") == source_hash():
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


def run_form(form, cfg, mesh, ic, args, torch, np, frmi):
    """Time `args.steps` RK4 steps of one precision form; per-kernel event timing."""
    kw = dict(system=cfg["system"], order=cfg["order"], riemann=cfg["riemann"])
    if form == "fp32":
        p0 = 1.0 / (1.4 * cfg["mach"] ** 2)
        kw.update(precision=frmi.FR_FP32, u_ref=(1.0, 0.0, 0.0, 0.0, p0 / 0.4))
    ctx = frmi.Context(mesh, **kw)
    lay = ctx.layout
    E, nsp, nfp = lay.n_elem[0], lay.n_sp[0], lay.n_fp[0]
    x = ctx.sol_points().reshape(E, nsp, 3)
    u0 = ctx.pack64(ic(x).ravel())
    u = u0.clone()
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        ctx.rk_step(u, cfg["dt"], 1)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        ctx.rk_step(u, cfg["dt"], 1)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = ev0.elapsed_time(ev1) / args.steps
    res = {"ctx": ctx, "ms": ms, "wall": wall, "finite": ctx.check(u), "E": E, "nsp": nsp, "nfp": nfp}
    if not args.no_kernel_timing:
        uk = u0.clone()
        ctx.profile(True)
        for _ in range(2):
            ctx.rk_step(uk, cfg["dt"], 1)
        res["times"] = ctx.profile_read()
        ctx.profile(False)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="ns_tgv_hex32_p3", choices=sorted(CONFIGS))
    ap.add_argument("--forms", default="fp32,fp64", help="precision forms to time; the first is the headline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (scale for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU path is a design, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

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
    mesh = inputs.hex_box(cfg["n"], perturb=cfg.get("perturb", 0.0), perturb_seed=cfg.get("perturb_seed"),
                          permute_seed=cfg.get("permute_seed"))

    def ic(xsol):
        s = inputs.tgv(xsol[..., 0], xsol[..., 1], xsol[..., 2], mach=cfg["mach"])
        return np.moveaxis(s, 0, 1).copy()

    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    runs = {f: run_form(f, cfg, mesh, ic, args, torch, np, frmi) for f in forms}
    head = runs[forms[0]]
    E, nsp, nfp = head["E"], head["nsp"], head["nfp"]
    dof = E * nsp
    gdofs = {f: 4 * dof / (r["ms"] * 1e-3) / 1e9 for f, r in runs.items()}
    out = {
        "metric": "RHS GDoF/s (FP32/learned vs FP64 plain) at stated L2 error; % HBM roofline",
        "value": round(gdofs[forms[0]], 4), "unit": "GDoF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(head["ms"], 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if forms[0] == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": args.config, "elements": int(E), "order": cfg["order"], "points_per_elem": int(nsp),
                   "dof": int(dof), "rhs_per_step": 4, "form": forms[0],
                   "rk_accumulation": "f64", "state_finite_after": bool(head["finite"]),
                   "wall_s_timed": round(head["wall"], 3)},
        "forms": {f: {"gdof_s": round(gdofs[f], 4), "ms_per_step": round(runs[f]["ms"], 4)} for f in forms},
    }
    if not args.no_kernel_timing:
        times = head["times"]
        fam = {k: v for k, v in times.items() if kernel_bytes_per_elem(k, nsp, nfp) is not None}
        dom = max(fam, key=lambda k: fam[k][1])
        launches, tot = fam[dom]
        avg_ms = tot / launches
        by = kernel_bytes_per_elem(dom, nsp, nfp) * E
        achieved = by / (avg_ms * 1e-3) / 1e9
        traffic = load_traffic(dom, args.config)
        out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                           "kernel": dom, "avg_launch_ms": round(avg_ms, 4), "bytes_per_launch": int(by)}
        for f in forms:
            out["forms"][f]["kernels_ms_per_step"] = {k: round(v[1] / 2, 4) for k, v in sorted(runs[f]["times"].items())}
            bpd = 80 if f == "fp64" else 40
            out["forms"][f]["rhs_m0_fraction"] = round(4 * dof * bpd / (runs[f]["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    if not args.no_cpu_baseline:
        base, uo, Ro = cpu_baseline(mesh, cfg, ic)
        out["cpu_baseline"] = base
        for f in forms:
            ctx = runs[f]["ctx"]
            ug = ctx.pack(uo[0].ravel())
            rg = ctx.new_native()
            ctx.rhs(ug, rg)
            got = ctx.unpack_rhs(rg).cpu().numpy().reshape(Ro[0].shape)
            err = np.sqrt(((got - Ro[0]) ** 2).sum(axis=(0, 2)) / (Ro[0] ** 2).sum(axis=(0, 2)))
            out["forms"][f]["rhs_rel_l2_vs_oracle"] = float(np.linalg.norm(got - Ro[0]) / np.linalg.norm(Ro[0]))
            out["forms"][f]["rhs_rel_l2_per_var"] = [float(v) for v in err]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
