"""Host logic of bench.py (no GPU): the byte model behind roofline.achieved, the
counter lookup guard, the workload table and the one-GPU rule."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_byte_model_hex_p3():
    nsp, nfp = 64, 96
    # FP32 NS divergence: u, grad, common fluxes in, R out, 24 geometry words
    assert bench.kernel_bytes_per_elem("hex_div_ns_f32_p3", nsp, nfp) == 4 * (25 * nsp + 5 * nfp) + 24 * 4
    assert bench.kernel_bytes_per_elem("hex_div_ns_p3", nsp, nfp) == 8 * (25 * nsp + 5 * nfp) + 24 * 8
    assert bench.kernel_bytes_per_elem("hex_trace_f32_p3", nsp, nfp) == 4 * 5 * (nsp + nfp)
    assert bench.kernel_bytes_per_elem("k_unknown_p3", nsp, nfp) is None


def test_byte_model_curved_variants():
    nsp, nfp = 64, 96
    for fam, extra in (("hex_div_ns", 10 * nsp), ("hex_grad", 10 * nsp), ("hex_face_ns", 3 * nfp // 2),
                       ("hex_div_euler", 10 * nsp + 3 * nfp)):
        for d, sfx in ((4, "_f32"), (8, "")):
            plain = bench.kernel_bytes_per_elem(f"{fam}{sfx}_p3", nsp, nfp)
            cur = bench.kernel_bytes_per_elem(f"{fam}_cur{sfx}_p3", nsp, nfp)
            assert cur == plain - 24 * d + d * extra, (fam, sfx)
    # the trace kernel reads no geometry either way
    assert bench.kernel_bytes_per_elem("hex_trace_cur_f32_p3", nsp, nfp) == \
        bench.kernel_bytes_per_elem("hex_trace_f32_p3", nsp, nfp)


def test_traffic_only_for_current_sources(tmp_path, monkeypatch):
    # a record taken on other sources is not reported
    assert bench.load_traffic("hex_div_ns_f32_p3", "no_such_workload") is None
    h = bench.source_hash("hex_div_ns_f32_p3")
    assert len(h) == 16 and h == bench.source_hash("hex_grad_f32_p3")
    assert bench.source_hash("tet_grad_f32") != h
    # each family hashes its own header and RHS driver: pyramids differ from both
    assert bench.source_hash("pyr_div_ns_f32") not in (h, bench.source_hash("tet_grad_f32"))


def test_workloads_and_one_gpu_rule():
    for name in ("ns_tgv_hex32_p3", "euler_tgv_hex4_p2", "ns_tgv_mixed_c5split_p4", "euler_shock_hex48_p3",
                 "ns_tgv_hex32_p3_curved", "ns_tgv_hex32_p3_adaptive"):
        assert name in bench.CONFIGS
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in (r.stdout + r.stderr)


def test_roofline_uses_the_m0_bytes_of_the_dominant_kernels_block():
    blocks = {"hex": (131072, 125, 150), "tet": (786432, 35, 60)}
    times = {"tet_grad_f32": (8, 19.6), "hex_grad_f32_p4": (8, 7.3), "rk4_update_f32": (8, 30.0)}
    r = bench.roofline_for(times, blocks, "fp32:learned")
    assert r["kernel"] == "tet_grad_f32"
    m0 = 40 * 786432 * 35
    assert r["bytes_per_launch_m0"] == m0
    assert abs(r["achieved"] - m0 / (19.6 / 8 * 1e-3) / 1e9) < 0.1
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-4
    assert r["kernel_model_bytes_per_launch"] == bench.kernel_bytes_per_elem("tet_grad_f32", 35, 60) * 786432
    r64 = bench.roofline_for({"tet_grad": (8, 30.0)}, blocks, "fp64:plain")
    assert r64["bytes_per_launch_m0"] == 80 * 786432 * 35


def test_cpu_baseline_sample_runs_the_oracle():
    from paper_2408_16509_amd import inputs
    cfg = dict(bench.CONFIGS["ns_tgv_mixed_c5split_p4"], oracle_sample=(1, 2, 2))
    b = bench.cpu_baseline_sample(cfg, inputs)
    assert b["kind"] == "oracle" and b["unit"] == "GDoF/s" and b["value"] > 0 and b["cores"] >= 1
    assert "4 hexahedra" in b["sample"] and "24 tetrahedra" in b["sample"]
