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


def test_workloads_and_one_gpu_rule():
    for name in ("ns_tgv_hex32_p3", "euler_tgv_hex4_p2", "ns_tgv_mixed_c5split_p4", "euler_shock_hex48_p3",
                 "ns_tgv_hex32_p3_curved", "ns_tgv_hex32_p3_adaptive"):
        assert name in bench.CONFIGS
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in (r.stdout + r.stderr)
