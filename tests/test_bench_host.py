"""Host-side logic of bench.py and of the cost model (no GPU): the one-GPU
refusal, the source-hash gate on stored HBM traffic, the algorithmic byte
and FP64 counts, and the CPU baseline's record."""
import os
import subprocess
import sys

import pytest

from paper_2403_13287_amd import costs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _profile(tmp_path, sha, traffic="4.8750e+08"):
    p = tmp_path / "k_flux.txt"
    p.write_text("# summary\n"
                 f"kernel_source_sha256: {sha}\n"
                 f"flux_hbm_bytes_per_launch: {traffic}\n")
    return str(p)


def test_stored_traffic_only_for_the_profiled_sources(tmp_path):
    sha = costs.kernel_source_hash()
    assert len(sha) == 64
    assert costs.stored_flux_traffic(_profile(tmp_path, sha)) == pytest.approx(4.875e8)
    assert costs.stored_flux_traffic(_profile(tmp_path, "0" * 64)) is None
    assert costs.stored_flux_traffic(str(tmp_path / "missing.txt")) is None
    assert costs.stored_flux_traffic(_profile(tmp_path, sha, "n/a")) is None


def test_source_hash_covers_the_forward_sources_only(tmp_path):
    """The hash changes with any forward source and ignores other files."""
    base = costs.kernel_source_hash()
    for rel in costs.FORWARD_SOURCES:
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        dst.write_bytes(open(os.path.join(ROOT, rel), "rb").read())
    assert costs.kernel_source_hash(str(tmp_path)) == base
    (tmp_path / "paper_2403_13287_amd" / "csrc" / "lskum_adjoint.hip").write_text("// other")
    assert costs.kernel_source_hash(str(tmp_path)) == base
    for rel in costs.FORWARD_SOURCES:
        p = tmp_path / rel
        data = p.read_bytes()
        p.write_bytes(data + b"\n")
        assert costs.kernel_source_hash(str(tmp_path)) != base, rel
        p.write_bytes(data)


def test_cost_model_counts():
    n, edges, kp = 1_000_000, 29_967_646, 32
    assert costs.conn_bytes(kp) == 132
    assert costs.flux_bytes(n, kp) == n * (33 + 32 + 64 + 64 + 64 + 32 + 132)
    assert costs.flux_bytes(n, kp) == pytest.approx(4.21e8)
    # the SSP stage in the flux epilogue: U, dt in; U, q_next out; U^n read
    # at one stage in 4 and written at another
    assert costs.flux_bytes(n, kp, stage=True) - costs.flux_bytes(n, kp) == \
        n * (32 + 8 + 32 + 32 + 8 + 8)
    assert costs.flux_flops(n, edges) == pytest.approx(edges * costs.EDGE_FLOPS)
    assert costs.flux_flops(n, edges, stage=True) == pytest.approx(
        edges * costs.EDGE_FLOPS + n * costs.STAGE_FLOPS)
    assert 0 < costs.STAGE_FLOPS < costs.EDGE_FLOPS
    # one stage of the 1M workload, as reported in the bench line: fused
    # (SSP) and with separate q-variables and stage passes (RK4)
    assert costs.stage_bytes(n, kp, 3) / 1e9 == pytest.approx(1.916, abs=5e-4)
    assert costs.stage_bytes(n, kp, 3, fused=False) / 1e9 == pytest.approx(2.005, abs=5e-4)
    assert costs.stage_bytes(n, kp, 3, fused=False) - costs.stage_bytes(n, kp, 3) == \
        n * (64 + 145 - 120)
    # each inner sweep adds its own pass and nothing else
    step = costs.stage_bytes(n, kp, 4) - costs.stage_bytes(n, kp, 3)
    assert step == costs.stage_bytes(n, kp, 1) - costs.stage_bytes(n, kp, 0)
    assert step == n * (16 + 64 + 64 + 64 + 132)


def test_cpu_baseline_record(tiny_cloud):
    sys.path.insert(0, ROOT)
    import bench
    from cloudgen.workloads import WORKLOADS
    from oracle.ref import RK4, Oracle

    wl = WORKLOADS["tiny"]
    U0 = Oracle(tiny_cloud, wl.mach, wl.aoa_deg).init_state()
    for options in (0, RK4):
        r = bench.cpu_baseline(tiny_cloud, wl, U0, options, None, min_seconds=0.2)
        assert set(r) == {"value", "unit", "cores", "kind", "sample", "host", "all_cores"}
        assert r["kind"] == "oracle" and r["cores"] == 1
        assert r["unit"] == "point-stage updates/s" and r["value"] > 0
        assert "9600 points" in r["sample"]
        assert ("options 4" in r["sample"]) == (options == RK4)
        assert r["host"]["nproc"] == os.cpu_count() and r["host"]["cpus_available"] >= 1
        a = r["all_cores"]
        assert a["cores"] >= 1 and a["value"] > 0 and a["unit"] == r["unit"]
        assert a["kind"].startswith("oracle") and f"{a['cores']} threads" in a["sample"]
    r = bench.cpu_baseline(tiny_cloud, wl, U0, 0, None, min_seconds=0.1, all_cores=False)
    assert "all_cores" not in r
