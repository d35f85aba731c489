"""CPU checks of bench.py's host-side pieces (no device work): every named
workload has a kernel label and builds its oracle baseline sample, and the
counter-derived traffic is either a positive byte count or absent."""

import math

import pytest

import bench
import h2inputs


@pytest.mark.parametrize("name", sorted(h2inputs.WORKLOADS))
def test_every_workload_has_a_kernel_label(name):
    label = bench.kernel_label(h2inputs.WORKLOADS[name])
    assert "exp" in label if h2inputs.WORKLOADS[name].get("kernel") == "exp" else "|x-y|" in label


@pytest.mark.parametrize("name,exact", [("square1k", False), ("cube64k_exp", True)])
def test_cpu_baseline_record(name, exact):
    rec = bench.cpu_baseline(h2inputs.WORKLOADS[name], budget_s=0.2, exact=exact)
    assert set(rec) >= {"value", "unit", "cores", "kind", "sample", "host_cpus", "cpu_model"}
    assert rec["kind"] == "oracle" and rec["cores"] >= 1 and rec["unit"] == "RHS*N/s"
    assert rec["host_cpus"] >= 1 and rec["cpu_model"]
    assert rec["value"] > 0 and math.isfinite(rec["value"])
    assert ("exact factor" in rec["sample"]) == exact


def test_measured_traffic_is_bytes_or_absent():
    for name, label, *_ in bench.SCHUR_KERNELS:
        t = bench.measured_traffic("cube1m", label)
        assert t is None or t > 1e9
        assert bench.measured_traffic("cube256k", label) is None
    assert bench.measured_traffic("cube1m", "no such kernel") is None


def test_traffic_record_matches_the_sources():
    """The committed traffic summary was taken on the current Schur sources, so
    the bench reports it (a stale one would be dropped as null)."""
    got = bench.measured_traffic("cube1m", "schur_kernel<float, 1>")
    assert got is not None and got > 0


def _trace(tmp_path, rows):
    import csv
    with open(tmp_path / "t_kernel_trace.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        for name, a, b in rows:
            w.writerow([name, a, b])


def test_profsum_busy_unions_overlapping_kernels(tmp_path, capsys):
    """Occupancy of a phase: the window runs from the first start of a
    first-regex kernel (after the last after-regex kernel) to the last end of a
    last-regex kernel; overlapping kernels on different streams count once."""
    from paper_1705_04601_amd import profsum
    ms = 1_000_000
    _trace(tmp_path, [
        ("qr_kernel", 0, 1 * ms),            # an earlier phase, before the window
        ("inverse_kernel", 2 * ms, 3 * ms),  # window start
        ("schur_kernel<float, 0>", 3 * ms, 6 * ms),
        ("schur_kernel<float, 1>", 4 * ms, 5 * ms),  # inside the previous one
        ("schur_kernel<float, 0>", 7 * ms, 8 * ms),  # after a 1 ms gap; window end
        ("gemm_solve_lds_kernel<0, 2, 4>", 9 * ms, 10 * ms),  # later phase, outside
    ])
    profsum.busy(str(tmp_path), "t", "inverse_kernel", "schur_kernel", "qr_kernel")
    out = capsys.readouterr().out
    assert "over 6.0 ms" in out and "busy 5.0 ms (0.833)" in out and "idle 1.0 ms in 1 gaps" in out
