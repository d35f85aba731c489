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
