"""The committed counter figures the benchmark reads (profiles/traffic.json)
are internally consistent: totals are read + write, each is the RK mix of
two stages with the base term f^n and one without, and reads and writes
follow from FETCH_SIZE / WRITE_SIZE by the factors of the copy calibration."""
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _entries():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        return json.load(fh)


@pytest.mark.parametrize("workload", ["wave2048", "spinodal4096", "channels"])
def test_traffic_entry_is_consistent(workload):
    e = _entries()[workload]
    assert len(e["kernel_hash"]) == 16
    tol = 2e-3
    assert e["bytes_per_launch"] == pytest.approx(e["read_bytes_per_launch"] + e["write_bytes_per_launch"], rel=tol)
    k = e["per_stage_kind"]
    for what in ("read", "write"):
        mix = (2 * k["with_fn"][what] + k["stage1"][what]) / 3
        assert e[f"{what}_bytes_per_launch"] == pytest.approx(mix, rel=tol)
    for kind in ("with_fn", "stage1"):
        assert k[kind]["read"] == pytest.approx(e["fetch_factor"] * e["fetch_kib_per_dispatch"][kind] * 1024, rel=tol)
        assert k[kind]["write"] == pytest.approx(e["write_factor"] * e["write_kib_per_dispatch"][kind] * 1024, rel=tol)
    # every read is a 128-byte request, counted as 64 bytes by FETCH_SIZE
    assert e["fetch_factor"] == pytest.approx(2.0, rel=1e-3)
    assert e["write_factor"] == pytest.approx(1.0, rel=1e-3)
    v = e["valu"]
    assert v["insts_per_launch"] > 0 and v["f64_flops_per_launch"] > 0
    # dual issue: at most one extra instruction per issue quad-cycle
    assert 0 <= v["dual_issue_quads_per_launch"] <= v["insts_per_launch"] / 2
    # the profiled launches' clock: GPU-active cycles per XCD over the dispatch time
    assert 0.5 < v["clock_ghz"] <= 2.4
    assert v["gui_cycles_per_xcd"] == pytest.approx(v["clock_ghz"] * 1e9 * v["profiled_launch_s"], rel=5e-3)
    assert os.path.exists(os.path.join(ROOT, v["source"]))
    assert os.path.exists(os.path.join(ROOT, e["source"]))
