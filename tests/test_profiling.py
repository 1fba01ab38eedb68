"""The rocprofv3 summaries of profiles/ (paper_0812_1282_amd/profiling.py) on
synthetic databases with the tables rocprofv3 writes (`kernels`,
`pmc_events`): kernel-name parsing, the trace table, and the traffic
calibration against a copy of known size. CPU only."""
import json
import sqlite3

import pytest

from paper_0812_1282_amd import profiling as pf

SWEEP_F16 = "void lbm::sweep_kernel<2, 1, 512, false, true, 0>(lbm::View const*, int)"
SWEEP_F16_DIAG = "void lbm::sweep_kernel<2, 1, 512, true, true, 0>(lbm::View const*, int)"
SWEEP_F64_IP0 = "void lbm::sweep_kernel<0, 1, 1024, false, true, 1>(lbm::View const*, int)"
SWEEP_F64_IP1 = "void lbm::sweep_kernel<0, 1, 1024, false, true, 2>(lbm::View const*, int)"
BAND_F64_0 = "void lbm::band_kernel<0, 1, true>(lbm::View const*, int)"
BAND_F64_1 = "void lbm::band_kernel<0, 2, true>(lbm::View const*, int)"
COPY = "__amd_rocclr_copyBuffer"


def _db(path, kernels=(), pmc=()):
    con = sqlite3.connect(path)
    con.execute("create table kernels (name text, duration real)")
    con.execute("create table pmc_events (name text, counter_name text, counter_value real)")
    con.executemany("insert into kernels values (?, ?)", kernels)
    con.executemany("insert into pmc_events values (?, ?, ?)", pmc)
    con.commit()
    con.close()
    return str(path)


def test_sweep_names_parse_into_format_block_and_phase():
    assert pf.sweep_key(SWEEP_F16) == ("f16s", 1, 512, False, True)
    assert pf.sweep_key(SWEEP_F16_DIAG)[3] is True
    assert pf.sweep_key(SWEEP_F64_IP0)[0] == "f64ip"
    assert pf.short_name(SWEEP_F64_IP1) == "sweep f64ip MRT block 1024 phase 1 tau_phi=1"
    assert pf.short_name(SWEEP_F16_DIAG) == "sweep f16s MRT block 512 +diag tau_phi=1"
    assert pf.band_key(BAND_F64_1) == ("f64ip", 1)
    assert pf.sweep_key(COPY) is None and pf.band_key(COPY) is None


def test_trace_table_counts_sums_and_medians(tmp_path):
    ns = [140_000.0, 141_000.0, 139_000.0, 500_000.0]   # durations in ns
    db = _db(tmp_path / "t.db", kernels=[(SWEEP_F16, d) for d in ns] + [(COPY, 20_000.0)])
    text = pf.trace_summary(db, "cmd")
    row = [line for line in text.splitlines() if line.startswith("| sweep f16s")][0]
    cells = [c.strip() for c in row.strip("|").split("|")]
    assert cells[1] == "4"
    assert float(cells[2]) == pytest.approx(sum(ns) / 1e6, abs=1e-3)      # total ms
    assert float(cells[3]) == pytest.approx(sum(ns) / 4 / 1e3, abs=1e-2)  # average us
    assert float(cells[4]) == pytest.approx(141.0, abs=1e-2)             # median us
    # sorted by total time: the sweep first
    assert text.splitlines()[6].startswith("| sweep f16s")


def test_traffic_is_scaled_by_the_copy_and_averaged_over_in_place_phases(tmp_path):
    copy = 1 << 30
    nodes = 1000
    # the copy's FETCH_SIZE reads half its bytes (factor 2), WRITE_SIZE all
    fetch = [(COPY, "FETCH_SIZE", copy / 2 / 1024), (COPY, "FETCH_SIZE", 10.0)]
    write = [(COPY, "WRITE_SIZE", copy / 1024)]
    # f16s: three dispatches; the median of FETCH_SIZE (21.484375 KiB) counts
    # 44,000 B read, WRITE_SIZE 44,000 B written
    fetch += [(SWEEP_F16, "FETCH_SIZE", v) for v in (20.0, 21.484375, 30.0)]
    write += [(SWEEP_F16, "WRITE_SIZE", 42.96875)] * 3
    # in place: two phases and two band pre-passes, one step of each phase
    fetch += [(SWEEP_F64_IP0, "FETCH_SIZE", 100.0), (SWEEP_F64_IP1, "FETCH_SIZE", 80.0),
              (BAND_F64_0, "FETCH_SIZE", 5.0), (BAND_F64_1, "FETCH_SIZE", 7.0)]
    write += [(SWEEP_F64_IP0, "WRITE_SIZE", 150.0), (SWEEP_F64_IP1, "WRITE_SIZE", 130.0),
              (BAND_F64_0, "WRITE_SIZE", 1.0), (BAND_F64_1, "WRITE_SIZE", 1.0)]
    # a diagnostics sweep is left out of the per-launch figure
    fetch.append((SWEEP_F16_DIAG, "FETCH_SIZE", 999.0))
    write.append((SWEEP_F16_DIAG, "WRITE_SIZE", 999.0))
    fdb = _db(tmp_path / "f.db", pmc=fetch)
    wdb = _db(tmp_path / "w.db", pmc=write)
    out = pf.traffic_summary(fdb, wdb, float(copy), nodes, "cmd")
    assert out["fetch_factor"] == pytest.approx(2.0)
    assert out["write_factor"] == pytest.approx(1.0)
    assert out["source_sha256"] == pf.source_hash()
    f16 = out["formats"]["f16s"]
    assert f16["fetch_bytes"] == pytest.approx(21.484375 * 1024 * 2)   # the median, scaled
    assert f16["write_bytes"] == pytest.approx(42.96875 * 1024)
    assert f16["stored_bytes"] == 88 * nodes
    assert f16["ratio"] == pytest.approx((f16["fetch_bytes"] + f16["write_bytes"]) / (88 * nodes))
    ip = out["formats"]["f64ip"]
    assert ip["fetch_bytes"] == pytest.approx((100.0 + 80.0 + 5.0 + 7.0) * 1024 * 2 / 2)
    assert ip["write_bytes"] == pytest.approx((150.0 + 130.0 + 1.0 + 1.0) * 1024 / 2)
    json.dumps(out)   # the summary is plain JSON


def test_traffic_needs_the_calibration_copy(tmp_path):
    fdb = _db(tmp_path / "f.db", pmc=[(SWEEP_F16, "FETCH_SIZE", 1.0)])
    wdb = _db(tmp_path / "w.db", pmc=[(SWEEP_F16, "WRITE_SIZE", 1.0)])
    with pytest.raises(SystemExit):
        pf.traffic_summary(fdb, wdb, 1024.0, 10, "cmd")
