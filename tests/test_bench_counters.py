"""Host logic of the benchmark's counter and trace summaries (CPU only):
synthetic rocprofv3 CSVs with known values go through bench.py's readers,
and the figures it records are checked against the arithmetic stated for
them (copy calibration, launches the device skipped dropped, GRBM_GUI_ACTIVE
summed over 8 XCDs, dual-issued VALU pairs counted once)."""
import csv
import json
import os

import pytest

import bench

LJ = "void md::k_lj32<8, 6, true, false, true>(long, HIP_vector_type<unsigned int, 4u> const*)"
COPY = "__amd_rocclr_copyBuffer"
GRID = 9830400


def _write_pass(d, rows):
    """rows: (dispatch, kernel, grid, counter, [values per instance])."""
    os.makedirs(os.path.join(d, "host"), exist_ok=True)
    with open(os.path.join(d, "host", "1_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        for disp, name, grid, ctr, vals in rows:
            for v in vals:
                w.writerow([disp, name, grid, ctr, v])


@pytest.fixture
def passes(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC", str(tmp_path / "traffic.json"))
    gib2 = 2 * (1 << 30) / 1024.0           # KiB moved each way by a 2 GiB copy
    fetch = str(tmp_path / "fetch")
    # copy: FETCH_SIZE reads 0.625 of what it moves (scale 1.6); LJ: three
    # full launches of 1000 KiB (two instances each) and one skipped launch
    _write_pass(fetch, [(1, COPY, 131072, "FETCH_SIZE", [0.625 * gib2]),
                        (2, LJ, GRID, "FETCH_SIZE", [400.0, 600.0]),
                        (3, LJ, GRID, "FETCH_SIZE", [500.0, 500.0]),
                        (4, LJ, GRID, "FETCH_SIZE", [1.0, 2.0]),
                        (5, LJ, GRID, "FETCH_SIZE", [700.0, 300.0])])
    write = str(tmp_path / "write")
    _write_pass(write, [(1, COPY, 131072, "WRITE_SIZE", [gib2]),
                        (2, LJ, GRID, "WRITE_SIZE", [50.0]),
                        (3, LJ, GRID, "WRITE_SIZE", [50.0])])
    sq = str(tmp_path / "sq")
    # 8 XCDs of 100,000 cycles each; 256 CUs
    rows = []
    for disp in (2, 3):
        rows += [(disp, LJ, GRID, "GRBM_GUI_ACTIVE", [100000.0] * 8),
                 (disp, LJ, GRID, "SQ_INSTS_VALU", [20.0e6]),
                 (disp, LJ, GRID, "SQ_ACTIVE_INST_VALU2", [4.0e6]),
                 (disp, LJ, GRID, "SQ_VALU_MFMA_BUSY_CYCLES", [0.0])]
    rows += [(4, LJ, GRID, "GRBM_GUI_ACTIVE", [100.0] * 8), (4, LJ, GRID, "SQ_INSTS_VALU", [10.0]),
             (4, LJ, GRID, "SQ_ACTIVE_INST_VALU2", [0.0]), (4, LJ, GRID, "SQ_VALU_MFMA_BUSY_CYCLES", [0.0])]
    _write_pass(sq, rows)
    ta = str(tmp_path / "ta")
    _write_pass(ta, [(2, LJ, GRID, "GRBM_GUI_ACTIVE", [100000.0] * 8),
                     (2, LJ, GRID, "TA_TA_BUSY_sum", [12.8e6]),
                     (2, LJ, GRID, "TCP_TOTAL_CACHE_ACCESSES_sum", [5.0e6])])
    return [fetch, write, sq, ta]


def test_counter_summary_arithmetic(passes):
    bench.summarize_counters(passes)
    rec = json.load(open(bench.TRAFFIC))["k_lj32_lj_voids_1.23M"]
    assert rec["grid_size"] == GRID
    assert rec["fetch_scale"] == pytest.approx(1.6)
    assert rec["write_scale"] == pytest.approx(1.0)
    # the skipped launch (3 KiB) is dropped: three launches of 1000 KiB
    assert rec["launches"] == 3
    assert rec["fetch_kib"] == pytest.approx(1000.0)
    assert rec["traffic_bytes"] == pytest.approx(1024.0 * (1000.0 * 1.6 + 50.0))
    cyc = 100000.0                                   # per XCD
    assert rec["cycles_per_xcd"] == pytest.approx(cyc)
    assert rec["valu_inst_per_cu_clk"] == pytest.approx(20.0e6 / (256 * cyc))
    assert rec["valu_issue_frac"] == pytest.approx((20.0e6 - 4.0e6) / (256 * cyc))
    assert rec["ta_busy_per_cu_clk"] == pytest.approx(12.8e6 / (256 * cyc))
    assert rec["tcp_total_cache_accesses"] == pytest.approx(5.0e6)
    assert rec["sources_sha256"] == bench._sources_sha(rec["sources"])


def test_counter_records_follow_their_sources(passes, monkeypatch):
    bench.summarize_counters(passes)
    assert bench.valu_frac("k_lj32_lj_voids_1.23M") == pytest.approx(16.0e6 / 25.6e6)
    # a record whose sources changed since the counters were taken reads as None
    data = json.load(open(bench.TRAFFIC))
    data["k_lj32_lj_voids_1.23M"]["sources_sha256"] = "0" * 64
    json.dump(data, open(bench.TRAFFIC, "w"))
    assert bench.valu_frac("k_lj32_lj_voids_1.23M") is None
    assert bench.recorded_traffic("k_lj32_lj_voids_1.23M") is None


def test_trace_summary_drops_skipped_launches(tmp_path, capsys):
    d = tmp_path / "trace" / "host"
    d.mkdir(parents=True)
    with open(d / "1_kernel_trace.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z", "Start_Timestamp", "End_Timestamp"])
        for t0, us in ((0, 120.0), (1000000, 124.0), (2000000, 8.0), (3000000, 122.0)):
            w.writerow([LJ, GRID, 1, 1, t0, t0 + int(us * 1000)])
    bench.summarize_trace(str(tmp_path / "trace"))
    lines = capsys.readouterr().out.strip().splitlines()
    assert lines[0].split("\t")[:3] == ["kernel", "grid", "launches"]
    f = lines[1].split("\t")
    assert int(f[1]) == GRID and int(f[2]) == 4
    assert float(f[3]) == pytest.approx((120 + 124 + 8 + 122) / 4, abs=0.01)
    assert int(f[5]) == 3 and float(f[6]) == pytest.approx(122.0, abs=0.01)


def test_dd_overlap_summary(tmp_path, capsys):
    """Two synthetic evaluations after two set-up ones: the halos' spans, the
    inner launches (larger grid) and whether each halo ends inside them."""
    d = tmp_path / "dd" / "host"
    d.mkdir(parents=True)
    ns = "md::(anonymous namespace)::"
    rows = []
    for e in range(4):
        b = e * 10_000_000
        rows += [(ns + "k_dd_scale_local(long, double const*)", 4000000, b, b + 38000),
                 (ns + "k_dd_pack(long, double const*, long)", 900352, b + 40000, b + 62000),
                 (ns + "k_dd_unpack(long, double const*)", 900352, b + 120000, b + 141000),
                 ("void md::k_eam_rho<md::FS32, 8, 4, true, false, true>(long)", 25739264, b + 39000, b + 317000),
                 ("void md::k_eam_rho<md::FS32, 8, 4, true, false, true>(long)", 6260736, b + 318000, b + 386000),
                 (ns + "k_dd_pack_w(long, HIP_vector_type<unsigned int, 4u>)", 900352, b + 387000, b + 404000),
                 (ns + "k_dd_unpack_w(long, unsigned int)", 900352, b + 480000, b + 697000),
                 ("void md::k_eam_force<md::FS32, 8, 4, true, false, true>(long)", 25739264, b + 387000, b + 676000),
                 ("void md::k_eam_force<md::FS32, 8, 4, true, false, true>(long)", 6260736, b + 677000, b + 751000)]
    with open(d / "1_kernel_trace.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z", "Start_Timestamp", "End_Timestamp"])
        for name, g, a, z in rows:
            w.writerow([name, g, 1, 1, a, z])
    bench.summarize_dd_overlap(str(tmp_path / "dd"))
    out = dict(line.split("\t")[:2] for line in capsys.readouterr().out.strip().splitlines()[1:])
    assert out["span_us"] == "mean 751.00"
    assert out["rho_inner_us"] == "mean 278.00" and out["rho_outer_us"] == "mean 68.00"
    assert out["position_halo_us"] == "mean 101.00" and out["position_halo_inside"] == "mean 1.00"
    # this F' halo ends after the inner force launch
    assert out["fprime_halo_us"] == "mean 310.00" and out["fprime_halo_inside"] == "mean 0.00"


def test_neighbor_candidate_model(capsys):
    """The candidate model on the perfect Cu crystal (plus its thermal start):
    every home atom has the 54 fcc neighbours within 5.4 A (shells of 12, 6,
    24 and 12), and the bounding-box test keeps a subset of what is streamed
    and all of what is listed."""
    bench.neighbor_candidates("cu54", samples=200)
    r = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert r["entries_per_home"] == pytest.approx(54.0)
    assert r["entries_per_home"] <= r["kept_per_home"] <= r["streamed_per_home"]
    assert r["chunks_per_home"] * 64 >= r["kept_per_home"]
    assert r["tested_per_entry"] > 1.0
