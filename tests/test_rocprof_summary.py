"""Host logic of the profile summaries (CPU only): the counter calibration
against the copy kernel and the early-exit accounting of the kernel trace,
on small synthetic rocprofv3 CSV files."""

import csv
import json

import pytest

from paper_1311_4521_amd import rocprof_summary as rs

DOM = "void tmh::hop_kernel<double, 0, 0>(tmh::HopArgs<double>)"
COPY = "tmh::(anonymous namespace)::stream_copy_kernel(unsigned int __vector(4)*)"


def write_counters(path, counter, rows):
    path.mkdir()
    with open(path / "run_counter_collection.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, (name, kib) in enumerate(rows):
            w.writerow({"Dispatch_Id": k, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": kib})


def test_traffic_scales_by_the_copy_kernel(tmp_path):
    copy_bytes = 805306368
    # FETCH_SIZE reads half the copy's bytes, WRITE_SIZE all of them
    write_counters(tmp_path / "f", "FETCH_SIZE",
                   [(COPY, copy_bytes / 2 / 1024), (DOM, 1000.0), (DOM, 1100.0), ("other", 5.0)])
    write_counters(tmp_path / "w", "WRITE_SIZE", [(COPY, copy_bytes / 1024), (DOM, 200.0), (DOM, 200.0)])
    out = tmp_path / "t.json"
    res = rs.traffic(str(tmp_path / "f"), str(tmp_path / "w"), str(out), copy_bytes=copy_bytes, sites=64)
    assert res["fetch_scale"] == pytest.approx(2.0) and res["write_scale"] == pytest.approx(1.0)
    assert res["fetch_bytes_per_launch"] == pytest.approx(2.0 * 1050.0 * 1024)
    assert res["write_bytes_per_launch"] == pytest.approx(200.0 * 1024)
    assert res["dispatches"] == [2, 2] and res["sites"] == 64
    assert res["source_hash"] == rs.hop_source_hash()
    assert json.load(open(out))["bytes_per_launch"] == pytest.approx(res["bytes_per_launch"])


def test_traffic_needs_both_kernels(tmp_path):
    write_counters(tmp_path / "f", "FETCH_SIZE", [(DOM, 1000.0)])
    write_counters(tmp_path / "w", "WRITE_SIZE", [(COPY, 1.0), (DOM, 1.0)])
    with pytest.raises(SystemExit):
        rs.traffic(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "t.json"))


def test_stats_counts_early_exits(tmp_path):
    d = tmp_path / "prof"
    d.mkdir()
    with open(d / "run_kernel_stats.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"])
        w.writeheader()
        w.writerow({"Name": DOM, "Calls": 4, "TotalDurationNs": 912000, "AverageNs": 228000, "Percentage": 90.0})
        w.writerow({"Name": COPY, "Calls": 1, "TotalDurationNs": 100000, "AverageNs": 100000, "Percentage": 10.0})
    with open(d / "run_kernel_trace.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        t = 0
        for name, dur in ((DOM, 300000), (DOM, 300000), (DOM, 2000), (DOM, 310000), (COPY, 100000)):
            w.writerow({"Kernel_Name": name, "Start_Timestamp": t, "End_Timestamp": t + dur})
            t += dur + 1000
    out = tmp_path / "s.md"
    rs.stats(str(d / "run_kernel_stats.csv"), str(out))
    lines = open(out).read().splitlines()
    dom = [l for l in lines if "hop_kernel" in l][0].split("|")
    assert dom[6].strip() == "1"                      # one early exit
    assert float(dom[7]) == pytest.approx(303.33, abs=0.01)
    cp = [l for l in lines if "stream_copy" in l][0].split("|")
    assert cp[6].strip() == "0" and float(cp[7]) == pytest.approx(100.0)


def write_multi(path, rows):
    path.mkdir()
    with open(path / "run_counter_collection.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, (name, counter, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": k, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_requests_bins_bytes_by_size(tmp_path):
    """Read bytes are 32/64/128 times the binned counts, write bytes 64 times
    the 64-byte requests plus 32 times the rest; the copy kernel checks them."""
    copy_bytes = 128 * 1000
    write_multi(tmp_path / "r", [
        (COPY, "TCC_EA0_RDREQ_128B_sum", 1000), (COPY, "TCC_EA0_RDREQ_64B_sum", 0),
        (COPY, "TCC_EA0_RDREQ_32B_sum", 0),
        (DOM, "TCC_EA0_RDREQ_128B_sum", 10), (DOM, "TCC_EA0_RDREQ_64B_sum", 3),
        (DOM, "TCC_EA0_RDREQ_32B_sum", 2),
        (DOM, "TCC_EA0_RDREQ_128B_sum", 20), (DOM, "TCC_EA0_RDREQ_64B_sum", 5),
        (DOM, "TCC_EA0_RDREQ_32B_sum", 0)])
    write_multi(tmp_path / "w", [
        (COPY, "TCC_EA0_WRREQ_sum", 2000), (COPY, "TCC_EA0_WRREQ_64B_sum", 2000),
        (DOM, "TCC_EA0_WRREQ_sum", 7), (DOM, "TCC_EA0_WRREQ_64B_sum", 4), (DOM, "TCC_EA0_RDREQ_DRAM_sum", 9)])
    out = tmp_path / "req.md"
    res = rs.requests(str(tmp_path / "r"), str(tmp_path / "w"), str(out), 2.0, copy_bytes)
    rd, wr, n, dram = res[DOM]
    assert rd == pytest.approx(128 * 15 + 64 * 4 + 32 * 1) and n == 2
    assert wr == pytest.approx(64 * 4 + 32 * 3) and dram == pytest.approx(9)
    text = open(out).read()
    assert "(1.0000 / 1.0000)" in text and "hop_kernel" in text


def test_gaps_share_between_kernels(tmp_path):
    p = tmp_path / "t_kernel_trace.csv"
    with open(p, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for name, s, e in (("batch_hop_kernel", 0, 100), ("other", 150, 160), ("batch_hop_kernel", 200, 290),
                           ("batch_vec_kernel", 300, 340), ("batch_hop_kernel", 350, 450)):
            w.writerow({"Kernel_Name": name, "Start_Timestamp": s, "End_Timestamp": e})
    assert rs.gaps(str(p), "batch_") == (330, 450, 4)
    assert rs.gaps(str(p), "batch_", 2) == (140, 150, 2)


def test_short_name_keeps_template_arguments():
    assert rs.short_name("void tmh::(anonymous namespace)::batch_tmarch_kernel<double, 0, false, 4, true>"
                         "(tmh::BatchHopTable<double>)") == "batch_tmarch_kernel<double, 0, false, 4, true>"
    assert rs.short_name("tmh::(anonymous namespace)::stream_copy_kernel(unsigned int __vector(4)*, long)") == \
        "stream_copy_kernel"
    assert rs.short_name("void tmh::hop_kernel<tmh::half_t, 0, 1>(tmh::HopArgs<tmh::half_t>)") == \
        "hop_kernel<half_t, 0, 1>"
    long = "void at::native::elementwise_kernel<" + "x" * 100 + ">(int)"
    assert rs.short_name(long, 40).endswith("...") and len(rs.short_name(long, 40)) == 40


def test_units_divides_by_the_active_cycles_and_drops_early_exits(tmp_path):
    d = tmp_path / "u"
    d.mkdir()
    rows = [  # (dispatch, kernel, counter, value)
        (0, COPY, "GRBM_GUI_ACTIVE", 1000.0), (0, COPY, "TA_BUSY_avr", 800.0),
        (1, DOM, "GRBM_GUI_ACTIVE", 2000.0), (1, DOM, "TA_BUSY_avr", 1000.0),
        (2, DOM, "GRBM_GUI_ACTIVE", 4000.0), (2, DOM, "TA_BUSY_avr", 3000.0),
        (3, DOM, "GRBM_GUI_ACTIVE", 100.0), (3, DOM, "TA_BUSY_avr", 100.0),  # early exit
        (4, "other", "GRBM_GUI_ACTIVE", 10.0), (4, "other", "TA_BUSY_avr", 1.0),
    ]
    with open(d / "run_counter_collection.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, name, c, v in rows:
            w.writerow({"Dispatch_Id": k, "Kernel_Name": name, "Counter_Name": c, "Counter_Value": v})
    out = tmp_path / "u.md"
    res = rs.units(str(out), [str(d)], command="cmd")
    assert res[COPY]["TA_BUSY_avr"] == (pytest.approx(0.8), 1)
    assert res[DOM]["TA_BUSY_avr"] == (pytest.approx((0.5 + 0.75) / 2), 2)
    assert "other" not in res
    text = out.read_text()
    assert text.startswith("cmd") and "`stream_copy_kernel" in text and "0.625" in text
