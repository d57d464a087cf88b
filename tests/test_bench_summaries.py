"""Host logic of bench.py's profile summaries (no GPU): rocprofv3 CSV files in
the layout the profiler writes are turned into the tables under profiles/,
and the traffic record is calibrated by the 1 GiB copy kernel."""
from __future__ import annotations

import csv
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

COPY = ("void at::native::vectorized_elementwise_kernel<4, at::native::CUDAFunctorOnSelf_add<int>, "
        "std::array<char*, 2ul> >(int, at::native::CUDAFunctorOnSelf_add<int>, std::array<char*, 2ul>)")
PF = "void gconn::k_sample_kout_pf<gconn::Rule<3, 1, 2>, unsigned int>(unsigned int const*, ...)"
INIT = "gconn::k_init(gconn::Ctrl*, unsigned int*, unsigned int, unsigned int*)"


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def _trace(d):
    rows = []
    t = 1000
    for name, us in [(INIT, 20.0), (PF, 900.0), (INIT, 10.0), (PF, 500.0), (INIT, 12.0),
                     (PF, 540.0)]:
        rows.append([name, t, t + int(us * 1000)])
        t += int(us * 1000) + 500
    _write(os.path.join(d, "x", "r_kernel_trace.csv"),
           ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)


def _pmc(d, counter, values):
    rows = [[name, counter, v] for name, v in values]
    _write(os.path.join(d, "x", "p_counter_collection.csv"),
           ["Kernel_Name", "Counter_Name", "Counter_Value"], rows)


def test_trace_table_excludes_the_first_call(tmp_path):
    _trace(str(tmp_path))
    table = bench.summarize_trace(str(tmp_path))
    lines = table.splitlines()
    assert lines[0].startswith("| kernel | calls |")
    pf = next(l for l in lines if "k_sample_kout_pf" in l)
    cells = [c.strip() for c in pf.split("|")[1:-1]]
    # calls, mean and median of the later calls, min of them, first call
    assert cells[1] == "3" and cells[2] == "520.0" and cells[3] == "520.0"
    assert cells[4] == "500.0" and cells[5] == "900.0"
    # the heaviest kernel comes first
    assert "k_sample_kout_pf" in lines[2]


def test_traffic_record_calibrated_by_the_copy(tmp_path):
    fd, wd = str(tmp_path / "fetch"), str(tmp_path / "write")
    # the copy reads and writes 1 GiB; its counters read half of it and all
    gib_kib = float(1 << 20)
    _pmc(fd, "FETCH_SIZE", [(COPY, gib_kib / 2), (COPY, gib_kib / 2), (PF, 1000.0), (PF, 1200.0),
                            (INIT, 10.0)])
    _pmc(wd, "WRITE_SIZE", [(COPY, gib_kib), (COPY, gib_kib), (PF, 400.0), (PF, 400.0),
                            (INIT, 65536.0)])
    out = tmp_path / "traffic.txt"
    md = bench.summarize_traffic(fd, wd, str(out))
    rec = json.loads(out.read_text())
    assert rec["source_sha"] == bench.source_sha()
    assert abs(rec["fetch_scale"] - 2.0) < 1e-9 and abs(rec["write_scale"] - 1.0) < 1e-9
    # (1100 KiB x 2 + 400 KiB) x 1024 bytes, per dispatch
    assert rec["per_kernel_bytes"]["k_sample_kout_pf"] == (1100 * 2 + 400) * 1024
    assert rec["hbm_bytes_per_launch"] == rec["per_kernel_bytes"]["k_sample_kout_pf"]
    assert rec["per_kernel_bytes"]["k_init"] == (10 * 2 + 65536) * 1024
    assert "elementwise" not in json.dumps(rec["per_kernel_bytes"])
    assert "| `k_sample_kout_pf<Rule<3, 1, 2>, unsigned int>` |" in md
    # bench reads the record back only while the sources hash to it
    assert bench.kernel_traffic(rec["per_kernel_bytes"], "k_sample_kout_pf") == \
        rec["hbm_bytes_per_launch"]


def test_pmc_table_means_per_dispatch(tmp_path):
    _pmc(str(tmp_path), "TCC_HIT_sum", [(PF, 10.0), (PF, 30.0), (INIT, 5.0)])
    table = bench.summarize_pmc(str(tmp_path))
    pf = next(l for l in table.splitlines() if "k_sample_kout_pf" in l)
    cells = [c.strip() for c in pf.split("|")[1:-1]]
    assert cells[1] == "2" and cells[2] == "20"
