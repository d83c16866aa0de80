"""Host logic of the profile summariser: dispatch grouping into gemm calls, path matching by
grid size, and the copy calibration of the HBM counters (fabricated rocprofv3 CSV rows)."""
import csv
import json

from paper_1804_10694_amd import profsum

PK = "void tg::packed_kernel<tg::PCfg<{m}, 128, 128, 16, 2, 2, 4> >(tg::PackedArgs)"
PR = "void tg::pack_rows_kernel<{m}>(void const*, long, int, int, void*, void*, int, int)"
PC = "void tg::pack_cols_kernel<{m}>(void const*, long, int, int, void*, void*, int, int)"
CP = "__amd_rocclr_copyBuffer"


def _pmc(path, rows, counter):
    cols = ["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value",
            "Start_Timestamp", "End_Timestamp"]
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(cols)
        for i, (name, grid, val) in enumerate(rows, 1):
            # two rows per dispatch (e.g. two counter instances) are summed
            for half in (val / 2, val / 2):
                w.writerow([i, grid, name, counter, half, 1000 * i, 1000 * i + 500])


def test_traffic_groups_calls_and_applies_calibration(tmp_path):
    bench = {"paths": {"f32_256x256x256": {"grid_threads": 1024, "schedule_key": "sched:0:a",
                                           "avg_ms": 1, "tflops": 1, "frac_peak": 1,
                                           "peak_tflops": 1}},
             "roofline": {"kernel_source_sha256": "abc"}}
    bp = tmp_path / "b.json"
    bp.write_text("noise\n" + json.dumps(bench) + "\n")
    call = [(PR.format(m=0), 4096, 10.0), (PC.format(m=0), 4096, 20.0), (PK.format(m=0), 1024, 70.0)]
    # cold call, two timed calls, a stray copy, then the 1 GiB calibration copy
    rows_f = call + call + [(call[0][0], 4096, 10.0), (call[1][0], 4096, 20.0),
                            (call[2][0], 1024, 130.0)] + [(CP, 64, 5.0), (CP, 64, 2 ** 20 / 2)]
    rows_f[-2] = (CP, 64, 5.0)
    _pmc(tmp_path / "f.csv", rows_f[:9] + [(PK.format(m=1), 999, 1.0)] + rows_f[9:], "FETCH_SIZE")
    _pmc(tmp_path / "w.csv", [(n, g, v / 10) for n, g, v in rows_f[:9]] + [(CP, 64, 2 ** 20 / 4)],
         "WRITE_SIZE")
    out, table = tmp_path / "t.md", tmp_path / "t.json"

    class A:
        fetch, write, bench = str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(bp)
        out_, title = str(out), "t"
        command_fetch = command_write = "cmd"
    A.out, A.table = str(out), str(table)
    profsum.cmd_traffic(A)
    t = json.loads(table.read_text())
    rec = t["sched:0:a@256x256x256"]
    # the last dispatch is the calibration copy; the smaller copy before it does not count
    f_factor = 2 ** 30 / ((2 ** 20 / 2) * 1024)
    w_factor = 2 ** 30 / ((2 ** 20 / 4) * 1024)
    # timed calls (cold one dropped): 100 and 160 KiB fetched, 10 and 16 KiB written
    assert abs(rec["read_bytes"] - 130.0 * 1024 * f_factor) < 1e-6 * rec["read_bytes"]
    assert abs(rec["written_bytes"] - 13.0 * 1024 * w_factor) < 1e-6 * rec["written_bytes"]
    assert rec["source_sha256"] == "abc"
    assert rec["compulsory_bytes"] == 4 * (3 * 256 * 256 + 256 * 256)


def test_short_names_and_kinds():
    n = PK.format(m=1)
    assert profsum.short_name(n) == "packed_kernel<PCfg<1,128,128,16,2,2,4>>"
    assert profsum.kind(n) == "packed_kernel"
    assert profsum.kind(PR.format(m=0)) == "pack_rows_kernel"
    assert profsum.kind(CP) is None
