"""bench.py's measurement arithmetic on the host: the byte and flop models of
the D=4, N=65536 workload, written out by hand here, and the conversion of two
rocprofv3 counter runs into bytes per launch."""
import csv
import math
import os

import bench
import synth

agg = __import__("pytest").importorskip("paper_1905_09071_amd")


def test_byte_model_c3():
    N, u, M, cs = 65536, 3, 131072, 16
    # fused column pass: combined spectrum in, n and the u columns in, k1 and n~ out, u spectra out
    assert bench.pass_bytes(3, N, u, M, cs) == M * cs + 8 * N * 4 + 2 * 8 * N + 3 * M * cs == 11534336
    # row pass: u spectra in, the combined spectrum out
    assert bench.pass_bytes(1, N, u, M, cs) == 4 * M * cs == 8388608


def test_flop_model_c3():
    c = synth.config("C3")
    tables = agg.plan_tables(4, 65536, c["kernel"], "fp32c")
    tsum, T = bench.gain_terms(tables, c["kernel"])
    assert (tsum, T) == (6, 3)     # terms {A,B}, {A,B,1}, {A,B,1,1}: 1 + 2 + 3 products
    L, N, u = 262144, 65536, 3
    want = 4 * 2.5 * L * 18 + (L // 2 + 1) * (6 * 6 + 2 * 3) + 4 * N * u + 10 * N
    assert math.isclose(bench.rhs_flops(N, u, L, tsum, T), want) and round(want / 1e6) == 54


def test_traffic_from_counter_runs(tmp_path):
    def write(path, counter, rows):
        with open(path, "w", newline="") as f:
            w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
            w.writeheader()
            for name, v in rows:
                w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v})
    col, row = "void agg::col_kernel<ff, 512, false, false>(agg::LaunchArgs)", "void agg::row_kernel<ff, 256, false>(agg::LaunchArgs)"
    fpath, wpath = tmp_path / "f.csv", tmp_path / "w.csv"
    write(fpath, "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 131072.0), (col, 100.0), (col, 300.0), (col, 200.0), (row, 50.0)])
    write(wpath, "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 262144.0), (col, 10.0), (col, 10.0), (col, 10.0), (row, 7.0)])
    out = tmp_path / "t.json"
    t = bench.write_traffic(str(fpath), str(wpath), 256, "fp32c", out_path=str(out))
    assert os.path.exists(out)
    assert t["fetch_scale"] == 2.0 and t["write_scale"] == 1.0
    # medians 200 KiB fetched (x2 for the copy calibration) and 10 KiB written
    assert t["bytes_per_launch"]["fp32c:3"] == (200 * 2 + 10) * 1024
    assert t["bytes_per_launch"]["fp32c:1"] == (50 * 2 + 7) * 1024
