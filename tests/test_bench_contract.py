"""bench.py's host-side contract (no GPU): one GPU only, the algorithmic byte
counts behind roofline.achieved, and the recorded-counter lookup."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_spmv_algorithmic_bytes_of_the_4m_node_workload():
    """col + val (f32) per entry, row_ptr, and p, r, q (FP64) plus M^-1 (f32)
    per row: 1,082,488,372 bytes per launch on the 4M-node graph."""
    n, nnz = 4_000_000, 119_311_046
    assert bench.spmv_bytes(n, nnz, 4) == nnz * 8 + 4 * (n + 1) + n * (3 * 8 + 4) == 1_082_488_372


def test_block_preconditioned_spmv_algorithmic_bytes():
    """The SpMV of the 2x2-block-preconditioned CG reads col + val, row_ptr
    and p and writes q: 1,034,488,372 bytes per launch on the 4M-node graph."""
    n, nnz = 4_000_000, 119_311_046
    assert bench.spmv_pq_bytes(n, nnz, 4) == nnz * 8 + 4 * (n + 1) + 16 * n == 1_034_488_372
    assert bench.PAIR_MIN_N == 65536


def test_spmm_algorithmic_bytes():
    """k = 64 FP64 columns on the 1M-node unit-weight graph: col per entry,
    row_ptr, P read, R read, Q written, M^-1."""
    n, nnz = 1_000_000, 9_899_994
    assert bench.spmm_bytes(n, nnz, 0, 64, 8) == nnz * 4 + 4 * (n + 1) + 3 * n * 64 * 8 + 4 * n


def test_recorded_traffic_lookup():
    assert bench.recorded_traffic("no_such_kernel") is None
    h = bench.kernel_source_hash()
    assert len(h) == 64 and all(c in "0123456789abcdef" for c in h)
    t = bench.recorded_traffic("k_cg_spmv<float, double>")
    # present only while the committed counters describe these sources
    assert t is None or t > bench.spmv_bytes(4_000_000, 119_311_046, 4)


def test_solve_byte_model():
    """Per-iteration vector streams of the solve model: 17.5 n-vectors for
    the pair path, 11 for Jacobi; a solve is iterations plus the epilogue."""
    n, nnz = 4_000_000, 119_311_046
    m = bench.solve_bytes(n, nnz, 4, 11, True)
    csr = nnz * 8 + 4 * (n + 1)
    assert m["c_v"] == 17.5 and m["bytes_per_iteration"] == int(csr + 17.5 * n * 8)
    assert m["bytes_per_solve"] == int(11 * (csr + 17.5 * n * 8) + csr + 3.5 * n * 8)
    assert bench.solve_bytes(n, nnz, 4, 14, False)["c_v"] == 11


def test_short_kernel_names():
    """rocprofv3's demangled names reduce to the keys of the counter record."""
    f = bench.short_kernel_name
    assert f("void fj::k_spmm_cg<fj::Unit, double, 64, 2, false, 64>(fj::Csr<fj::Unit>, int)") == \
        "k_spmm_cg<Unit, double, 64, 2, false, 64>"
    assert f("fj::k_fin_pair(int, int, double const*, fj::Ctrl*)") == "k_fin_pair"
    assert f("void fj::k_ml_rows<fj::OpPre>(int, fj::OpPre, fj::Ctrl const*)") == "k_ml_rows<OpPre>"
    assert f("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_profile_summary_from_synthetic_csvs(tmp_path, monkeypatch):
    """--summarize-profiles: working-dispatch means (above 30 % of the largest),
    the copy calibration scale, and the bytes per launch it records."""
    import csv
    import json

    def counters(sub, name, rows):
        d = tmp_path / sub
        d.mkdir()
        with open(d / "run_counter_collection.csv", "w", newline="") as f:
            w = csv.writer(f)
            w.writerow(["Kernel_Name", "Counter_Name", "Counter_Value"])
            for k, v in rows:
                w.writerow([k, name, v])

    copy = "__amd_rocclr_copyBuffer"
    kern = "void fj::k_x<double>(int)"
    counters("cfetch", "FETCH_SIZE", [(copy, 512 * 1024)])  # half of 1 GiB: scale 2
    counters("cwrite", "WRITE_SIZE", [(copy, 1024 * 1024)])
    counters("fetch", "FETCH_SIZE", [(kern, 100.0), (kern, 100.0), (kern, 1.0)])  # the 1.0 is an empty launch
    counters("write", "WRITE_SIZE", [(kern, 50.0), (kern, 50.0), (kern, 50.0)])
    (tmp_path / "stats").mkdir()
    with open(tmp_path / "stats" / "run_kernel_trace.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writerow([kern, 0, 2000])
        w.writerow([kern, 5000, 9000])
    out = tmp_path / "counters.json"
    monkeypatch.setattr(bench, "COUNTERS", str(out))
    bench.summarize_profiles(str(tmp_path))
    rec = json.loads(out.read_text())
    k = rec["kernels"]["k_x<double>"]
    assert k["working_dispatches"] == 2 and k["dispatches"] == 3 and k["fetch_kib"] == 100.0
    assert k["bytes_per_launch"] == int(round(100.0 * 1024 * 2.0 + 50.0 * 1024 * 1.0))
    assert rec["copy_calibration"]["fetch_scale"] == 2.0 and rec["source_sha256"] == bench.kernel_source_hash()
