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
