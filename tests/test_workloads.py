"""Seeded input generators: determinism, structure, value ranges."""
import numpy as np

from paper_2101_08143_amd import workloads as W


def test_ba_structure_and_determinism():
    a = W.barabasi_albert(2000, 3, 1001)
    b = W.barabasi_albert(2000, 3, 1001)
    a.validate()
    assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col)
    assert a.m == 6 + 3 * (2000 - 4)
    assert np.diff(a.row_ptr).min() >= 3


def test_chung_lu_structure_and_determinism():
    a = W.chung_lu(50_000, 2.2, 12.0, 7, weighted=True)
    b = W.chung_lu(50_000, 2.2, 12.0, 7, weighted=True)
    a.validate()
    assert np.array_equal(a.col, b.col) and np.array_equal(a.val, b.val)
    assert a.val.dtype == np.float32 and a.val.min() >= 0.5 and a.val.max() < 2.0
    mean_deg = a.nnz / a.n
    assert 0.9 * 12.0 < mean_deg <= 12.0
    deg = np.diff(a.row_ptr)
    assert deg.max() <= 2 * np.sqrt(50_000 * 12.0)
    assert W.chung_lu(50_000, 2.2, 12.0, 8).nnz != a.nnz


def test_chung_lu_weights_capped_and_rescaled():
    w = W.chung_lu_weights(100_000, 2.1, 20.0)
    assert abs(w.mean() - 20.0) < 1e-9 * 20
    assert w.max() <= np.sqrt(100_000 * 20.0) * (1 + 1e-9)
    assert np.all(np.diff(w) <= 0)


def test_opinions_ranges():
    for kind in ("uniform", "exp", "pareto", "exp_paper", "powerlaw_paper"):
        s = W.opinions(kind, 10_000, 3)
        assert s.dtype == np.float64 and s.min() >= 0.0 and s.max() <= 1.0
    for kind in ("exp", "pareto"):
        s = W.opinions(kind, 1000, 4)
        assert s.min() == 0.0 and s.max() == 1.0
    assert W.opinions("exp_paper", 1000, 5).max() == 1.0
    blk = W.opinion_block(500, ["uniform"] * 3 + ["exp"] * 2, 9)
    assert blk.shape == (500, 5) and blk.flags["C_CONTIGUOUS"]
    assert np.array_equal(blk[:, 3], W.opinions("exp", 500, 12))


def test_validate_rejects_bad_graphs():
    g = W.path_graph(4)
    g.validate()
    bad = W.CSRGraph(n=3, row_ptr=np.array([0, 1, 1, 1], np.int32), col=np.array([1], np.int32))
    try:
        bad.validate()
    except ValueError as e:
        assert "symmetric" in str(e)
    else:
        raise AssertionError("asymmetric graph accepted")
