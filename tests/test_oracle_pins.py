"""The CPU oracle against values and properties fixed by the paper and by
mathematics (see tests/oracle_pins.py for what each pin checks)."""
import numpy as np
import pytest

import oracle_pins as P
from oracle import circulant, dense, forest, sparse
from paper_2101_08143_amd import workloads as W


def sparse_indices(g, s):
    vals, _, info = sparse.indices(g, s)
    assert info["status"] == 0
    return vals


def sparse_solve(g, s):
    z, info = sparse.solve(g, s)
    assert info["status"] == 0
    return z


def sparse_fj(g, s):
    z, info = sparse.fj_iterate(g, s, tol=1e-15)
    assert info["status"] == 0
    return z


def test_p5_forest_matrix_dense():
    P.pin_p5_forest_matrix(dense)


def test_p5_forest_enumeration():
    P.pin_p5_forest_enumeration(forest)


def test_forest_bruteforce_vs_dense():
    P.pin_forest_bruteforce(dense, forest)


def test_prop1_and_lemma41_forms():
    P.pin_prop1_and_lemma41(dense)


@pytest.mark.parametrize("which", ["dense", "sparse"])
def test_closed_forms(which):
    P.pin_closed_forms(dense.indices if which == "dense" else sparse_indices)


@pytest.mark.parametrize("which", ["dense", "sparse"])
def test_circulant(which):
    if which == "dense":
        P.pin_circulant(dense.indices, dense.equilibrium, circulant)
    else:
        P.pin_circulant(sparse_indices, sparse_solve, circulant,
                        sizes=((997, 0.7), (1000, None), (65536, 1.7)),
                        torus=((30, 41, 1.3), (256, 300, 0.6)))


@pytest.mark.parametrize("which", ["dense", "sparse"])
def test_identities(which):
    if which == "dense":
        P.pin_identities(dense.indices, dense.equilibrium)
    else:
        P.pin_identities(sparse_indices, sparse_solve)


def test_p5_sparse_solve():
    P.pin_p5_sparse(sparse_solve)


def test_fj_dynamics():
    P.pin_fj_dynamics(sparse_fj, sparse_solve)


def test_sparse_matches_dense_on_small_graphs():
    for g in (W.barabasi_albert(800, 3, 61), W.random_graph(300, 0.03, 62, weighted=True),
              W.chung_lu(1500, 2.2, 12.0, 63, weighted=True)):
        s = W.opinions("exp", g.n, 64)
        a = dense.indices(g, s)
        b = sparse_indices(g, s)
        for k in P.NAMES:
            assert abs(a[k] - b[k]) <= 1e-11 * abs(a[k]), k


@pytest.mark.slow
def test_sparse_matches_dense_ba10k():
    """The dense 'Exact' analogue at n = 10^4 (Barabasi-Albert, m = 3)."""
    import scipy.linalg
    g = W.barabasi_albert(10_000, 3, 1001)
    s = W.opinions("uniform", g.n, 2001)
    M = np.eye(g.n) + dense.laplacian_dense(g)
    z_dense = scipy.linalg.solve(M, s, assume_a="pos")
    del M
    a = dense.indices_by_definition(g, s, z_dense)
    b = sparse_indices(g, s)
    for k in P.NAMES:
        assert abs(a[k] - b[k]) <= 1e-10 * abs(a[k]), k


@pytest.mark.slow
def test_sparse_large_cycle_vs_fft():
    n = 1 << 20
    s = np.random.default_rng(7).random(n)
    g = W.cycle_graph(n, 1.25)
    z = sparse_solve(g, s)
    assert np.abs(z - circulant.cycle_equilibrium(s, 1.25)).max() < 1e-11
    got = sparse_indices(g, s)
    want = circulant.cycle_indices(s, 1.25)
    for k in P.NAMES:
        assert abs(got[k] - want[k]) <= 1e-9 * abs(want[k]), k


@pytest.mark.slow
def test_oracle_certifies_itself_chung_lu():
    """The oracle's own a-posteriori bound is <= 1e-9 on a weighted power-law graph."""
    g = W.chung_lu(200_000, 2.2, 30.0, 1003, weighted=True)
    s = W.opinions("exp", g.n, 2003)
    vals, z, info = sparse.indices(g, s)
    assert info["status"] == 0 and info["certified"], info


def test_error_bounds_against_known_errors():
    P.pin_error_bounds(sparse)


def test_certified_flag():
    P.pin_certified_flag(sparse)


def test_sparse_lemma41_prop1_forms():
    P.pin_sparse_forms(sparse.indices_at, sparse_solve)
