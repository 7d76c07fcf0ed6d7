"""The time-phased SpMV (rows dealt to wave-chunks, entries ordered by column
phase, row sums in LDS) against the CPU oracle, through the C ABI: the bare
operator (fj_apply_phased) on every graph shape, and CG solves that run their
SpMV on it (FJ_PHASED_SPMV, and by default from 65536 nodes on)."""
import sys

import numpy as np
import pytest

from oracle import sparse as O
from paper_2101_08143_amd import workloads as W

pytestmark = pytest.mark.gpu

NAMES = ("internal_conflict", "disagreement", "polarization", "controversy", "dc_index")
EPS = 1e-6


def say(msg):
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_fj():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2101_08143_amd import fj
    fj.lib()
    return torch, fj


def hubs_f64():
    """Three hubs of 2500-4000 neighbours (dealt row by row, each longer than
    a 512-entry window of one phase) over 12000 leaves, FP64 weights."""
    rng = np.random.default_rng(21)
    edges = [(h, j) for h, m in ((0, 4000), (1, 3000), (2, 2500)) for j in rng.choice(np.arange(3, 12003), m,
                                                                                      replace=False)]
    edges += [(i, i + 1) for i in range(3, 12002)]
    w = rng.uniform(0.1, 10.0, len(edges))
    return W.csr_from_edges(12003, edges, w)


GRAPHS = {
    "single_node": lambda: W.csr_from_edges(1, []),
    "edgeless7": lambda: W.csr_from_edges(7, []),
    "path5": lambda: W.path_graph(5),
    "K50": lambda: W.complete_graph(50, 0.7),
    "ba3000": lambda: W.barabasi_albert(3000, 3, 11),
    "gnp500_f64": lambda: W.random_graph(500, 0.02, 12, weighted=True),
    "gnp400_f32": lambda: W.random_graph(400, 0.03, 13, weighted=True, val_dtype=np.float32),
    "star6001": lambda: W.csr_from_edges(6001, [(0, j) for j in range(1, 6001)]),
    "isolated9000": lambda: W.csr_from_edges(9000, [(i, i + 1) for i in range(3000, 3500)]),
    "cycle4099_w": lambda: W.cycle_graph(4099, 0.8),
    "hubs12003_f64": hubs_f64,
    "cl100k_unit": lambda: W.chung_lu(100_000, 2.1, 20.0, 14),
    "cl600k_f32": lambda: W.chung_lu(600_000, 2.2, 12.0, 16, weighted=True),  # 5 phases
    "cycle4300k_w": lambda: W.cycle_graph(4_300_000, 0.8),  # short chunks, more than resident; 33 phases
    "skewed_cl600k_f64": lambda: W.log_uniform_weights(W.chung_lu(600_000, 2.2, 12.0, 17), 1e4, 6),  # long chunks
}


def tolerance(g, x):
    """|error| of either form of ((I + L) x)_i is below a few ulps of
    |x_i| (1 + d_i) + sum_j w_ij |x_j|; 1e-13 of it leaves a wide margin."""
    w = np.abs(g.weights_f64())
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    mag = np.abs(x) * (1 + np.bincount(rows, weights=w, minlength=g.n))
    mag += np.bincount(rows, weights=w * np.abs(x[g.col]), minlength=g.n)
    return 1e-13 * mag + 1e-300


@pytest.mark.parametrize("name", list(GRAPHS))
def test_apply_phased_matches_oracle(torch_fj, name):
    """fj_apply_phased equals the oracle's (I + L) x within rounding, agrees
    with the CSR-order pass, and repeats bit for bit."""
    torch, fj = torch_fj
    g = GRAPHS[name]()
    say(f"apply_phased {name} n={g.n} nnz={g.nnz}")
    G = fj.Graph.from_csr(g, device="cuda:0", validate=True)
    x = np.random.default_rng(3).standard_normal(g.n)
    xd = torch.from_numpy(x).to("cuda:0")
    y1 = fj.fj_apply(G, xd, phased=True)
    y2 = fj.fj_apply(G, xd, phased=True)
    yw = fj.fj_apply(G, xd).cpu().numpy()
    ref = O.apply(g, x)
    tol = tolerance(g, x)
    got = y1.cpu().numpy()
    assert np.all(np.abs(got - ref) <= tol), float(np.max(np.abs(got - ref) / tol))
    assert np.all(np.abs(got - yw) <= 2 * tol)
    assert torch.equal(y1, y2)


SOLVE_GRAPHS = {
    "cl100k_unit": lambda: W.chung_lu(100_000, 2.1, 20.0, 14),
    "cl120k_f32": lambda: W.chung_lu(120_000, 2.2, 30.0, 17, weighted=True),
    "ba100k": lambda: W.barabasi_albert(100_000, 4, 18),
    "skewed_cl100k": lambda: W.log_uniform_weights(W.chung_lu(100_000, 2.5, 10.0, 19), 1e4, 5),
}


@pytest.mark.parametrize("name", sorted(SOLVE_GRAPHS))
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_on_phased_spmv_matches_oracle(torch_fj, name, precision):
    """CG with the 2x2 blocks, its SpMV on the phased layout (FJ_PHASED_SPMV)
    and on the row windows (FJ_WINDOW_SPMV): both certify every index
    against the oracle, in about the same number of iterations."""
    torch, fj = torch_fj
    g = SOLVE_GRAPHS[name]()
    say(f"solve phased {name} {precision} n={g.n} nnz={g.nnz}")
    G = fj.Graph.from_csr(g, device="cuda:0", validate=True)
    s = W.opinions("exp", g.n, 23)
    sd = torch.from_numpy(s).to("cuda:0")
    ref, _, _ = O.indices(g, s)
    prec = fj.FJ_FP64 if precision == "fp64" else fj.FJ_MIXED
    its = {}
    for form, flag in (("phased", fj.FJ_PHASED_SPMV), ("window", fj.FJ_WINDOW_SPMV)):
        vals, infos, rc = fj.fj_indices(G, sd, fj.make_opts(eps=EPS, precision=prec, flags=flag))
        assert rc == fj.FJ_OK, (form, fj.info_dict(infos[0]))
        for j, nm in enumerate(NAMES):
            err = abs(vals[0][nm] - ref[nm]) / abs(ref[nm])
            assert err <= EPS and err <= infos[0].bound[j] + 1e-12, (form, nm, err)
        its[form] = infos[0].iters
    say(f"  iterations {its}")
    assert abs(its["phased"] - its["window"]) <= max(2, its["window"] // 5), its


def test_default_runs_phased_on_large_graphs(torch_fj):
    """On a 600K-node and a 100K-node graph the default one-vector solve is the
    FJ_PHASED_SPMV solve bit for bit; FJ_WINDOW_SPMV gives the same z within the residual
    target; a multilevel solve also runs its SpMV on the layout."""
    torch, fj = torch_fj
    g = W.chung_lu(600_000, 2.2, 12.0, 16, weighted=True)
    say(f"default phased n={g.n} nnz={g.nnz}")
    G = fj.Graph.from_csr(g, device="cuda:0", validate=True)
    s = W.opinions("uniform", g.n, 29)
    sd = torch.from_numpy(s).to("cuda:0")
    zd, _, rc1 = fj.fj_solve(G, sd, fj.make_opts(rtol=1e-10))
    zp, _, rc2 = fj.fj_solve(G, sd, fj.make_opts(rtol=1e-10, flags=fj.FJ_PHASED_SPMV))
    zw, _, rc3 = fj.fj_solve(G, sd, fj.make_opts(rtol=1e-10, flags=fj.FJ_WINDOW_SPMV))
    assert rc1 == rc2 == rc3 == fj.FJ_OK
    assert torch.equal(zd, zp)
    zref, _ = O.solve(g, s, rtol=1e-14)
    for z in (zd, zw):
        assert np.linalg.norm(z.cpu().numpy() - zref) <= 1.1e-10 * np.linalg.norm(s)
    # a 100K-node graph (short of the L2-sized vector): the default is phased there too
    g2 = W.chung_lu(100_000, 2.5, 10.0, 3)
    G2 = fj.Graph.from_csr(g2, device="cuda:0", validate=True)
    s2 = torch.from_numpy(W.opinions("uniform", g2.n, 30)).to("cuda:0")
    z2d, _, r1 = fj.fj_solve(G2, s2, fj.make_opts(rtol=1e-10))
    z2p, _, r2 = fj.fj_solve(G2, s2, fj.make_opts(rtol=1e-10, flags=fj.FJ_PHASED_SPMV))
    assert r1 == r2 == fj.FJ_OK and torch.equal(z2d, z2p)
    H = fj.Hierarchy(G)
    zm, _, rc = fj.fj_solve(G, sd, fj.make_opts(rtol=1e-10, hierarchy=H))
    assert rc == fj.FJ_OK
    assert np.linalg.norm(zm.cpu().numpy() - zref) <= 1.1e-10 * np.linalg.norm(s)
    H.close()


@pytest.mark.parametrize("name", ["ba3000", "gnp500_f64", "star6001", "isolated9000", "cl100k_unit"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_jacobi_solve_on_phased_spmv_matches_oracle(torch_fj, name, precision):
    """Jacobi-preconditioned CG (FJ_DIAG_PRECOND) with its SpMV and the three
    fused dot products on the phased layout (FJ_PHASED_SPMV): every index
    certified against the oracle."""
    torch, fj = torch_fj
    g = GRAPHS[name]()
    say(f"jacobi phased {name} {precision} n={g.n} nnz={g.nnz}")
    G = fj.Graph.from_csr(g, device="cuda:0", validate=True)
    s = W.opinions("uniform", g.n, 37)
    ref, _, _ = O.indices(g, s)
    prec = fj.FJ_FP64 if precision == "fp64" else fj.FJ_MIXED
    vals, infos, rc = fj.fj_indices(G, torch.from_numpy(s).to("cuda:0"),
                                    fj.make_opts(eps=EPS, precision=prec,
                                                 flags=fj.FJ_DIAG_PRECOND | fj.FJ_PHASED_SPMV), check=False)
    assert rc in (fj.FJ_OK, fj.FJ_ERR_UNCERTIFIABLE), fj.info_dict(infos[0])
    for j, nm in enumerate(NAMES):
        diff = abs(vals[0][nm] - ref[nm])
        assert diff <= infos[0].abs_bound[j] + 1e-12, (nm, diff)
        if np.isfinite(infos[0].bound[j]):
            assert diff <= EPS * abs(ref[nm]) and diff <= infos[0].bound[j] * abs(ref[nm]) + 1e-12, (nm, diff)


U = np.finfo(np.float64).eps / 2


@pytest.mark.parametrize("steps", [1, 5, 40])
def test_dynamics_on_phased_layout_matches_oracle(torch_fj, steps):
    """From 65536 nodes on, FJ steps run on the phased layout: each step
    within a few ulps per term of the oracle's sweep (the step is a
    max-norm contraction, so per-step errors add up at most linearly), and a
    restart continues bit for bit."""
    torch, fj = torch_fj
    g = GRAPHS["cl600k_f32"]()
    say(f"dynamics phased cl600k_f32 steps={steps}")
    G = fj.Graph.from_csr(g, device="cuda:0", validate=True)
    s = np.random.default_rng(31).random(g.n)
    sd = torch.from_numpy(s).to("cuda:0")
    z, info = fj.fj_dynamics(G, sd, steps, tol=-1.0)
    ref, oinfo = O.fj_iterate(g, s, max_sweeps=steps, tol=-1.0)
    assert info["iters"] == steps == oinfo["sweeps"] and info["status"] == 0
    dmax = int(np.diff(g.row_ptr).max())
    err = np.abs(z.cpu().numpy() - ref).max()
    assert err <= steps * 4.0 * (dmax + 3) * U, err
    if steps == 5:
        z2, _ = fj.fj_dynamics(G, sd, 2)
        z3, _ = fj.fj_dynamics(G, sd, 3, z0=z2)
        assert torch.equal(z3, z)
