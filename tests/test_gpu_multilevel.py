"""The multilevel preconditioner (FJ_MULTILEVEL: CG preconditioned by an
aggregation V-cycle, a Laplacian solver of the class Lemma ST asks for)
against the CPU oracle, through the C ABI."""
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


def skewed(g, span, seed):
    """The same graph with weights log-uniform over a factor `span`."""
    return W.log_uniform_weights(g, span, seed)


def check_indices(vals, infos, ref, tag):
    for j, nm in enumerate(NAMES):
        err = abs(vals[0][nm] - ref[nm]) / abs(ref[nm])
        assert err <= EPS and err <= infos[0].bound[j] + 1e-12, (tag, nm, err)


def test_wide_weight_spread_halves_the_iterations(torch_fj):
    """100K-node Chung-Lu graph, weights log-uniform over a factor 1e6: the
    V-cycle solve matches the oracle's z and indices in at most half the CG
    iterations of the 2x2 block preconditioner (the default) and far fewer
    than Jacobi's."""
    torch, fj = torch_fj
    g = skewed(W.chung_lu(100_000, 2.5, 10.0, 31), 1e6, 7)
    say(f"multilevel span=1e6 n={g.n} nnz={g.nnz}")
    G = fj.Graph.from_csr(g, device="cuda:0", validate=True)
    H = fj.Hierarchy(G)
    levels, ns, nnzs, dense = H.shape()
    say(f"  hierarchy: {levels} levels {ns}, entries {nnzs}, dense last {dense}")
    assert levels >= 2 and ns[0] == g.n and all(ns[l + 1] < ns[l] for l in range(levels - 1))
    assert nnzs[0] == g.nnz and dense == (ns[-1] <= 2048)
    s = W.opinions("uniform", g.n, 32)
    sd = torch.from_numpy(s).to("cuda:0")
    zref, _ = O.solve(g, s, rtol=1e-14)
    ref, _, _ = O.indices(g, s)
    its = {}
    for name, o in (("pairs", fj.make_opts(rtol=1e-10)), ("jacobi", fj.make_opts(rtol=1e-10, flags=fj.FJ_DIAG_PRECOND)),
                    ("multilevel", fj.make_opts(rtol=1e-10, hierarchy=H))):
        z, info, rc = fj.fj_solve(G, sd, o)
        assert rc == fj.FJ_OK, name
        assert np.linalg.norm(z.cpu().numpy() - zref) <= 1.1e-10 * np.linalg.norm(s), name
        its[name] = info[0].iters
    say(f"  iterations to 1e-10: {its}")
    assert its["multilevel"] <= 0.5 * its["pairs"], its
    vals, infos, rc = fj.fj_indices(G, sd, fj.make_opts(eps=EPS, hierarchy=H))
    assert rc == fj.FJ_OK
    check_indices(vals, infos, ref, "multilevel")
    H.close()


GRAPHS = {
    "ba3000": lambda: W.barabasi_albert(3000, 3, 11),
    "gnp500_f64": lambda: W.random_graph(500, 0.02, 12, weighted=True),
    "cl50k_f32": lambda: W.chung_lu(50_000, 2.2, 30.0, 15, weighted=True),
    "star6001": lambda: W.csr_from_edges(6001, [(0, j) for j in range(1, 6001)]),
    "cycle4099_w": lambda: W.cycle_graph(4099, 0.8),
    "isolated9000": lambda: W.csr_from_edges(9000, [(i, i + 1) for i in range(0, 600, 2)]),
    "skewed_cl20k": lambda: skewed(W.chung_lu(20_000, 2.5, 10.0, 5), 1e4, 3),
}


@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("kind", ["uniform", "exp"])
def test_indices_match_oracle(torch_fj, name, kind):
    """Every graph family: certified indices within eps of the oracle, and the
    hierarchy's levels shrink."""
    torch, fj = torch_fj
    g = GRAPHS[name]()
    say(f"multilevel {name} {kind} n={g.n} nnz={g.nnz}")
    G = fj.Graph.from_csr(g, device="cuda:0", validate=True)
    H = fj.Hierarchy(G, coarse_max=256)
    levels, ns, _, dense = H.shape()
    assert ns[0] == g.n and all(ns[l + 1] < ns[l] for l in range(levels - 1))
    assert dense == (ns[-1] <= 2048)
    s = W.opinions(kind, g.n, 41)
    ref, _, _ = O.indices(g, s)
    vals, infos, rc = fj.fj_indices(G, torch.from_numpy(s).to("cuda:0"), fj.make_opts(eps=EPS, hierarchy=H))
    assert rc == fj.FJ_OK, fj.info_dict(infos[0])
    check_indices(vals, infos, ref, name)
    say(f"  {levels} levels {ns}: {infos[0].iters} iterations")
    H.close()


def test_warm_start_and_determinism(torch_fj):
    """FJ_WARM_START runs with the V-cycle, two solves give the same z bit for
    bit, and FJ_TWO_SOLVE (a 2-column batched solve, which has no V-cycle) is
    refused."""
    torch, fj = torch_fj
    g = skewed(W.chung_lu(20_000, 2.5, 10.0, 5), 1e6, 9)
    G = fj.Graph.from_csr(g, device="cuda:0", validate=True)
    H = fj.Hierarchy(G)
    s = W.opinions("uniform", g.n, 43)
    sd = torch.from_numpy(s).to("cuda:0")
    ref, _, _ = O.indices(g, s)
    zref, _ = O.solve(g, s, rtol=1e-14)
    _, _, rc = fj.fj_indices(G, sd, fj.make_opts(eps=EPS, flags=fj.FJ_TWO_SOLVE, hierarchy=H), check=False)
    assert rc == fj.FJ_ERR_INVALID_ARG
    vals, infos, rc = fj.fj_indices(G, sd, fj.make_opts(eps=EPS, hierarchy=H))
    assert rc == fj.FJ_OK
    check_indices(vals, infos, ref, "multilevel")
    z1, _, rc1 = fj.fj_solve(G, sd, fj.make_opts(rtol=1e-10, hierarchy=H))
    z2, _, rc2 = fj.fj_solve(G, sd, fj.make_opts(rtol=1e-10, hierarchy=H))
    assert rc1 == rc2 == fj.FJ_OK
    assert torch.equal(z1, z2)
    # warm start from a perturbed solution
    z0 = torch.from_numpy(zref + 1e-4 * np.sin(np.arange(g.n))).to("cuda:0")
    z, info, rc = fj.fj_solve(G, sd, fj.make_opts(rtol=1e-10, flags=fj.FJ_WARM_START, hierarchy=H), Z=z0.clone())
    assert rc == fj.FJ_OK
    assert np.linalg.norm(z.cpu().numpy() - zref) <= 1.1e-10 * np.linalg.norm(s)
    H.close()


def test_hierarchy_must_fit_the_call(torch_fj):
    """A hierarchy built for another graph, or k > 1, is rejected."""
    torch, fj = torch_fj
    g1 = W.barabasi_albert(3000, 3, 11)
    g2 = W.barabasi_albert(3001, 3, 11)
    G1 = fj.Graph.from_csr(g1, device="cuda:0")
    G2 = fj.Graph.from_csr(g2, device="cuda:0")
    H2 = fj.Hierarchy(G2)
    s = torch.from_numpy(W.opinions("uniform", g1.n, 1)).to("cuda:0")
    _, _, rc = fj.fj_indices(G1, s, fj.make_opts(hierarchy=H2), check=False)
    assert rc == fj.FJ_ERR_INVALID_ARG
    H1 = fj.Hierarchy(G1)
    S2 = torch.stack([s, s], dim=1).contiguous()
    _, _, rc = fj.fj_indices(G1, S2, fj.make_opts(hierarchy=H1), check=False)
    assert rc == fj.FJ_ERR_INVALID_ARG
    H1.close()
    H2.close()


DEGENERATE = {
    "edgeless7": (lambda: W.csr_from_edges(7, []), 0),
    "single_edge": (lambda: W.csr_from_edges(2, [(0, 1)], [3.5]), 0),
    "K50": (lambda: W.complete_graph(50, 0.7), 1),
    "path300_deep": (lambda: W.path_graph(300, 2.0), 1),   # coarse_max 1: as many levels as the cap allows
    "two_stars": (lambda: W.csr_from_edges(203, [(0, j) for j in range(2, 102)] + [(1, j) for j in range(102, 203)]), 4),
}


@pytest.mark.parametrize("name", sorted(DEGENERATE))
def test_degenerate_graphs_match_dense_oracle(torch_fj, name):
    """Edgeless, a single edge, a complete graph (one aggregate), a path
    coarsened down to the level cap, and two stars: the V-cycle solve gives
    the dense oracle's z, and the certified indices match the dense
    definitions wherever they are certifiable."""
    from oracle import dense as D
    torch, fj = torch_fj
    build, coarse = DEGENERATE[name]
    g = build()
    G = fj.Graph.from_csr(g, device="cuda:0", validate=True)
    H = fj.Hierarchy(G, coarse_max=coarse)
    levels, ns, _, dense = H.shape()
    say(f"degenerate {name}: {levels} levels {ns}")
    assert 1 <= levels <= 16 and ns[0] == g.n and all(ns[l + 1] < ns[l] for l in range(levels - 1))
    s = W.opinions("uniform", g.n, 5)
    sd = torch.from_numpy(s).to("cuda:0")
    M = np.eye(g.n) + D.laplacian_dense(g)
    zref = np.linalg.solve(M, s)
    z, info, rc = fj.fj_solve(G, sd, fj.make_opts(rtol=1e-12, hierarchy=H))
    assert rc == fj.FJ_OK
    assert np.abs(z.cpu().numpy() - zref).max() <= 1e-10 * max(1.0, np.abs(zref).max())
    ref = D.indices(g, s)
    vals, infos, rc = fj.fj_indices(G, sd, fj.make_opts(eps=EPS, hierarchy=H), check=False)
    assert rc in (fj.FJ_OK, fj.FJ_ERR_UNCERTIFIABLE)
    for j, nm in enumerate(NAMES):
        diff = abs(vals[0][nm] - ref[nm])
        assert diff <= infos[0].abs_bound[j] + 1e-12, (nm, diff, infos[0].abs_bound[j])
        if np.isfinite(infos[0].bound[j]):
            assert diff <= EPS * abs(ref[nm]), (nm, diff)
    H.close()
