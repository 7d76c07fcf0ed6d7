"""Block CG (FJ_BLOCK_CG: one Krylov space shared by the columns of a block,
the k x k products on the matrix cores) against the CPU oracle, column by
column, through the C ABI."""
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


GRAPHS = {
    "ba3000": lambda: W.barabasi_albert(3000, 3, 11),
    "gnp500_f64": lambda: W.random_graph(500, 0.02, 12, weighted=True),
    "cl50k_f32": lambda: W.chung_lu(50_000, 2.2, 30.0, 15, weighted=True),
    "cl100k_unit": lambda: W.chung_lu(100_000, 2.1, 20.0, 14),
    "star6001": lambda: W.csr_from_edges(6001, [(0, j) for j in range(1, 6001)]),
    "cycle4099_w": lambda: W.cycle_graph(4099, 0.8),
}


def _block(n, k, seed):
    kinds = ["uniform", "exp", "pareto"]
    return np.stack([W.opinions(kinds[c % 3], n, seed + c) for c in range(k)], axis=1).copy()


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("k", [3, 16, 20, 64])
def test_block_cg_matches_oracle(torch_fj, name, k):
    """Every column of a block CG solve (blocks of 16, 32 and 64 columns,
    padded where k is narrower) within 1e-6 of the oracle and inside its own
    certified bound."""
    torch, fj = torch_fj
    g = GRAPHS[name]()
    say(f"block cg {name} k={k} n={g.n}")
    G = fj.Graph.from_csr(g, device="cuda:0", validate=True)
    S = _block(g.n, k, 300)
    vals, infos, rc = fj.fj_indices(G, torch.from_numpy(S).to("cuda:0"),
                                    fj.make_opts(eps=EPS, flags=fj.FJ_BLOCK_CG), check=False)
    assert rc == fj.FJ_OK, [fj.info_dict(i) for i in infos[:2]]
    cols = range(k) if k <= 16 else (0, 1, k // 2, k - 1)
    for c in cols:
        ref, _, oinfo = O.indices(g, S[:, c].copy())
        assert oinfo["certified"]
        for j, nm in enumerate(NAMES):
            err = abs(vals[c][nm] - ref[nm]) / abs(ref[nm])
            assert err <= EPS and err <= infos[c].bound[j] + 1e-12, (c, nm, err, infos[c].bound[j])


def test_block_cg_solution_and_iterations(torch_fj):
    """fj_solve with FJ_BLOCK_CG: each column's z within its certified
    distance of the oracle's; iterations reported beside per-column CG."""
    torch, fj = torch_fj
    g = W.chung_lu(60_000, 2.4, 12.0, 31, weighted=True)
    say(f"block cg solve n={g.n}")
    G = fj.Graph.from_csr(g, device="cuda:0", validate=True)
    S = _block(g.n, 32, 400)
    Sd = torch.from_numpy(S).to("cuda:0")
    rtol = 1e-11
    Z, infos, rc = fj.fj_solve(G, Sd, fj.make_opts(rtol=rtol, flags=fj.FJ_BLOCK_CG))
    assert rc == fj.FJ_OK
    _, pinfos, _ = fj.fj_solve(G, Sd, fj.make_opts(rtol=rtol))
    Z = Z.cpu().numpy()
    for c in (0, 7, 31):
        zref, _ = O.solve(g, S[:, c].copy(), rtol=1e-14)
        s_norm = np.linalg.norm(S[:, c])
        assert infos[c].rel_residual <= rtol
        assert np.linalg.norm(Z[:, c] - zref) <= (infos[c].rel_residual + 1e-13) * s_norm
    say(f"iterations: block {infos[0].iters}, per column max {max(i.iters for i in pinfos)}")


def test_block_cg_is_deterministic(torch_fj):
    torch, fj = torch_fj
    g = W.chung_lu(40_000, 2.2, 16.0, 32)
    G = fj.Graph.from_csr(g, device="cuda:0", validate=True)
    Sd = torch.from_numpy(_block(g.n, 24, 500)).to("cuda:0")
    say("block cg determinism")
    o = fj.make_opts(flags=fj.FJ_BLOCK_CG)
    a = fj.fj_indices(G, Sd, o)[0]
    b = fj.fj_indices(G, Sd, o)[0]
    assert a == b


def test_block_cg_degenerate_columns(torch_fj):
    """Constant and repeated columns make the search block rank-deficient:
    their directions are dropped and the other columns still certify."""
    torch, fj = torch_fj
    g = W.barabasi_albert(5000, 3, 33)
    G = fj.Graph.from_csr(g, device="cuda:0", validate=True)
    S = _block(g.n, 16, 600)
    S[:, 3] = 0.4          # constant: z = s, P = D = C_I = 0
    S[:, 5] = S[:, 4]      # a repeated column
    say("block cg rank-deficient block")
    vals, infos, rc = fj.fj_indices(G, torch.from_numpy(S).to("cuda:0"), fj.make_opts(flags=fj.FJ_BLOCK_CG),
                                    check=False)
    assert rc == fj.FJ_ERR_UNCERTIFIABLE  # column 3 has zero indices
    assert infos[3].status == fj.FJ_ERR_UNCERTIFIABLE
    for c in (0, 4, 5, 15):
        assert infos[c].status == fj.FJ_OK
        ref, _, _ = O.indices(g, S[:, c].copy())
        for nm in NAMES:
            assert abs(vals[c][nm] - ref[nm]) <= EPS * abs(ref[nm]), (c, nm)
    assert vals[4] == vals[5] or all(abs(vals[4][nm] - vals[5][nm]) <= 1e-9 * abs(vals[4][nm]) for nm in NAMES)
    assert abs(vals[3]["controversy"] - g.n * 0.16) <= 1e-9 * g.n * 0.16
