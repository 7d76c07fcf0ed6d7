"""The continuous-batching server through the C ABI: results certified and
matching the oracle, each request's result bitwise the same alone and in the
mix, admission by HBM footprint, error paths."""
import sys

import numpy as np
import pytest

from oracle import sparse as O
from paper_2101_08143_amd import workloads as W

pytestmark = pytest.mark.gpu
NAMES = ("internal_conflict", "disagreement", "polarization", "controversy", "dc_index")


def say(msg):
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2101_08143_amd import fj
    graphs = [W.barabasi_albert(3000, 3, 11), W.chung_lu(50_000, 2.2, 30.0, 15, weighted=True),
              W.chung_lu(100_000, 2.1, 20.0, 14), W.random_graph(400, 0.03, 13, weighted=True)]
    G = []
    for g in graphs:
        say(f"prepare n={g.n}")
        G.append(fj.Graph.from_csr(g, device="cuda:0"))
    rng = np.random.default_rng(9)
    reqs = []
    for r in range(40):
        gi = int(rng.integers(0, len(graphs)))
        k = int(rng.integers(1, 17))
        S = np.ascontiguousarray(rng.random((graphs[gi].n, k)))
        reqs.append((gi, S))
    return torch, fj, graphs, G, reqs


PRECISIONS = ["fp64", "mixed"]


def _prec(fj, precision):
    return fj.FJ_MIXED if precision == "mixed" else fj.FJ_FP64


def _run(fj, torch, G, reqs, arena_bytes, block_columns=16, precision="fp64", **server_kw):
    srv = fj.Server(arena_bytes, block_columns=block_columns, iters_per_replay=6, precision=_prec(fj, precision),
                    **server_kw)
    gids = [srv.add_graph(g) for g in G]
    ids = [srv.submit(gids[gi], torch.from_numpy(S).to("cuda:0")) for gi, S in reqs]
    res = {r["id"]: r for r in srv.drain(timeout_s=240)}
    srv.close()
    return [res[i] for i in ids]


@pytest.mark.parametrize("precision", PRECISIONS)
def test_server_certified_and_matches_oracle(env, precision):
    torch, fj, graphs, G, reqs = env
    say(f"server mixed run {precision}")
    mixed = _run(fj, torch, G, reqs, 1 << 30, precision=precision)
    assert all(r["status"] == fj.FJ_OK for r in mixed)
    for (gi, S), r in list(zip(reqs, mixed))[:8]:
        for c in range(0, S.shape[1], 5):
            ref, _, _ = O.indices(graphs[gi], S[:, c])
            for name in NAMES:
                assert abs(r["values"][c][name] - ref[name]) <= 1e-6 * abs(ref[name])
    env_cache[precision] = mixed


env_cache = {}


@pytest.mark.parametrize("precision", PRECISIONS)
def test_server_result_same_alone_and_in_mix(env, precision):
    torch, fj, graphs, G, reqs = env
    mixed = env_cache.get(precision) or _run(fj, torch, G, reqs, 1 << 30, precision=precision)
    for idx in (0, 7, 19, 33):
        say(f"alone request {idx} {precision}")
        alone = _run(fj, torch, G, [reqs[idx]], 1 << 30, precision=precision)[0]
        assert alone["values"] == mixed[idx]["values"], idx


@pytest.mark.parametrize("precision", PRECISIONS)
def test_server_several_blocks_per_large_graph(env, precision):
    """Every graph large (large_entries = 1) with 3 blocks each: requests spread
    over a graph's blocks, report the caller's graph id, and give bitwise the
    results of the one-block server (a column's arithmetic never depends on
    its block)."""
    torch, fj, graphs, G, reqs = env
    say(f"three blocks per graph {precision}")
    ref = env_cache.get(precision) or _run(fj, torch, G, reqs, 1 << 30, precision=precision)
    res = _run(fj, torch, G, reqs, 4 << 30, precision=precision, large_entries=1, large_blocks=3)
    for (gi, _), a, b in zip(reqs, res, ref):
        assert a["status"] == fj.FJ_OK and a["graph"] == gi
        assert a["values"] == b["values"]


@pytest.mark.parametrize("precision", PRECISIONS)
def test_server_admission_by_footprint(env, precision):
    """An arena that holds only one block at a time: requests on other graphs
    wait until an idle block can be released, and all still complete certified."""
    torch, fj, graphs, G, reqs = env
    biggest = max(g.n for g in graphs)
    arena = fj.Server.block_bytes(biggest, 16, _prec(fj, precision)) + 4096
    say(f"small arena {precision}")
    res = _run(fj, torch, G, reqs[:12], arena, precision=precision)
    assert all(r["status"] == fj.FJ_OK for r in res)
    ref = env_cache.get(precision)
    if ref:
        for a, b in zip(res, ref[:12]):
            assert a["values"] == b["values"]


def test_server_errors(env):
    torch, fj, graphs, G, reqs = env
    srv = fj.Server(1 << 20, block_columns=16)
    gid = srv.add_graph(G[2])
    with pytest.raises(fj.FJError) as e:  # the 100k-node block cannot fit a 1 MiB arena
        srv.submit(gid, torch.zeros((graphs[2].n, 2), dtype=torch.float64, device="cuda:0"))
    assert e.value.status == fj.FJ_ERR_WORKSPACE
    gid0 = srv.add_graph(G[3])
    with pytest.raises(fj.FJError) as e:
        srv.submit(gid0, torch.zeros((graphs[3].n, 17), dtype=torch.float64, device="cuda:0"))
    assert e.value.status == fj.FJ_ERR_INVALID_ARG
    srv.close()
    with pytest.raises(fj.FJError) as e:
        fj.Server(1 << 20, block_columns=16, precision=7)
    assert e.value.status == fj.FJ_ERR_INVALID_ARG
    with pytest.raises(fj.FJError) as e:
        fj.Server(1 << 20, block_columns=16, large_blocks=5)
    assert e.value.status == fj.FJ_ERR_INVALID_ARG
    assert fj.Server.block_bytes(1000, 16, 7) == 0


@pytest.mark.parametrize("precision", PRECISIONS)
def test_server_rejects_opinions_out_of_range(env, precision):
    """A request whose opinions leave [0, 1] comes back FJ_ERR_OPINION_RANGE;
    the requests sharing its block are unaffected."""
    torch, fj, graphs, G, reqs = env
    say(f"server range check {precision}")
    bad = np.array(reqs[2][1], copy=True)
    bad[5, 0] = 1.5
    res = _run(fj, torch, G, [reqs[2], (reqs[2][0], bad), reqs[3]], 1 << 30, precision=precision)
    assert res[1]["status"] == fj.FJ_ERR_OPINION_RANGE
    assert res[0]["status"] == fj.FJ_OK and res[2]["status"] == fj.FJ_OK
    ref = env_cache.get(precision)
    if ref:
        assert res[0]["values"] == ref[2]["values"] and res[2]["values"] == ref[3]["values"]


@pytest.mark.parametrize("precision", PRECISIONS)
def test_server_graph_replays_equal_eager_batched_path(env, precision):
    """Server columns come from replayed HIP graphs interleaved with eager
    admission and epilogue kernels; a 16-vector request must equal the eager
    batched fj_indices on the same 16 vectors (same block width and
    precision), bitwise, also when it enters the block in pieces."""
    torch, fj, graphs, G, reqs = env
    rng = np.random.default_rng(3)
    for gi in (1, 2):
        S = np.ascontiguousarray(rng.random((graphs[gi].n, 16)))
        say(f"replay vs eager graph {gi} {precision}")
        eager, _, rc = fj.fj_indices(G[gi], torch.from_numpy(S).to("cuda:0"),
                                     fj.make_opts(precision=_prec(fj, precision)))
        assert rc == fj.FJ_OK
        served = _run(fj, torch, G, [(gi, S), reqs[0], reqs[1], (gi, S)], 1 << 30, precision=precision)
        assert served[0]["values"] == eager
        assert served[3]["values"] == eager


@pytest.mark.parametrize("precision", PRECISIONS)
def test_server_cancel(env, precision):
    """Cancelling a queued request and one already iterating: both come back
    FJ_ERR_CANCELLED, the freed columns take later requests, and the other
    requests still give their results bitwise."""
    torch, fj, graphs, G, reqs = env
    say(f"server cancel {precision}")
    srv = fj.Server(1 << 30, block_columns=16, iters_per_replay=6, precision=_prec(fj, precision))
    gids = [srv.add_graph(g) for g in G]
    picks = [r for r in reqs if r[0] == 1][:4]
    ids = [srv.submit(gids[gi], torch.from_numpy(S).to("cuda:0")) for gi, S in picks]
    srv.step()  # admits what fits and starts iterating
    srv.cancel(ids[0])
    srv.cancel(ids[-1])
    with pytest.raises(fj.FJError):
        srv.cancel(12345678)
    res = {r["id"]: r for r in srv.drain(timeout_s=240)}
    assert res[ids[0]]["status"] == fj.FJ_ERR_CANCELLED and res[ids[-1]]["status"] == fj.FJ_ERR_CANCELLED
    alone = _run(fj, torch, G, picks[1:3], 1 << 30, precision=precision)
    for rid, ref in zip(ids[1:3], alone):
        assert res[rid]["status"] == fj.FJ_OK and res[rid]["values"] == ref["values"]
    srv.close()


@pytest.fixture(scope="module")
def serving_config():
    """The serving workload at full size: 32 Chung-Lu graphs (n log-uniform in
    [1e4, 2e6]) resident on the device, 16 U[0,1] vectors per graph."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2101_08143_amd import fj
    graphs, G, pools = [], [], []
    for p in W.serving_graph_params():
        g = W.serving_graph(p)
        say(f"serving graph seed={p['seed']} n={g.n} nnz={g.nnz}")
        graphs.append(g)
        G.append(fj.Graph.from_csr(g, device="cuda:0"))
        pools.append(np.random.default_rng(p["seed"] + 11).random((g.n, 16)))
    return torch, fj, graphs, G, pools


@pytest.mark.slow
@pytest.mark.parametrize("precision", PRECISIONS)
def test_serving_full_size_sampled(serving_config, precision):
    """96 requests of 1-16 vectors on the 32 full-size serving graphs, submitted
    at once (16-column blocks, 8 captured iterations per replay, as the
    benchmark runs them): every request certified; sampled columns on the
    largest, the smallest and four other graphs within 1e-6 of the oracle."""
    torch, fj, graphs, G, pools = serving_config
    reqs = W.serving_requests(96, len(graphs), seed=3100, kmax=16)
    srv = fj.Server(96 << 30, block_columns=16, iters_per_replay=8, precision=_prec(fj, precision))
    gids = [srv.add_graph(g) for g in G]
    say(f"serving full size {precision}")
    ids = [srv.submit(gids[gi], torch.from_numpy(np.ascontiguousarray(pools[gi][:, :k])).to("cuda:0"))
           for gi, k, _ in reqs]
    res = {r["id"]: r for r in srv.drain(timeout_s=240)}
    srv.close()
    assert all(res[i]["status"] == fj.FJ_OK for i in ids)
    by_size = sorted(range(len(graphs)), key=lambda gi: graphs[gi].nnz)
    wanted = [by_size[-1], by_size[0]] + by_size[8:32:6]
    checked = 0
    for gi in wanted:
        hits = [j for j, (g2, _, _) in enumerate(reqs) if g2 == gi]
        if not hits:
            continue
        j = hits[0]
        k = reqs[j][1]
        for c in sorted({0, k - 1}):
            say(f"oracle graph {gi} column {c}")
            ref, _, _ = O.indices(graphs[gi], pools[gi][:, c])
            for name in NAMES:
                assert abs(res[ids[j]]["values"][c][name] - ref[name]) <= 1e-6 * abs(ref[name]), (gi, c, name)
        checked += 1
    assert checked >= 4
