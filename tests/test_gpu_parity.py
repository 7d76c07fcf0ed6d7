"""GPU path vs the CPU oracle, through the C ABI (libfjgpu via the ctypes
binding). Every case prints its name before touching the GPU."""
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


def small_graphs():
    """Graphs that span several windows, ragged tails, hubs longer than the
    LDS stage, isolated nodes and empty rows at both ends."""
    iso_edges = [(i, i + 1) for i in range(3000, 3500)] + [(3000, j) for j in range(3600, 4700)]
    return {
        "path5": W.path_graph(5),
        "ba3000": W.barabasi_albert(3000, 3, 11),
        "gnp500_f64": W.random_graph(500, 0.02, 12, weighted=True),
        "gnp400_f32": W.random_graph(400, 0.03, 13, weighted=True, val_dtype=np.float32),
        "cl100k_unit": W.chung_lu(100_000, 2.1, 20.0, 14),
        "cl50k_f32": W.chung_lu(50_000, 2.2, 30.0, 15, weighted=True),
        "star6001": W.csr_from_edges(6001, [(0, j) for j in range(1, 6001)]),
        "isolated9000": W.csr_from_edges(9000, iso_edges),
        "cycle4099_w": W.cycle_graph(4099, 0.8),
    }


@pytest.fixture(scope="module")
def graphs(torch_fj):
    torch, fj = torch_fj
    out = {}
    for name, g in small_graphs().items():
        say(f"prepare {name} n={g.n} nnz={g.nnz}")
        out[name] = (g, fj.Graph.from_csr(g, device="cuda:0", validate=True))
    torch.cuda.synchronize()
    return out


def _tolerance_apply(g, x):
    w = np.abs(g.weights_f64())
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    mag = np.abs(x) * (1 + np.bincount(rows, weights=w, minlength=g.n))
    mag += np.bincount(rows, weights=w * np.abs(x[g.col]), minlength=g.n)
    return 1e-13 * mag + 1e-300


@pytest.mark.parametrize("name", list(small_graphs().keys()))
def test_apply_matches_oracle(torch_fj, graphs, name):
    torch, fj = torch_fj
    g, G = graphs[name]
    say(f"apply {name}")
    x = np.random.default_rng(1).standard_normal(g.n)
    y = fj.fj_apply(G, torch.from_numpy(x).to("cuda:0")).cpu().numpy()
    ref = O.apply(g, x)
    assert np.all(np.abs(y - ref) <= _tolerance_apply(g, x))


def _random_case(seed):
    """A graph of random family, size, weights and opinion law (seeded)."""
    rng = np.random.default_rng(seed)
    fam = seed % 5
    if fam == 0:
        g = W.random_graph(int(rng.integers(20, 3000)), float(rng.uniform(0.002, 0.05)), seed,
                           weighted=bool(rng.integers(0, 2)), val_dtype=np.float32 if rng.integers(0, 2) else np.float64)
    elif fam == 1:
        g = W.barabasi_albert(int(rng.integers(50, 20000)), int(rng.integers(1, 6)), seed)
    elif fam == 2:
        g = W.chung_lu(int(rng.integers(1000, 60000)), float(rng.uniform(2.05, 3.0)), float(rng.uniform(2, 40)), seed,
                       weighted=bool(rng.integers(0, 2)))
    elif fam == 3:
        g = W.cycle_graph(int(rng.integers(3, 50000)), float(rng.uniform(0.1, 5.0)))
    else:
        g = W.torus_graph(int(rng.integers(3, 200)), int(rng.integers(3, 200)))
    kind = ["uniform", "exp", "pareto"][seed % 3]
    return g, W.opinions(kind, g.n, seed + 1)


@pytest.mark.parametrize("seed", list(range(40)))
def test_random_graphs_match_oracle(torch_fj, seed):
    """Forty seeded graphs of mixed families (G(n,p), Barabasi-Albert,
    Chung-Lu, weighted cycles, tori), sizes, weight types and opinion laws:
    FP64 indices within 1e-6 of the oracle and inside their own bounds; the
    mixed path certified too."""
    torch, fj = torch_fj
    g, s = _random_case(seed)
    say(f"random graph seed={seed} n={g.n} nnz={g.nnz}")
    G = fj.Graph.from_csr(g, device="cuda:0", validate=True)
    ref, zref, oinfo = O.indices(g, s)
    # the oracle's own absolute error per index (its certificate, rho ~ 1e-13 ||s||)
    rho_o = oinfo["relres"] * float(np.linalg.norm(s))
    o_abs = [rho_o * (2 * np.sqrt(max(ref[nm], 0.0)) + rho_o) for nm in NAMES[:4]]
    o_abs.append((np.sqrt(ref["controversy"]) + rho_o) * rho_o)
    sd = torch.from_numpy(s).to("cuda:0")
    for prec in (fj.FJ_FP64, fj.FJ_MIXED):
        vals, infos, rc = fj.fj_indices(G, sd, fj.make_opts(eps=EPS, precision=prec), check=False)
        inf0 = infos[0]
        # an uncertifiable index is only acceptable where the oracle cannot certify it either
        if rc == fj.FJ_ERR_UNCERTIFIABLE:
            assert not oinfo["certified"], (prec, fj.info_dict(inf0), oinfo["bounds"])
        else:
            assert rc == fj.FJ_OK, (prec, fj.info_dict(inf0))
        for j, nm in enumerate(NAMES):
            diff = abs(vals[0][nm] - ref[nm])
            # every index: within the absolute bound of both certificates
            assert diff <= inf0.abs_bound[j] + o_abs[j] + 1e-300, (prec, nm, diff, inf0.abs_bound[j])
            if np.isfinite(inf0.bound[j]):  # and, where it has one, within its relative bound
                err = diff / abs(ref[nm])
                assert err <= EPS and err <= inf0.bound[j] + 1e-12, (prec, nm, err)


@pytest.mark.parametrize("name", ["cl50k_f32", "gnp500_f64", "star6001", "isolated9000"])
def test_gather_bound_probe(torch_fj, graphs, name):
    """The measurement aid fj_gather_bound computes y[t] = sum of w_e x[col_e]
    over entries 8t .. 8t+7 (a padded tail counts zero)."""
    torch, fj = torch_fj
    g, G = graphs[name]
    say(f"gather bound {name}")
    x = np.random.default_rng(7).random(g.n)
    y = fj.fj_gather_bound(G, torch.from_numpy(x).to("cuda:0")).cpu().numpy()
    pad = (-g.nnz) % 8
    prod = np.concatenate([g.weights_f64() * x[g.col], np.zeros(pad)]).reshape(-1, 8)
    assert np.allclose(y, prod.sum(axis=1), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("name", ["cl50k_f32", "gnp500_f64", "star6001", "isolated9000", "path5", "gnp400_f32"])
@pytest.mark.parametrize("xbytes", [8, 4])
def test_gather_bound_sliced(torch_fj, graphs, name, xbytes):
    """fj_gather_bound_sliced: one stream reproduces fj_gather_bound bitwise;
    eight streams hold exactly the entries the slicing rule gives them (tail
    ranges from the returned edges, hub entries dealt in eight equal runs in
    CSR order), each in CSR order, and every workgroup is counted."""
    torch, fj = torch_fj
    g, G = graphs[name]
    say(f"gather sliced {name} x{8 * xbytes}")
    x64 = np.random.default_rng(8).random(g.n)
    x = x64 if xbytes == 8 else x64.astype(np.float32)
    xd = torch.from_numpy(x).to("cuda:0")
    xs = x.astype(np.float64)
    w = g.weights_f64()
    y1, _ = fj.fj_gather_bound_sliced(G, xd, slices=1)
    if xbytes == 8:
        y0 = fj.fj_gather_bound(G, xd).cpu().numpy()
        assert np.array_equal(y1.cpu().numpy()[:len(y0)], y0)
    for hub in (0, g.n // 16):
        check = torch.zeros(2, dtype=torch.int32, device="cuda:0")
        y8, b = fj.fj_gather_bound_sliced(G, xd, slices=8, hub_cols=hub, check=check)
        y8 = y8.cpu().numpy()
        assert b[0] == min(hub, g.n) and b[8] == g.n and all(b[s] <= b[s + 1] for s in range(8))
        col = g.col.astype(np.int64)
        is_hub = col < b[0]
        tail_cnt = np.bincount(np.searchsorted(b[1:8], col[~is_hub], side="right"), minlength=8)
        if (~is_hub).any():  # ranges balanced up to one column's entries
            per_col = np.bincount(col, minlength=g.n)
            assert tail_cnt.max() <= (~is_hub).sum() / 8 + per_col[b[0]:].max() + 1
        hub_rank = np.cumsum(is_hub) - 1
        sid = np.where(is_hub, hub_rank * 8 // max(int(is_hub.sum()), 1),
                       np.searchsorted(b[1:8], col, side="right"))
        prod = w * xs[col]
        at = 0
        for s_ in range(8):
            ps = prod[sid == s_]
            ps = np.concatenate([ps, np.zeros((-len(ps)) % 8)]).reshape(-1, 8).sum(axis=1)
            assert np.allclose(y8[at:at + len(ps)], ps, rtol=1e-13, atol=1e-13), (hub, s_)
            at += len(ps)
        hits, wgs = check.cpu().numpy().tolist()
        assert wgs >= 8 and wgs % 8 == 0 and 0 <= hits <= wgs
        say(f"  hub {hub}: {hits} of {wgs} workgroups on XCD b % 8")


@pytest.mark.parametrize("name", [n for n in small_graphs() if n not in ("path5",)])
@pytest.mark.parametrize("kind", ["uniform", "exp"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_indices_match_oracle(torch_fj, graphs, name, kind, precision):
    torch, fj = torch_fj
    g, G = graphs[name]
    s = W.opinions(kind, g.n, 21)
    say(f"indices {name} {kind} {precision}")
    prec = fj.FJ_MIXED if precision == "mixed" else fj.FJ_FP64
    vals, infos, rc = fj.fj_indices(G, torch.from_numpy(s).to("cuda:0"), fj.make_opts(eps=EPS, precision=prec),
                                    check=False)
    ref, _, oinfo = O.indices(g, s)
    assert oinfo["status"] == 0 and oinfo["certified"]
    assert rc == fj.FJ_OK, (fj.fj_status_string(rc), fj.info_dict(infos[0]))
    for c, k in enumerate(NAMES):
        err = abs(vals[0][k] - ref[k]) / abs(ref[k])
        assert err <= EPS, (k, vals[0][k], ref[k], err)
        assert err <= infos[0].bound[c] + 1e-12, (k, err, infos[0].bound[c])


@pytest.mark.parametrize("name", ["ba3000", "cl100k_unit", "cl50k_f32", "star6001", "isolated9000"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_matches_oracle(torch_fj, graphs, name, precision):
    torch, fj = torch_fj
    g, G = graphs[name]
    s = W.opinions("uniform", g.n, 22)
    say(f"solve {name} {precision}")
    rtol = 1e-11
    prec = fj.FJ_MIXED if precision == "mixed" else fj.FJ_FP64
    z, infos, rc = fj.fj_solve(G, torch.from_numpy(s).to("cuda:0"), fj.make_opts(rtol=rtol, precision=prec))
    z = z.cpu().numpy()
    zref, oinfo = O.solve(g, s, rtol=1e-14)
    assert infos[0].rel_residual <= rtol
    # ||z - z_true|| <= ||s - (I+L) z|| because I <= I + L
    bound = infos[0].rel_residual * np.linalg.norm(s) + 1e-13 * np.linalg.norm(s)
    assert np.linalg.norm(z - zref) <= bound
    assert np.abs(z.sum() - s.sum()) <= 1e-9 * s.sum()


def test_p5_solve_reproduces_printed_forest_matrix(torch_fj, graphs):
    """Section 2.2 worked example: (I+L)^{-1} e_j for P5 is column j of the printed Omega."""
    torch, fj = torch_fj
    g, G = graphs["path5"]
    import oracle_pins
    total, _, M = oracle_pins.load_p5_golden()
    say("p5 columns")
    for j in range(5):
        s = np.eye(5)[:, j]
        z, _, _ = fj.fj_solve(G, torch.from_numpy(s).to("cuda:0"), fj.make_opts(rtol=1e-14))
        assert np.allclose(z.cpu().numpy() * total, M[:, j], rtol=0, atol=1e-11)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_bitwise_deterministic(torch_fj, graphs, precision):
    torch, fj = torch_fj
    g, G = graphs["cl100k_unit"]
    s = torch.from_numpy(W.opinions("uniform", g.n, 23)).to("cuda:0")
    say(f"determinism {precision}")
    o = fj.make_opts(precision=fj.FJ_MIXED if precision == "mixed" else fj.FJ_FP64)
    a = fj.fj_indices(G, s, o)[0][0]
    b = fj.fj_indices(G, s, o)[0][0]
    assert a == b
    z1 = fj.fj_solve(G, s, o)[0].cpu().numpy()
    z2 = fj.fj_solve(G, s, o)[0].cpu().numpy()
    assert np.array_equal(z1, z2)


def test_degenerate_cases(torch_fj, graphs):
    torch, fj = torch_fj
    dev = "cuda:0"
    # constant opinions: z = s and P = D = C_I = 0, so no relative bound exists
    g, G = graphs["ba3000"]
    say("constant s")
    s = np.full(g.n, 0.4)
    vals, infos, rc = fj.fj_indices(G, torch.from_numpy(s).to(dev), check=False)
    assert rc == fj.FJ_ERR_UNCERTIFIABLE
    assert abs(vals[0]["controversy"] - g.n * 0.16) <= 1e-9 * g.n * 0.16
    assert abs(vals[0]["dc_index"] - g.n * 0.16) <= 1e-9 * g.n * 0.16
    for k in ("internal_conflict", "disagreement", "polarization"):
        assert vals[0][k] <= 1e-20
    # the absolute bounds stand in for the missing relative ones: exact values P = D = C_I = 0, C = I_dc = 0.16 n
    exact = dict(internal_conflict=0.0, disagreement=0.0, polarization=0.0, controversy=g.n * 0.16,
                 dc_index=g.n * 0.16)
    for j, k in enumerate(NAMES):
        assert np.isfinite(infos[0].abs_bound[j]) and abs(vals[0][k] - exact[k]) <= infos[0].abs_bound[j], k
    assert infos[0].residual_norm >= 0.0 and np.isfinite(infos[0].residual_norm)
    # edgeless graph: z = s, D = C_I = 0
    ge = W.csr_from_edges(257, np.zeros((0, 2), dtype=np.int64))
    say("edgeless")
    Ge = fj.Graph.from_csr(ge, device=dev)
    s = W.opinions("uniform", 257, 3)
    vals, infos, rc = fj.fj_indices(Ge, torch.from_numpy(s).to(dev), check=False)
    assert rc == fj.FJ_ERR_UNCERTIFIABLE
    sb = s - s.mean()
    assert abs(vals[0]["polarization"] - sb @ sb) <= 1e-12 * (sb @ sb)
    assert abs(vals[0]["controversy"] - s @ s) <= 1e-12 * (s @ s)
    assert vals[0]["disagreement"] == 0.0 and vals[0]["internal_conflict"] == 0.0
    exact = dict(internal_conflict=0.0, disagreement=0.0, polarization=float(sb @ sb), controversy=float(s @ s),
                 dc_index=float(s @ s))
    for j, k in enumerate(NAMES):
        assert abs(vals[0][k] - exact[k]) <= infos[0].abs_bound[j], k
    assert not np.isfinite(infos[0].bound[0]) and not np.isfinite(infos[0].bound[1])
    # edgeless and large enough for the block preconditioner: no pairs, M = I
    gb = W.csr_from_edges(70_000, np.zeros((0, 2), dtype=np.int64))
    say("edgeless 70000")
    Gb = fj.Graph.from_csr(gb, device=dev)
    s = W.opinions("uniform", gb.n, 4)
    z, _, rc = fj.fj_solve(Gb, torch.from_numpy(s).to(dev))
    assert rc == fj.FJ_OK and np.abs(z.cpu().numpy() - s).max() <= 1e-15
    # a star larger than the threshold: the hub pairs with one leaf, the other leaves stay single
    gs = W.csr_from_edges(70_001, [(0, j) for j in range(1, 70_001)])
    say("star 70001")
    Gs = fj.Graph.from_csr(gs, device=dev, validate=True)
    s = W.opinions("uniform", gs.n, 5)
    vals, infos, rc = fj.fj_indices(Gs, torch.from_numpy(s).to(dev), check=False)
    ref, _, _ = O.indices(gs, s)
    assert rc == fj.FJ_OK
    for nm in NAMES:
        assert abs(vals[0][nm] - ref[nm]) <= EPS * abs(ref[nm]), nm
    # one node
    g1 = W.csr_from_edges(1, np.zeros((0, 2), dtype=np.int64))
    say("single node")
    G1 = fj.Graph.from_csr(g1, device=dev)
    z, _, rc = fj.fj_solve(G1, torch.tensor([0.3], dtype=torch.float64, device=dev))
    assert rc == fj.FJ_OK and z.cpu().numpy()[0] == 0.3


def test_error_paths(torch_fj, graphs):
    torch, fj = torch_fj
    dev = "cuda:0"
    g, G = graphs["ba3000"]
    s = W.opinions("uniform", g.n, 4)
    say("opinion range")
    bad = s.copy()
    bad[17] = 1.5
    _, _, rc = fj.fj_indices(G, torch.from_numpy(bad).to(dev), check=False)
    assert rc == fj.FJ_ERR_OPINION_RANGE
    bad[17] = np.nan
    _, _, rc = fj.fj_indices(G, torch.from_numpy(bad).to(dev), check=False)
    assert rc == fj.FJ_ERR_OPINION_RANGE
    say("no range check")
    shifted = s * 3.0 - 1.0
    vals, _, rc = fj.fj_indices(G, torch.from_numpy(shifted).to(dev),
                                fj.make_opts(flags=fj.FJ_NO_RANGE_CHECK), check=False)
    ref, _, _ = O.indices(g, shifted)
    assert rc == fj.FJ_OK
    for k in NAMES:
        assert abs(vals[0][k] - ref[k]) <= EPS * abs(ref[k])
    say("iteration cap")
    vals, infos, rc = fj.fj_indices(G, torch.from_numpy(s).to(dev), fj.make_opts(max_iter=1), check=False)
    assert rc == fj.FJ_ERR_NOT_CONVERGED and infos[0].iters == 1
    say("workspace too small")
    ws = torch.empty(1024, dtype=torch.uint8, device=dev)
    _, _, rc = fj.fj_indices(G, torch.from_numpy(s).to(dev), ws=ws, check=False)
    assert rc == fj.FJ_ERR_WORKSPACE
    say("invalid graphs")
    for rp, col in (([0, 1, 1, 1], [1]),            # asymmetric
                    ([0, 1, 2, 2], [0, 0]),         # self-loop
                    ([0, 1, 2, 2], [5, 0])):        # column out of range
        bad_g = W.CSRGraph(n=3, row_ptr=np.array(rp, np.int32), col=np.array(col, np.int32))
        with pytest.raises(fj.FJError) as e:
            fj.Graph.from_csr(bad_g, device=dev)
        assert e.value.status == fj.FJ_ERR_INVALID_GRAPH


# ---------------------------------------------------------------- full sizes


_ORACLE_CACHE = {}


@pytest.mark.slow
@pytest.mark.parametrize("name", ["ba10k", "cl1m", "cl4m"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_size_workloads(torch_fj, name, precision):
    """The configured workloads at full size: all five indices within 1e-6 of
    the oracle, the reported bounds valid, and z within the certified
    residual, for the FP64 path and the FP32-inner / FP64-refined path."""
    torch, fj = torch_fj
    g, s, spec = W.workload(name)
    say(f"full {name} {precision} n={g.n} nnz={g.nnz}")
    G = fj.Graph.from_csr(g, device="cuda:0", validate=True)
    prec = fj.FJ_MIXED if precision == "mixed" else fj.FJ_FP64
    opts = fj.make_opts(eps=EPS, rtol=spec["rtol"], precision=prec)
    sd = torch.from_numpy(s).to("cuda:0")
    vals, infos, rc = fj.fj_indices(G, sd, opts, check=False)
    assert rc == fj.FJ_OK, fj.info_dict(infos[0])
    if name not in _ORACLE_CACHE:
        say(f"oracle {name}")
        ref, zref, oinfo = O.indices(g, s)
        assert oinfo["certified"], oinfo
        _ORACLE_CACHE[name] = (ref, zref)
    ref, zref = _ORACLE_CACHE[name]
    for c, k in enumerate(NAMES):
        err = abs(vals[0][k] - ref[k]) / abs(ref[k])
        assert err <= EPS, (k, err)
        assert err <= infos[0].bound[c] + 1e-12
    z, zinfo, rc = fj.fj_solve(G, sd, opts)
    assert rc == fj.FJ_OK
    diff = np.linalg.norm(z.cpu().numpy() - zref)
    assert diff <= (zinfo[0].rel_residual + 1e-13) * np.linalg.norm(s)
    del G
    torch.cuda.empty_cache()


# ---------------------------------------------------------------- k columns

def _block(n, k, seed):
    kinds = ["uniform", "exp", "pareto"]
    return W.opinion_block(n, [kinds[c % 3] for c in range(k)], seed)


@pytest.mark.parametrize("k", [2, 3, 16, 64, 70])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_indices_match_oracle(torch_fj, graphs, k, precision):
    """k opinion vectors in one call (one CSR pass per iteration for all of
    them): every column's five indices within 1e-6 of the oracle."""
    torch, fj = torch_fj
    g, G = graphs["cl50k_f32"]
    S = _block(g.n, k, 100 + k)
    say(f"batched indices k={k} {precision}")
    prec = fj.FJ_MIXED if precision == "mixed" else fj.FJ_FP64
    vals, infos, rc = fj.fj_indices(G, torch.from_numpy(S).to("cuda:0"), fj.make_opts(eps=EPS, precision=prec),
                                    check=False)
    assert rc == fj.FJ_OK, [fj.info_dict(i) for i in infos if i.status != 0][:2]
    for c in range(k) if k <= 16 else range(0, k, 7):
        ref, _, _ = O.indices(g, S[:, c])
        for j, name in enumerate(NAMES):
            err = abs(vals[c][name] - ref[name]) / abs(ref[name])
            assert err <= EPS, (c, name, err)
            assert err <= infos[c].bound[j] + 1e-12


@pytest.mark.parametrize("name", ["cl50k_f32", "star6001", "gnp500_f64"])
@pytest.mark.parametrize("k", [3, 16])
@pytest.mark.parametrize("cpl", [1, 2, 4])
@pytest.mark.parametrize("split", [1, 0])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_every_spmm_shape_matches_oracle(torch_fj, name, k, cpl, split, precision):
    """Each SpMM launch shape the autotuner can pick (columns per lane, full or
    a small grid, items split over lane groups or one group per row), pinned in
    turn on a freshly prepared graph: certified indices within 1e-6 of the
    oracle."""
    torch, fj = torch_fj
    g = small_graphs()[name]
    G = fj.Graph.from_csr(g, device="cuda:0", validate=False)
    kb = 4 if k == 3 else 16
    prec = fj.FJ_MIXED if precision == "mixed" else fj.FJ_FP64
    S = _block(g.n, k, 300 + k)
    say(f"spmm shape {name} k={k} cpl={cpl} split={split} {precision}")
    grid = 64 if cpl == 2 else 512
    fj.fj_spmm_set_choice(G, kb, cpl, grid, precision=prec, split=split)
    assert fj.fj_spmm_choice(G, kb, prec) == (cpl, grid, split, 1)
    vals, infos, rc = fj.fj_indices(G, torch.from_numpy(S).to("cuda:0"), fj.make_opts(eps=EPS, precision=prec),
                                    check=False)
    assert rc == fj.FJ_OK
    for c in range(k):
        ref, _, _ = O.indices(g, S[:, c])
        for j, nm in enumerate(NAMES):
            err = abs(vals[c][nm] - ref[nm]) / abs(ref[nm])
            assert err <= EPS and err <= infos[c].bound[j] + 1e-12, (c, nm, err)


@pytest.mark.parametrize("name", ["cl50k_f32", "star6001", "gnp500_f64"])
@pytest.mark.parametrize("k,kb,passes", [(20, 32, 2), (64, 64, 2), (40, 64, 4)])
@pytest.mark.parametrize("cpl", [1, 2])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_column_passes_match_oracle(torch_fj, name, k, kb, passes, cpl, precision):
    """The column-pass SpMM shapes for wide blocks (2 passes of 16 or 32
    columns, 4 of 16; one lane group per row), pinned on a freshly prepared
    graph: certified indices within 1e-6 of the oracle (sampled columns)."""
    torch, fj = torch_fj
    g = small_graphs()[name]
    G = fj.Graph.from_csr(g, device="cuda:0", validate=False)
    prec = fj.FJ_MIXED if precision == "mixed" else fj.FJ_FP64
    S = _block(g.n, k, 700 + k)
    say(f"spmm passes {name} k={k} passes={passes} cpl={cpl} {precision}")
    fj.fj_spmm_set_choice(G, kb, cpl, 512, precision=prec, split=0, passes=passes)
    assert fj.fj_spmm_choice(G, kb, prec) == (cpl, 512, 0, passes)
    vals, infos, rc = fj.fj_indices(G, torch.from_numpy(S).to("cuda:0"), fj.make_opts(eps=EPS, precision=prec),
                                    check=False)
    assert rc == fj.FJ_OK
    for c in range(0, k, 5):
        ref, _, _ = O.indices(g, S[:, c])
        for j, nm in enumerate(NAMES):
            err = abs(vals[c][nm] - ref[nm]) / abs(ref[nm])
            assert err <= EPS and err <= infos[c].bound[j] + 1e-12, (c, nm, err)


def test_batched_autotuner_records_a_shape(torch_fj):
    """The first batched solve of a fresh (graph, width, precision) tunes and
    caches a shape; FJ_NO_TUNE runs the default shape; both are certified."""
    torch, fj = torch_fj
    g = small_graphs()["cl100k_unit"]
    G = fj.Graph.from_csr(g, device="cuda:0", validate=False)
    S = torch.from_numpy(_block(g.n, 16, 401)).to("cuda:0")
    say("spmm autotuner")
    assert fj.fj_spmm_choice(G, 16, fj.FJ_FP64) is None
    v0, _, rc0 = fj.fj_indices(G, S, fj.make_opts(eps=EPS, flags=fj.FJ_NO_TUNE), check=False)
    assert rc0 == fj.FJ_OK and fj.fj_spmm_choice(G, 16, fj.FJ_FP64) is None
    v1, _, rc1 = fj.fj_indices(G, S, fj.make_opts(eps=EPS), check=False)
    assert rc1 == fj.FJ_OK
    cpl, grid, split, passes = fj.fj_spmm_choice(G, 16, fj.FJ_FP64)
    assert cpl in (1, 2, 4) and 1 <= grid <= 4096 and split in (0, 1) and passes == 1
    v2, _, _ = fj.fj_indices(G, S, fj.make_opts(eps=EPS), check=False)
    assert v2 == v1  # the cached choice is reused: bitwise repeatable
    for c in range(16):
        for nm in NAMES:
            assert abs(v0[c][nm] - v1[c][nm]) <= 2 * EPS * abs(v0[c][nm])


@pytest.mark.parametrize("k", [1, 16])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_zero_and_mean_start_both_match_oracle(torch_fj, graphs, k, precision):
    """By default every CG solve starts from mean(s) 1 (its residual is the
    centred s, since (I + L) 1 = 1) and runs deflated; FJ_ZERO_START gives
    plain Jacobi-PCG from 0. Both certify and match the oracle; the deflated
    FP64 solves need fewer iterations, the mixed ones no more."""
    torch, fj = torch_fj
    g, G = graphs["cl100k_unit"]
    say(f"zero vs mean start k={k} {precision}")
    prec = fj.FJ_MIXED if precision == "mixed" else fj.FJ_FP64
    S = _block(g.n, k, 500 + k)
    Sd = torch.from_numpy(S if k > 1 else S[:, 0].copy()).to("cuda:0")
    res = {}
    for flags in (0, fj.FJ_ZERO_START):
        vals, infos, rc = fj.fj_indices(G, Sd, fj.make_opts(eps=EPS, precision=prec, flags=flags), check=False)
        assert rc == fj.FJ_OK
        res[flags] = (vals, infos)
    for c in range(0, k, 5):
        ref, _, _ = O.indices(g, S[:, c])
        for flags, (vals, infos) in res.items():
            for nm in NAMES:
                assert abs(vals[c][nm] - ref[nm]) <= EPS * abs(ref[nm]), (flags, c, nm)
    its = {f: max(inf.iters for inf in infos) for f, (_, infos) in res.items()}
    if precision == "fp64":
        assert its[0] < its[fj.FJ_ZERO_START], its
    else:
        assert its[0] <= its[fj.FJ_ZERO_START], its


@pytest.mark.parametrize("name", ["cl100k_unit", "cl50k_f32", "ba3000"])
@pytest.mark.parametrize("k", [1, 8])
def test_deflated_cg_keeps_the_mean_and_saves_iterations(torch_fj, graphs, name, k):
    """The default FP64 solve (one vector, or a batch of columns) runs CG
    deflated by the constant vector: every iterate keeps mean(x) = mean(s)
    (which the exact z satisfies, since 1^T (I + L) = 1^T), the solution
    matches the oracle's, and it needs fewer iterations than plain Jacobi-PCG
    from zero (a CPU model of both predicts 17 against 21 on cl100k_unit)."""
    torch, fj = torch_fj
    g, G = graphs[name]
    say(f"deflated CG {name} k={k}")
    S = np.random.default_rng(5).random((g.n, k))
    Sd = torch.from_numpy(S if k > 1 else S[:, 0].copy()).to("cuda:0")
    its = {}
    Z = {}
    for flags in (0, fj.FJ_ZERO_START):
        z, info, rc = fj.fj_solve(G, Sd, fj.make_opts(rtol=1e-10, flags=flags))
        assert rc == fj.FJ_OK
        Z[flags] = z.cpu().numpy().reshape(g.n, k)
        its[flags] = max(i.iters for i in info)
    for c in range(k):
        s = S[:, c]
        zref, _ = O.solve(g, s, rtol=1e-14)
        for flags in Z:
            assert np.linalg.norm(Z[flags][:, c] - zref) <= 1.1e-10 * np.linalg.norm(s), (flags, c)
        assert abs(Z[0][:, c].mean() - s.mean()) <= 1e-13 * s.mean(), c
    assert its[0] <= its[fj.FJ_ZERO_START] - 2, its


@pytest.mark.parametrize("name", ["cl50k_f32", "cl100k_unit"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_warm_start(torch_fj, graphs, precision, name):
    """FJ_WARM_START: from the converged z no iteration runs and z is returned
    as it was; from a perturbed z the solve converges to the oracle's z in
    fewer iterations than from zero; k > 1 is refused. (cl100k_unit: with
    the 2x2 block preconditioner.)"""
    torch, fj = torch_fj
    g, G = graphs[name]
    say(f"warm start {name} {precision}")
    prec = fj.FJ_MIXED if precision == "mixed" else fj.FJ_FP64
    s = np.random.default_rng(41).random(g.n)
    sd = torch.from_numpy(s).to("cuda:0")
    o = fj.make_opts(rtol=1e-10, precision=prec)
    ow = fj.make_opts(rtol=1e-10, precision=prec, flags=fj.FJ_WARM_START)
    z_cold, info_cold, rc = fj.fj_solve(G, sd, o)
    assert rc == fj.FJ_OK
    z0 = z_cold.clone()
    z_w, info_w, rc = fj.fj_solve(G, sd, ow, Z=z0)
    assert rc == fj.FJ_OK and info_w[0].iters == 0 and torch.equal(z_w, z_cold)
    zp = z_cold + 1e-4 * torch.from_numpy(np.random.default_rng(42).standard_normal(g.n)).to("cuda:0")
    z_p, info_p, rc = fj.fj_solve(G, sd, ow, Z=zp.clone())
    assert rc == fj.FJ_OK and info_p[0].iters < info_cold[0].iters
    zref, _ = O.solve(g, s, rtol=1e-14)
    assert np.linalg.norm(z_p.cpu().numpy() - zref) <= 1.1e-10 * np.linalg.norm(s)
    S2 = torch.from_numpy(_block(g.n, 2, 5)).to("cuda:0")
    Z2 = torch.zeros_like(S2)
    _, _, rc = fj.fj_solve(G, S2, ow, Z=Z2, check=False)
    assert rc == fj.FJ_ERR_INVALID_ARG


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_solve_matches_oracle(torch_fj, graphs, precision):
    torch, fj = torch_fj
    g, G = graphs["cl100k_unit"]
    S = _block(g.n, 5, 7)
    say(f"batched solve {precision}")
    prec = fj.FJ_MIXED if precision == "mixed" else fj.FJ_FP64
    Z, infos, rc = fj.fj_solve(G, torch.from_numpy(S).to("cuda:0"), fj.make_opts(rtol=1e-11, precision=prec))
    Z = Z.cpu().numpy()
    for c in range(5):
        zref, _ = O.solve(g, S[:, c], rtol=1e-14)
        assert infos[c].rel_residual <= 1e-11
        assert np.linalg.norm(Z[:, c] - zref) <= (infos[c].rel_residual + 1e-13) * np.linalg.norm(S[:, c])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_column_alone_equals_column_in_mix(torch_fj, graphs, precision):
    """A column's result does not depend on the other columns of its block:
    alone (the rest zero) or among 63 others, bitwise."""
    torch, fj = torch_fj
    g, G = graphs["cl50k_f32"]
    S = _block(g.n, 64, 55)
    prec = fj.FJ_MIXED if precision == "mixed" else fj.FJ_FP64
    o = fj.make_opts(precision=prec)
    say(f"alone vs mix {precision}")
    mix, _, _ = fj.fj_indices(G, torch.from_numpy(S).to("cuda:0"), o, check=False)
    zmix = fj.fj_solve(G, torch.from_numpy(S).to("cuda:0"), o, check=False)[0].cpu().numpy()
    for c in (0, 17, 63):
        A = np.zeros_like(S)
        A[:, c] = S[:, c]
        alone, _, _ = fj.fj_indices(G, torch.from_numpy(A).to("cuda:0"), o, check=False)
        assert alone[c] == mix[c], c
        zal = fj.fj_solve(G, torch.from_numpy(A).to("cuda:0"), o, check=False)[0].cpu().numpy()
        assert np.array_equal(zal[:, c], zmix[:, c])


@pytest.mark.parametrize("name", ["ba3000", "cl50k_f32", "isolated9000"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_two_solve_literal_algorithm(torch_fj, graphs, name, precision):
    """FJ_TWO_SOLVE: Algorithm 1 as printed (solves for s and for s - mean(s);
    D and P from the second, C_I and C from the first, I_dc = D + C)."""
    torch, fj = torch_fj
    g, G = graphs[name]
    s = W.opinions("exp", g.n, 31)
    say(f"two-solve {name} {precision}")
    prec = fj.FJ_MIXED if precision == "mixed" else fj.FJ_FP64
    vals, infos, rc = fj.fj_indices(G, torch.from_numpy(s).to("cuda:0"),
                                    fj.make_opts(eps=EPS, precision=prec, flags=fj.FJ_TWO_SOLVE), check=False)
    assert rc == fj.FJ_OK, fj.info_dict(infos[0])
    ref, _, _ = O.indices(g, s)
    for j, k in enumerate(NAMES):
        err = abs(vals[0][k] - ref[k]) / abs(ref[k])
        assert err <= EPS, (k, err)
        assert err <= infos[0].bound[j] + 1e-12


@pytest.mark.slow
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_full_size_batched_k64(torch_fj, precision):
    """The 1M-node Chung-Lu graph with k = 64 opinion vectors (21 uniform, 21
    exponential, 22 Pareto, min-max scaled): all columns certified; sampled
    columns checked against the oracle."""
    torch, fj = torch_fj
    g, _, _ = W.workload("cl1m")
    S = W.opinion_block(g.n, ["uniform"] * 21 + ["exp"] * 21 + ["pareto"] * 22, 2004)
    say(f"full k64 {precision}")
    G = fj.Graph.from_csr(g, device="cuda:0", validate=True)
    prec = fj.FJ_MIXED if precision == "mixed" else fj.FJ_FP64
    vals, infos, rc = fj.fj_indices(G, torch.from_numpy(S).to("cuda:0"), fj.make_opts(eps=EPS, precision=prec),
                                    check=False)
    assert rc == fj.FJ_OK
    for c in (0, 20, 21, 41, 42, 63):
        say(f"oracle column {c}")
        ref, _, _ = O.indices(g, S[:, c])
        for j, k in enumerate(NAMES):
            err = abs(vals[c][k] - ref[k]) / abs(ref[k])
            assert err <= EPS, (c, k, err)
    del G
    torch.cuda.empty_cache()


def test_concurrent_calls_on_distinct_workspaces(torch_fj, graphs):
    """The ABI is thread-safe for calls that use distinct workspaces: six host
    threads, each with its own stream and workspaces, run single (two of them
    block preconditioned on one shared plan), batched and mixed-precision
    index solves on shared graphs at the same time; every result is bitwise
    the one the same call gives alone."""
    import threading
    torch, fj = torch_fj
    say("concurrent calls")
    jobs = []
    for t, (name, k, prec) in enumerate([("cl50k_f32", 1, fj.FJ_FP64), ("cl100k_unit", 4, fj.FJ_FP64),
                                         ("ba3000", 1, fj.FJ_MIXED), ("cl50k_f32", 8, fj.FJ_MIXED),
                                         ("cl100k_unit", 1, fj.FJ_FP64), ("cl100k_unit", 1, fj.FJ_MIXED)]):
        g, G = graphs[name]
        S = np.random.default_rng(60 + t).random((g.n, k))
        Sd = torch.from_numpy(S if k > 1 else S[:, 0].copy()).to("cuda:0")
        o = fj.make_opts(eps=EPS, precision=prec)
        jobs.append((G, Sd, o, G.workspace(k, o), torch.cuda.Stream()))
    ref = [fj.fj_indices(G, Sd, o, ws=ws)[0] for G, Sd, o, ws, _ in jobs]
    torch.cuda.synchronize()
    got = [[] for _ in jobs]
    errors = []

    def worker(j):
        G, Sd, o, ws, st = jobs[j]
        try:
            for _ in range(3):
                got[j].append(fj.fj_indices(G, Sd, o, ws=ws, stream=st)[0])
        except Exception as e:  # reported below; the other threads keep going
            errors.append((j, repr(e)))

    threads = [threading.Thread(target=worker, args=(j,)) for j in range(len(jobs))]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for j in range(len(jobs)):
        assert len(got[j]) == 3 and all(v == ref[j] for v in got[j]), j


@pytest.mark.parametrize("name", ["cl50k_f32", "cl100k_unit"])
@pytest.mark.parametrize("k", [1, 4])
@pytest.mark.parametrize("zero_start", [False, True])
def test_restart_passes_certify(torch_fj, graphs, k, zero_start, name):
    """A loose first-pass residual target (rtol 1e-3) cannot certify 1e-6, so
    the solve restarts from the true residual with a tighter target (a second
    pass, deflated or plain; on cl100k_unit with one vector, block
    preconditioned) and then certifies; the indices match the oracle."""
    torch, fj = torch_fj
    g, G = graphs[name]
    say(f"restart passes {name} k={k} zero_start={zero_start}")
    S = _block(g.n, k, 700 + k)
    Sd = torch.from_numpy(S if k > 1 else S[:, 0].copy()).to("cuda:0")
    flags = fj.FJ_ZERO_START if zero_start else 0
    vals, infos, rc = fj.fj_indices(G, Sd, fj.make_opts(eps=EPS, rtol=1e-3, flags=flags), check=False)
    assert rc == fj.FJ_OK
    assert max(i.passes for i in infos) >= 2
    for c in range(k):
        ref, _, _ = O.indices(g, S[:, c])
        for j, nm in enumerate(NAMES):
            err = abs(vals[c][nm] - ref[nm]) / abs(ref[nm])
            assert err <= EPS and err <= infos[c].bound[j] + 1e-12, (c, nm, err)


def _skewed_weights(g, span, seed):
    """The same graph with weights log-uniform over a factor `span`, equal in
    both directions of every edge (a hash of the edge's end points)."""
    return W.log_uniform_weights(g, span, seed)


@pytest.mark.parametrize("span", [4.0, 1e4])
def test_pair_preconditioner(torch_fj, span):
    """One-vector FP64 solves of graphs of >= 65536 nodes use 2x2 blocks of
    I + L on a heavy-edge matching: on a graph whose weights spread over a
    factor 1e4 they need far fewer iterations than Jacobi (FJ_DIAG_PRECOND;
    a CPU model of both: 67 against 119 to relative residual 1e-9), and both
    match the oracle's z and indices."""
    torch, fj = torch_fj
    g = _skewed_weights(W.chung_lu(100_000, 2.5, 10.0, 31), span, 7)
    say(f"pair preconditioner span={span:g} n={g.n} nnz={g.nnz}")
    G = fj.Graph.from_csr(g, device="cuda:0", validate=True)
    s = W.opinions("uniform", g.n, 32)
    sd = torch.from_numpy(s).to("cuda:0")
    zref, _ = O.solve(g, s, rtol=1e-14)
    ref, _, _ = O.indices(g, s)
    its = {}
    for flags in (0, fj.FJ_DIAG_PRECOND):
        z, info, rc = fj.fj_solve(G, sd, fj.make_opts(rtol=1e-10, flags=flags))
        assert rc == fj.FJ_OK
        assert np.linalg.norm(z.cpu().numpy() - zref) <= 1.1e-10 * np.linalg.norm(s), flags
        its[flags] = info[0].iters
        vals, infos, rc = fj.fj_indices(G, sd, fj.make_opts(eps=EPS, flags=flags))
        assert rc == fj.FJ_OK
        for j, nm in enumerate(NAMES):
            err = abs(vals[0][nm] - ref[nm]) / abs(ref[nm])
            assert err <= EPS and err <= infos[0].bound[j] + 1e-12, (flags, nm, err)
    if span > 100:
        assert its[0] <= 0.75 * its[fj.FJ_DIAG_PRECOND], its
    else:
        assert its[0] <= its[fj.FJ_DIAG_PRECOND], its


@pytest.mark.parametrize("name", ["ba3000", "cl50k_f32", "gnp500_f64", "isolated9000", "path5"])
def test_reorder_by_degree_keeps_indices(torch_fj, graphs, name):
    """A randomly relabelled graph, reordered by degree: a valid CSR (checked
    by fj_prepare's validation) with non-increasing degrees, whose certified
    indices with the permuted opinions match the oracle's for the original
    labels, and whose z comes back to those labels through the inverse
    permutation."""
    import dataclasses
    torch, fj = torch_fj
    g, _ = graphs[name]
    rng = np.random.default_rng(17)
    lab = rng.permutation(g.n)  # old node o becomes node lab[o]
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    keep = rows < g.col  # each undirected edge once
    w = None if g.val is None else g.val[keep]
    edges = np.stack([lab[rows[keep]], lab[g.col[keep]]], axis=1)
    gr = W.csr_from_edges(g.n, edges.tolist(), None if w is None else w.tolist(),
                          val_dtype=np.float64 if g.val is None else g.val.dtype)
    if g.val is None:
        gr = dataclasses.replace(gr, val=None)
    say(f"reorder {name} n={g.n}")
    Gr = fj.Graph.from_csr(gr, device="cuda:0", validate=True)
    G2, perm = fj.reorder_by_degree(Gr, validate=True)
    p = perm.cpu().numpy()
    assert np.array_equal(np.sort(p), np.arange(g.n))
    deg2 = np.diff(G2.row_ptr.cpu().numpy())
    assert np.all(deg2[:-1] >= deg2[1:])
    s = W.opinions("uniform", g.n, 23)
    sr = np.empty_like(s)
    sr[lab] = s  # the opinions in the random labels
    ref, _, _ = O.indices(g, s)
    s2 = fj.permute(perm, torch.from_numpy(sr).to("cuda:0"))
    vals, infos, rc = fj.fj_indices(G2, s2, fj.make_opts(eps=EPS), check=False)
    assert rc in (fj.FJ_OK, fj.FJ_ERR_UNCERTIFIABLE)
    for j, nm in enumerate(NAMES):
        diff = abs(vals[0][nm] - ref[nm])
        assert diff <= infos[0].abs_bound[j] + 1e-12, (nm, diff)
        if np.isfinite(infos[0].bound[j]):
            assert diff <= EPS * abs(ref[nm]), (nm, diff)
    z2, _, rc = fj.fj_solve(G2, s2, fj.make_opts(rtol=1e-12))
    assert rc == fj.FJ_OK
    zr = fj.permute(perm, z2, inverse=True).cpu().numpy()  # random labels
    zref, _ = O.solve(g, s, rtol=1e-14)
    assert np.abs(zr[lab] - zref).max() <= 1e-10
