"""fj_indices_noalloc (the entry point for callers that cannot allocate)
against fj_indices on the same inputs, through the C ABI: two calls in a row,
the second on a smaller graph, so stale scratch contents from the first call
must not matter; one- and several-column, FP64 and FJ_MIXED; and a solve too
large for the static scratch is refused on the host."""
import sys

import numpy as np
import pytest

from paper_2101_08143_amd import workloads as W

pytestmark = pytest.mark.gpu

NAMES = ("internal_conflict", "disagreement", "polarization", "controversy", "dc_index")


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


def _same(fj, a, b):
    (va, ia, ra), (vb, ib, rb) = a, b
    assert ra == rb
    for c in range(len(va)):
        for j, nm in enumerate(NAMES):
            assert va[c][nm] == vb[c][nm], (c, nm, va[c][nm], vb[c][nm])
            assert ia[c].bound[j] == ib[c].bound[j] or not np.isfinite(ia[c].bound[j])
        assert ia[c].iters == ib[c].iters and ia[c].status == ib[c].status


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("k", [1, 4])
def test_noalloc_matches_workspace_entry_point(torch_fj, precision, k):
    torch, fj = torch_fj
    prec = fj.FJ_MIXED if precision == "mixed" else fj.FJ_FP64
    big = W.chung_lu(200_000, 2.2, 16.0, 71, weighted=True)
    small = W.chung_lu(30_000, 2.5, 8.0, 72)
    o = fj.make_opts(eps=1e-6, precision=prec, flags=fj.FJ_NO_TUNE)
    for name, g in (("cl200k", big), ("cl30k", small)):
        say(f"noalloc {name} k={k} {precision}")
        G = fj.Graph.from_csr(g, device="cuda:0", validate=True)
        S = torch.from_numpy(np.stack([W.opinions(kind, g.n, 80 + c)
                                       for c, kind in zip(range(k), ("uniform", "exp", "pareto", "uniform"))],
                                      axis=1).copy()).to("cuda:0")
        S = S.view(-1) if k == 1 else S
        a = fj.fj_indices_noalloc(G, S, o, check=False)
        b = fj.fj_indices(G, S, o, check=False)
        assert a[2] == fj.FJ_OK, fj.info_dict(a[1][0])
        _same(fj, a, b)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_on_the_phased_layout(torch_fj, precision):
    """The SpMV on the time-phased layout of the plan: by default on a
    600K-node graph, forced (FJ_PHASED_SPMV) on a 30K-node one (Jacobi CG);
    the no-allocation entry point matches fj_indices bit for bit."""
    torch, fj = torch_fj
    prec = fj.FJ_MIXED if precision == "mixed" else fj.FJ_FP64
    for name, g, flags in (("cl600k", W.chung_lu(600_000, 2.2, 12.0, 73, weighted=True), 0),
                           ("cl30k", W.chung_lu(30_000, 2.5, 8.0, 72), fj.FJ_PHASED_SPMV)):
        say(f"noalloc phased {name} {precision}")
        G = fj.Graph.from_csr(g, device="cuda:0", validate=True)
        s = torch.from_numpy(W.opinions("exp", g.n, 90)).to("cuda:0")
        o = fj.make_opts(eps=1e-6, precision=prec, flags=flags)
        a = fj.fj_indices_noalloc(G, s, o, check=False)
        b = fj.fj_indices(G, s, o, check=False)
        assert a[2] == fj.FJ_OK, fj.info_dict(a[1][0])
        _same(fj, a, b)


def test_noalloc_rejects_oversized_solve(torch_fj):
    torch, fj = torch_fj
    import ctypes
    # 2M nodes, one FP64 vector: about 96 MB of workspace > the 64 MiB array (checked before any GPU work)
    csr = fj.fj_csr(n=2_000_000, nnz=0, row_ptr=256, col_idx=None, val=None, val_type=fj.FJ_VAL_UNIT)
    o = fj.fj_default_opts()
    assert fj.lib().fj_workspace_bytes(ctypes.byref(csr), 1, ctypes.byref(o)) > 64 << 20
    out = (fj.fj_indices_t * 1)()
    rc = fj.lib().fj_indices_noalloc(ctypes.byref(csr), ctypes.c_void_p(256), 1, ctypes.c_void_p(256), 1,
                                     ctypes.byref(o), None, out, None)
    assert rc == fj.FJ_ERR_WORKSPACE
    assert "static scratch" in fj.last_error()
