"""Host-side checks that need no GPU: the library loads, exports every
function include/fj.h declares, rejects bad arguments before touching the
device, and the row-window partition the kernels assume holds on the
generated workloads."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_2101_08143_amd import build as B
from paper_2101_08143_amd import fj
from paper_2101_08143_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fj.h")
KERNELS = os.path.join(ROOT, "paper_2101_08143_amd", "csrc", "fj_kernels.hpp")


@pytest.fixture(scope="module")
def lib():
    if B.stale():
        B.build()
    return fj.lib()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fj_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert sorted(fj.EXPORTS) == declared_functions()


def test_library_exports_every_declared_function(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for code in range(0, 12):
        assert fj.fj_status_string(code) not in ("", "unknown status")
    assert fj.fj_status_string(99) == "unknown status"


def test_sizes_are_pure_host_functions(lib):
    csr = fj.fj_csr(n=1000, nnz=5000, row_ptr=1, col_idx=1, val=None, val_type=fj.FJ_VAL_UNIT)
    pb = lib.fj_plan_bytes(ctypes.byref(csr))
    o = fj.fj_default_opts()
    wb1 = lib.fj_workspace_bytes(ctypes.byref(csr), 1, ctypes.byref(o))
    assert pb > 1000 * 4 and pb % 256 == 0
    assert wb1 >= 4 * 8 * 1000 and wb1 % 256 == 0
    bad = fj.fj_csr(n=-1, nnz=0, row_ptr=None, col_idx=None, val=None, val_type=0)
    assert lib.fj_plan_bytes(ctypes.byref(bad)) == 0
    assert lib.fj_workspace_bytes(ctypes.byref(csr), 0, ctypes.byref(o)) == 0


def test_argument_errors_are_caught_on_the_host(lib):
    """Each of these returns before any HIP call, so it runs without a GPU."""
    csr = fj.fj_csr(n=10, nnz=20, row_ptr=256, col_idx=512, val=None, val_type=fj.FJ_VAL_UNIT)
    o = fj.fj_default_opts()
    out = (fj.fj_indices_t * 1)()
    info = (fj.fj_info * 1)()
    call = lambda c, o_, k=1, lds=1: lib.fj_indices(ctypes.byref(c), ctypes.c_void_p(256), k,
                                                   ctypes.c_void_p(256), lds, ctypes.byref(o_),
                                                   ctypes.c_void_p(256), 1 << 30, None, out, info)
    for eps in (0.0, 0.5, -1.0, float("nan")):
        oo = fj.fj_default_opts()
        oo.eps = eps
        assert call(csr, oo) == fj.FJ_ERR_INVALID_ARG
    oo = fj.fj_default_opts()
    oo.reserved = 1
    assert call(csr, oo) == fj.FJ_ERR_INVALID_ARG
    assert call(csr, o, k=1, lds=0) == fj.FJ_ERR_INVALID_ARG
    badval = fj.fj_csr(n=10, nnz=20, row_ptr=256, col_idx=512, val=1024, val_type=fj.FJ_VAL_UNIT)
    assert call(badval, o) == fj.FJ_ERR_INVALID_ARG
    badtype = fj.fj_csr(n=10, nnz=20, row_ptr=256, col_idx=512, val=1024, val_type=7)
    assert call(badtype, o) == fj.FJ_ERR_INVALID_ARG
    nonodes = fj.fj_csr(n=0, nnz=4, row_ptr=256, col_idx=512, val=None, val_type=0)
    assert lib.fj_prepare(ctypes.byref(nonodes), None, ctypes.c_void_p(256), 1 << 20, None) == \
        fj.FJ_ERR_INVALID_GRAPH
    # the sliced gather aid: 1 or 8 streams, 4- or 8-byte x, hub_cols >= 0
    for sl, xb, hub in ((3, 8, 0), (8, 2, 0), (8, 8, -1), (0, 8, 0)):
        assert lib.fj_gather_bound_sliced(ctypes.byref(csr), ctypes.c_void_p(256), xb, ctypes.c_void_p(256), sl, hub,
                                          None, None, None) == fj.FJ_ERR_INVALID_ARG
    # misaligned or undersized plan
    assert lib.fj_prepare(ctypes.byref(csr), None, ctypes.c_void_p(257), 1 << 20, None) == fj.FJ_ERR_WORKSPACE
    assert lib.fj_prepare(ctypes.byref(csr), None, ctypes.c_void_p(256), 16, None) == fj.FJ_ERR_WORKSPACE


def _constants():
    src = open(KERNELS).read()
    win = int(re.search(r"#define FJ_WIN (\d+)", src).group(1))
    assert "constexpr int LONGROW = WIN / 2;" in src
    return win, win // 2


def _windows(g, WIN):
    key = g.row_ptr[:-1].astype(np.int64) + np.arange(g.n)
    K = (g.n + g.nnz + WIN - 1) // WIN
    blk = np.searchsorted(key, np.arange(K + 1, dtype=np.int64) * WIN, side="left")
    blk[-1] = g.n
    return K, blk


@pytest.mark.parametrize("name", ["ba", "cl_unit", "cl_weighted", "star", "isolated"])
def test_window_partition_invariants(name):
    """Rows per window <= WIN and staged entries < WIN + LONGROW: the LDS
    capacity the window pass relies on (mirrors k_windows on the CPU)."""
    WIN, LONGROW = _constants()
    if name == "ba":
        g = W.barabasi_albert(5000, 3, 1)
    elif name == "cl_unit":
        g = W.chung_lu(200_000, 2.1, 20.0, 2)
    elif name == "cl_weighted":
        g = W.chung_lu(100_000, 2.2, 30.0, 3, weighted=True)
    elif name == "star":
        g = W.csr_from_edges(6001, [(0, j) for j in range(1, 6001)])
    else:
        edges = [(i, i + 1) for i in range(3000, 3500)]
        g = W.csr_from_edges(9000, edges)
    K, blk = _windows(g, WIN)
    rp = g.row_ptr.astype(np.int64)
    covered = 0
    for k in range(K):
        r0, r1 = blk[k], blk[k + 1]
        assert r0 <= r1
        if r0 == r1:
            continue
        covered += r1 - r0
        assert r1 - r0 <= WIN
        elast, eend = rp[r1 - 1], rp[r1]
        long_last = eend - elast > LONGROW
        ns = (elast if long_last else eend) - rp[r0]
        assert 0 <= ns < WIN + LONGROW
    assert covered == g.n


def test_apriori_delta(lib):
    """Algorithm 1's delta (its first line) for a 10^4-node unit-weight graph
    and U[0,1] opinions: about 1e-23, far below FP64 resolution, which is why
    the library certifies a posteriori instead."""
    n, sbar = 10_000, (10_000 / 12) ** 0.5
    d = fj.fj_apriori_delta(n, 1.0, 1.0, sbar, 1e-6)
    assert d == pytest.approx(1e-6 * sbar / (3 * n**3 * (n + 1) * n**0.5), rel=1e-12)
    assert 5e-24 < d < 2e-23 and d < 2.0**-52
    assert fj.fj_apriori_delta(4_000_000, 0.5, 2.0, 100.0, 1e-6) < 1e-34
    assert math.isnan(fj.fj_apriori_delta(0, 1.0, 1.0, 1.0, 1e-6))
    assert math.isnan(fj.fj_apriori_delta(10, 1.0, 1.0, 1.0, 0.5))


API = os.path.join(ROOT, "paper_2101_08143_amd", "csrc", "fj_api.hip")
GUARD_DIR = os.path.join(ROOT, "paper_2101_08143_amd", "csrc")


def test_every_status_entry_point_is_guarded():
    """Every extern "C" function that returns a status runs its body through
    guarded() (no C++ exception crosses the ABI)."""
    src = open(API).read()
    body = src.split('extern "C" {', 1)[1]
    csrc = os.path.dirname(API)
    for inc in re.findall(r'^#include "(fj_\w+\.hpp)"', body, flags=re.M):  # entry points kept in headers
        body += open(os.path.join(csrc, inc)).read()
    sigs = re.findall(r"^int (fj_\w+)\([^{]*\{\n([^\n]*)\n", body, flags=re.M)
    for name, first in sigs:
        assert first.strip() == "return guarded([&]() -> int {", name
    header = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    declared = set(re.findall(r"^int (fj_\w+)\(", header, flags=re.M))
    assert declared and declared <= {name for name, _ in sigs}, declared - {name for name, _ in sigs}


def test_guard_maps_exceptions_to_status(tmp_path):
    """An allocation failure planted on the CPU (and any other exception) comes
    out of guarded() as a status code and a message, never as an exception."""
    prog = tmp_path / "guard.cpp"
    prog.write_text(r'''
#include <cstdio>
#include <cstring>
#include <new>
#include <stdexcept>
#include <type_traits>
#include "fj_guard.hpp"
char* volatile sink = nullptr;
int main() {
    auto ok = []() -> int { return 0; };
    static_assert(noexcept(fj::guarded(ok)), "guarded must be noexcept");
    const int a = fj::guarded([]() -> int {
        volatile size_t huge = size_t(1) << 62;
        sink = new char[huge];  // fails: no such address space (kept, so it cannot be elided)
        return FJ_OK;
    });
    const bool ma = std::strstr(fj::g_last_error, "allocation") != nullptr;
    const int b = fj::guarded([]() -> int { throw std::runtime_error("planted"); });
    const bool mb = std::strstr(fj::g_last_error, "planted") != nullptr;
    const int c = fj::guarded([]() -> int { throw 7; });
    const int d = fj::guarded([]() -> int { return FJ_ERR_WORKSPACE; });
    std::printf("%d %d %d %d %d %d\n", a, b, c, d, ma ? 1 : 0, mb ? 1 : 0);
    return 0;
}
''')
    exe = tmp_path / "guard"
    import subprocess
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", GUARD_DIR, "-o", str(exe), str(prog)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    assert [int(x) for x in out] == [fj.FJ_ERR_HOST_MEMORY, fj.FJ_ERR_INTERNAL, fj.FJ_ERR_INTERNAL,
                                    fj.FJ_ERR_WORKSPACE, 1, 1]


def test_info_layout_matches_header():
    """fj_info in the binding has the header's fields in the header's order."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct fj_info \{(.*?)\} fj_info;", src, flags=re.S).group(1)
    fields = re.findall(r"(\w+)(?:\[\d+\])?;", body)
    assert fields == [f[0] for f in fj.fj_info._fields_]


def test_block_cg_argument_errors(lib):
    """FJ_BLOCK_CG is FP64 only, needs k >= 2, and excludes FJ_TWO_SOLVE and
    FJ_WARM_START (checked before any device work)."""
    csr = fj.fj_csr(n=10, nnz=20, row_ptr=256, col_idx=512, val=None, val_type=fj.FJ_VAL_UNIT)
    out = (fj.fj_indices_t * 4)()
    for prec, flags, k in ((fj.FJ_MIXED, fj.FJ_BLOCK_CG, 4), (fj.FJ_FP64, fj.FJ_BLOCK_CG, 1),
                           (fj.FJ_FP64, fj.FJ_BLOCK_CG | fj.FJ_TWO_SOLVE, 4),
                           (fj.FJ_FP64, fj.FJ_BLOCK_CG | fj.FJ_WARM_START, 4)):
        o = fj.make_opts(precision=prec, flags=flags)
        rc = lib.fj_indices(ctypes.byref(csr), ctypes.c_void_p(256), k, ctypes.c_void_p(256), k,
                            ctypes.byref(o), ctypes.c_void_p(256), 1 << 30, None, out, None)
        assert rc == fj.FJ_ERR_INVALID_ARG, (prec, flags, k)
    o = fj.make_opts(flags=fj.FJ_BLOCK_CG)
    assert lib.fj_workspace_bytes(ctypes.byref(csr), 3, ctypes.byref(o)) > \
        lib.fj_workspace_bytes(ctypes.byref(csr), 3, ctypes.byref(fj.make_opts()))


def test_spmm_shape_rules(lib):
    """Column passes only for 32- and 64-column blocks, rows design, cpl <= 2
    and at least 16 columns per pass (checked before any device work)."""
    csr = fj.fj_csr(n=10, nnz=20, row_ptr=256, col_idx=512, val=None, val_type=fj.FJ_VAL_UNIT)
    bad = [(16, 1, 0, 2), (32, 1, 0, 4), (64, 1, 1, 2), (64, 4, 0, 2), (64, 1, 0, 3)]
    for kb, cpl, split, passes in bad:
        assert lib.fj_spmm_set_choice(ctypes.byref(csr), kb, 0, cpl, 64, split, passes) == fj.FJ_ERR_INVALID_ARG, \
            (kb, cpl, split, passes)


def test_opts_layout_matches_header():
    """fj_opts in the binding has the header's fields in the header's order."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct fj_opts \{(.*?)\} fj_opts;", src, flags=re.S).group(1)
    fields = re.findall(r"\*?(\w+);", body)
    assert fields == [f[0] for f in fj.fj_opts._fields_]
    assert ctypes.sizeof(fj.fj_opts) == 40


def test_multilevel_argument_errors(lib):
    """FJ_MULTILEVEL needs FP64 and a hierarchy, excludes FJ_DIAG_PRECOND and
    FJ_BLOCK_CG and fj_indices_noalloc; the hierarchy calls check their
    arguments (all before any device work)."""
    csr = fj.fj_csr(n=10, nnz=20, row_ptr=256, col_idx=512, val=None, val_type=fj.FJ_VAL_UNIT)
    out = (fj.fj_indices_t * 4)()
    fake = 4096  # never dereferenced: every case fails before the hierarchy is read
    for prec, flags, h, k in ((fj.FJ_FP64, fj.FJ_MULTILEVEL, None, 1), (fj.FJ_MIXED, fj.FJ_MULTILEVEL, fake, 1),
                              (fj.FJ_FP64, fj.FJ_MULTILEVEL | fj.FJ_DIAG_PRECOND, fake, 1),
                              (fj.FJ_FP64, fj.FJ_MULTILEVEL | fj.FJ_BLOCK_CG, fake, 4),
                              (fj.FJ_FP64, fj.FJ_MULTILEVEL | fj.FJ_TWO_SOLVE, fake, 1)):
        o = fj.make_opts(precision=prec, flags=flags)
        o.hierarchy = h
        rc = lib.fj_indices(ctypes.byref(csr), ctypes.c_void_p(256), k, ctypes.c_void_p(256), k,
                            ctypes.byref(o), ctypes.c_void_p(256), 1 << 30, None, out, None)
        assert rc == fj.FJ_ERR_INVALID_ARG, (prec, flags, h, k)
    o = fj.make_opts(flags=fj.FJ_MULTILEVEL)
    o.hierarchy = fake
    assert lib.fj_indices_noalloc(ctypes.byref(csr), ctypes.c_void_p(256), 1, ctypes.c_void_p(256), 1,
                                  ctypes.byref(o), None, out, None) == fj.FJ_ERR_INVALID_ARG
    h = ctypes.c_void_p()
    assert lib.fj_hierarchy_create(ctypes.byref(csr), 0, None, None) == fj.FJ_ERR_INVALID_ARG
    assert lib.fj_hierarchy_create(ctypes.byref(csr), -1, ctypes.byref(h), None) == fj.FJ_ERR_INVALID_ARG
    assert lib.fj_hierarchy_destroy(None) == fj.FJ_OK
    lv = ctypes.c_int32(0)
    assert lib.fj_hierarchy_shape(None, ctypes.byref(lv), None, None, None) == fj.FJ_ERR_INVALID_ARG


def test_server_option_errors(lib):
    """fj_server_create checks its options before any device work."""
    base = dict(arena=4096, arena_bytes=1 << 20, block_columns=16, iters_per_replay=8, eps=1e-6, max_iter=0,
                precision=fj.FJ_FP64, large_lanes=0, large_iters_per_replay=0, large_blocks=0, large_entries=0)
    h = ctypes.c_void_p()
    for field, bad in (("large_blocks", 5), ("large_blocks", -1), ("large_lanes", 9), ("block_columns", 32),
                       ("iters_per_replay", 0), ("large_entries", -1)):
        o = fj.fj_server_opts(**{**base, field: bad})
        assert lib.fj_server_create(ctypes.byref(o), ctypes.byref(h)) == fj.FJ_ERR_INVALID_ARG, field


def test_reorder_and_permute_argument_errors(lib):
    """fj_reorder_by_degree needs its outputs; fj_permute needs k >= 1,
    strides >= k, inverse 0 or 1 and distinct arrays (all before device work)."""
    csr = fj.fj_csr(n=10, nnz=20, row_ptr=256, col_idx=512, val=1024, val_type=fj.FJ_VAL_F32)
    p = ctypes.c_void_p(4096)
    assert lib.fj_reorder_by_degree(ctypes.byref(csr), None, p, p, p, None) == fj.FJ_ERR_INVALID_ARG
    assert lib.fj_reorder_by_degree(ctypes.byref(csr), p, p, p, None, None) == fj.FJ_ERR_INVALID_ARG
    x, y = ctypes.c_void_p(4096), ctypes.c_void_p(8192)
    for n, k, ldx, ldy, inv, xx, yy in ((10, 0, 1, 1, 0, x, y), (10, 2, 1, 2, 0, x, y), (10, 1, 1, 1, 2, x, y),
                                        (10, 1, 1, 1, 0, x, x), (-1, 1, 1, 1, 0, x, y)):
        assert lib.fj_permute(n, k, p, xx, ldx, yy, ldy, inv, None) == fj.FJ_ERR_INVALID_ARG
    assert lib.fj_permute(0, 1, None, None, 1, None, 1, 0, None) == fj.FJ_OK


def test_phased_layout_arguments(lib):
    """The plan holds the time-phased layout (about 4 + value + 2 bytes per
    entry and 16 per node more); FJ_WINDOW_SPMV and FJ_PHASED_SPMV exclude
    each other; fj_apply_phased checks its arguments (all before device work)."""
    unit = fj.fj_csr(n=1000, nnz=5000, row_ptr=256, col_idx=512, val=None, val_type=fj.FJ_VAL_UNIT)
    f64 = fj.fj_csr(n=1000, nnz=5000, row_ptr=256, col_idx=512, val=1024, val_type=fj.FJ_VAL_F64)
    pu, pd = lib.fj_plan_bytes(ctypes.byref(unit)), lib.fj_plan_bytes(ctypes.byref(f64))
    assert pd - pu >= 8 * 5000  # the FP64 weights of the layout
    assert pu >= 6 * 5000 + 12 * 1000
    out = (fj.fj_indices_t * 1)()
    o = fj.make_opts(flags=fj.FJ_WINDOW_SPMV | fj.FJ_PHASED_SPMV)
    rc = lib.fj_indices(ctypes.byref(unit), ctypes.c_void_p(256), 1, ctypes.c_void_p(256), 1,
                        ctypes.byref(o), ctypes.c_void_p(256), 1 << 30, None, out, None)
    assert rc == fj.FJ_ERR_INVALID_ARG
    empty = fj.fj_csr(n=0, nnz=0, row_ptr=None, col_idx=None, val=None, val_type=fj.FJ_VAL_UNIT)
    assert lib.fj_apply_phased(ctypes.byref(empty), ctypes.c_void_p(256), None, None, None) == fj.FJ_OK
    assert lib.fj_apply_phased(ctypes.byref(unit), None, ctypes.c_void_p(256), ctypes.c_void_p(512),
                               None) == fj.FJ_ERR_WORKSPACE
    assert lib.fj_apply_phased(ctypes.byref(unit), ctypes.c_void_p(256), None, ctypes.c_void_p(512),
                               None) == fj.FJ_ERR_INVALID_ARG
    assert lib.fj_apply_phased(ctypes.byref(unit), ctypes.c_void_p(256), ctypes.c_void_p(512),
                               ctypes.c_void_p(512), None) == fj.FJ_ERR_INVALID_ARG


def _plan_bytes_model(n, nnz, vb):
    """fj_plan_bytes written out from the plan layout include/fj.h describes:
    row windows, descriptors, diagonal, matching, flags, then the time-phased
    layout in bench.py's reading (chunks, phases, slots reserved)."""
    import bench

    def up(x):
        return (x + 255) // 256 * 256
    K = -(-(n + nnz) // 1024)
    off = 0
    for size in (4 * (K + 1), 32 * K, 4 * n, 4 * n, 8 * n, 4 * n, 4 * n, 4 * 64):
        off = up(off + size)
    W, P, _ = bench.phased_shape(n, nnz)
    slots = nnz + 7 * W * P
    for size in (4 * W * (P + 1), 4 * (W + 1), 4 * n, 8 * n, 2 * slots, 4 * slots, vb * slots):
        off = up(off + size)
    return off


@pytest.mark.parametrize("n,nnz,vt", [(5, 8, 0), (100_000, 1_957_254, 0), (600_000, 7_000_000, 1),
                                      (1_000_000, 9_991_220, 0), (4_000_000, 119_311_046, 1),
                                      (4_194_304, 16_777_216, 0), (4_300_000, 8_600_000, 2)])
def test_plan_bytes_follow_the_phased_shape(lib, n, nnz, vt):
    """The plan size fj_plan_bytes reports matches the layout written out with
    bench.py's phased_shape (short or long chunks, phases, reserved slots), so
    the bench's layout byte counts describe the layout the library builds."""
    vtype = (fj.FJ_VAL_UNIT, fj.FJ_VAL_F32, fj.FJ_VAL_F64)[vt]
    csr = fj.fj_csr(n=n, nnz=nnz, row_ptr=256, col_idx=512, val=None if vt == 0 else 1024, val_type=vtype)
    assert lib.fj_plan_bytes(ctypes.byref(csr)) == _plan_bytes_model(n, nnz, (0, 4, 8)[vt])
