"""ctypes front end of fj_oracle.c (test infrastructure only).

build() compiles fj_oracle.c with gcc (-O2 -fopenmp, strict IEEE: no
-ffast-math, so the compensated sums stay compensated).
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fj_oracle.c")
_LIB = os.path.join(_HERE, "libfj_oracle.so")
_lib = None

INDEX_NAMES = ("internal_conflict", "disagreement", "polarization", "controversy", "dc_index")


def build(src: str = _SRC, out: str = _LIB) -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
           "-o", out + ".tmp", src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def _load(path):
    L = ctypes.CDLL(path)
    i32, i64, dp, ip = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p
    L.fjo_threads.restype = ctypes.c_int
    L.fjo_apply.argtypes = [i32, ip, ip, dp, dp, dp]
    L.fjo_degrees.argtypes = [i32, ip, dp, dp]
    L.fjo_pcg.argtypes = [i32, ip, ip, dp, dp, dp, ctypes.c_double, i32,
                          ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
    L.fjo_pcg.restype = ctypes.c_int
    L.fjo_indices.argtypes = [i32, ip, ip, dp, dp, dp, dp]
    L.fjo_fj_iterate.argtypes = [i32, ip, ip, dp, dp, dp, i32, ctypes.c_double,
                                 ctypes.POINTER(i32)]
    L.fjo_fj_iterate.restype = ctypes.c_int
    return L


@contextlib.contextmanager
def swapped(path):
    """Use the oracle library at ``path`` inside the block (for mutation tests,
    which plant mistakes in a copy of fj_oracle.c and check that pins fail)."""
    global _lib
    saved = _lib
    _lib = _load(path)
    try:
        yield
    finally:
        _lib = saved


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = _load(_LIB)
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _arrays(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    w = None if g.val is None else np.ascontiguousarray(g.val, dtype=np.float64)
    return rp, col, w


def threads() -> int:
    return lib().fjo_threads()


def apply(g, x):
    """(I + L) x."""
    rp, col, w = _arrays(g)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(g.n)
    lib().fjo_apply(g.n, _ptr(rp), _ptr(col), _ptr(w), _ptr(x), _ptr(y))
    return y


def degrees(g):
    rp, col, w = _arrays(g)
    d = np.empty(g.n)
    lib().fjo_degrees(g.n, _ptr(rp), _ptr(w), _ptr(d))
    return d


def solve(g, s, rtol=1e-13, max_iter=20000):
    """z with ||s - (I+L)z|| <= rtol ||s||. Returns (z, info dict)."""
    rp, col, w = _arrays(g)
    s = np.ascontiguousarray(s, dtype=np.float64)
    z = np.empty(g.n)
    it = ctypes.c_int32(0)
    rel = ctypes.c_double(0.0)
    t0 = time.perf_counter()
    st = lib().fjo_pcg(g.n, _ptr(rp), _ptr(col), _ptr(w), _ptr(s), _ptr(z), rtol, max_iter,
                       ctypes.byref(it), ctypes.byref(rel))
    return z, dict(status=st, iters=it.value, relres=rel.value, seconds=time.perf_counter() - t0)


def indices_at(g, s, z) -> dict:
    """Section 3.2 definitions at z, plus diagnostics (see fj_oracle.c)."""
    rp, col, w = _arrays(g)
    s = np.ascontiguousarray(s, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    out = np.empty(10)
    lib().fjo_indices(g.n, _ptr(rp), _ptr(col), _ptr(w), _ptr(s), _ptr(z), _ptr(out))
    keys = INDEX_NAMES + ("residual_norm", "lz_norm2", "zlz", "sum_z", "sum_s")
    return dict(zip(keys, out.tolist()))


def error_bounds(vals: dict) -> dict:
    """Relative error bound of each index at a z with residual r = s - (I+L)z.

    With e = z_true - z = (I+L)^{-1} r and I <= I+L (Section 4), each of
    ||e||, ||L e|| (eigenvalues lambda/(1+lambda) < 1), ||W^{1/2} B e|| and
    ||e - mean(e)|| is at most rho = ||r||; so |sqrt(X) - sqrt(X~)| <= rho for
    the four squared-norm indices, and |s^T e| = |z_true^T r| <= (||z|| + rho) rho.
    """
    rho = vals["residual_norm"]
    out = {}
    for k in ("internal_conflict", "disagreement", "polarization", "controversy"):
        rx = np.sqrt(max(vals[k], 0.0))
        out[k] = rho * (2 * rx + rho) / (rx - rho) ** 2 if rx > rho else np.inf
    a = (np.sqrt(vals["controversy"]) + rho) * rho
    idc = vals["dc_index"]
    out["dc_index"] = a / (idc - a) if idc > a else np.inf
    return out


def indices(g, s, rtol=1e-13, max_iter=20000, certify=1e-9):
    """Oracle indices: PCG to rtol, definitions at z, and a check that every
    index's relative error bound is <= ``certify``. Returns (values, z, info)."""
    z, info = solve(g, s, rtol=rtol, max_iter=max_iter)
    vals = indices_at(g, s, z)
    bounds = error_bounds(vals)
    info["bounds"] = bounds
    info["certified"] = all(b <= certify for b in bounds.values())
    return vals, z, info


def fj_iterate(g, s, max_sweeps=100000, tol=1e-14):
    """Eq. FJmodel applied synchronously from z = s until it stops changing."""
    rp, col, w = _arrays(g)
    s = np.ascontiguousarray(s, dtype=np.float64)
    z = np.empty(g.n)
    sw = ctypes.c_int32(0)
    st = lib().fjo_fj_iterate(g.n, _ptr(rp), _ptr(col), _ptr(w), _ptr(s), _ptr(z), max_sweeps,
                              tol, ctypes.byref(sw))
    return z, dict(status=st, sweeps=sw.value)
