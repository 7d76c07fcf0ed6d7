"""Seeded synthetic inputs: graphs in symmetric CSR form and opinion vectors.

This module builds inputs only. It holds none of the method's arithmetic (no
Laplacian, no solve, no index) so that the CPU oracle and the GPU path can both
be fed from it without sharing any computation.

Graphs follow the paper's setting (Section 2.1): undirected, weighted, simple
(no self-loops, no multi-edges), stored with both directions of every edge,
column indices strictly increasing inside each row, int32 indices.

Opinion vectors follow the experimental section (internal opinion
distributions): uniform on [0,1], exponential and power law, each normalised to
[0,1]. The configured workloads use min-max scaling; the paper's own
divide-by-maximum variants are kept as options.

All randomness is numpy ``default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np

__all__ = [
    "CSRGraph",
    "csr_from_edges",
    "barabasi_albert",
    "chung_lu",
    "opinions",
    "opinion_block",
    "path_graph",
    "cycle_graph",
    "torus_graph",
    "complete_graph",
    "random_graph",
    "workload",
    "WORKLOADS",
]


@dataclasses.dataclass
class CSRGraph:
    """Symmetric CSR: row_ptr int32[n+1], col int32[nnz], val None|f32|f64[nnz].

    ``val is None`` means every edge has unit weight.
    """

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: Optional[np.ndarray] = None
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def m(self) -> int:
        """Number of undirected edges."""
        return self.nnz // 2

    def weights_f64(self) -> np.ndarray:
        if self.val is None:
            return np.ones(self.nnz, dtype=np.float64)
        return self.val.astype(np.float64)

    def edges(self):
        """Undirected edge list (i < j) with weights, in CSR order."""
        rows = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))
        cols = self.col.astype(np.int64)
        keep = rows < cols
        w = self.weights_f64()[keep]
        return rows[keep], cols[keep], w

    def validate(self) -> None:
        """Check the structural contract; raise ValueError on violation."""
        rp, c = self.row_ptr, self.col
        if rp.dtype != np.int32 or c.dtype != np.int32:
            raise ValueError("row_ptr and col must be int32")
        if rp.shape != (self.n + 1,) or rp[0] != 0 or np.any(np.diff(rp.astype(np.int64)) < 0):
            raise ValueError("row_ptr must be non-decreasing from 0 with n+1 entries")
        if c.shape != (self.nnz,):
            raise ValueError("col length must equal row_ptr[n]")
        if self.nnz and (c.min() < 0 or c.max() >= self.n):
            raise ValueError("column index out of range")
        rows = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(rp))
        if np.any(rows == c):
            raise ValueError("self-loop present")
        key = rows * self.n + c
        if np.any(np.diff(key) <= 0):
            raise ValueError("columns must be strictly increasing inside each row")
        tkey = c.astype(np.int64) * self.n + rows
        order = np.argsort(tkey, kind="stable")
        if not np.array_equal(tkey[order], key):
            raise ValueError("graph is not symmetric")
        if self.val is not None:
            v = self.val
            if v.shape != (self.nnz,) or v.dtype not in (np.float32, np.float64):
                raise ValueError("val must be f32 or f64 with nnz entries")
            if not np.all(np.isfinite(v)) or np.any(v <= 0):
                raise ValueError("weights must be finite and positive")
            if not np.array_equal(v[order], v):
                raise ValueError("weights are not symmetric")


def _csr_from_unique_pairs(n: int, u: np.ndarray, v: np.ndarray,
                           w: Optional[np.ndarray], name: str) -> CSRGraph:
    """Build symmetric CSR from unique undirected pairs sorted by (u, v), u < v."""
    m = u.shape[0]
    u = u.astype(np.int64, copy=False)
    v = v.astype(np.int64, copy=False)
    cnt_lo = np.bincount(u, minlength=n)   # entries (u -> v) with v > u
    cnt_hi = np.bincount(v, minlength=n)   # entries (v -> u) with u < v
    deg = cnt_lo + cnt_hi
    row_ptr64 = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=row_ptr64[1:])
    nnz = int(row_ptr64[-1])
    if nnz >= 2**31:
        raise ValueError("nnz does not fit int32 row pointers")
    col = np.empty(nnz, dtype=np.int32)
    val = None if w is None else np.empty(nnz, dtype=w.dtype)
    ar = np.arange(m, dtype=np.int64)
    # Entries whose column is smaller than the row: row v, column u, sorted by (v, u).
    order = np.argsort(v, kind="stable")  # pairs are sorted by u, so u stays sorted per v
    vs = v[order]
    first_hi = np.cumsum(cnt_hi) - cnt_hi
    pos = row_ptr64[vs] + (ar - first_hi[vs])
    col[pos] = u[order]
    if val is not None:
        val[pos] = w[order]
    del order, vs, pos
    # Entries whose column is larger than the row: row u, column v, already sorted.
    first_lo = np.cumsum(cnt_lo) - cnt_lo
    pos = row_ptr64[u] + cnt_hi[u] + (ar - first_lo[u])
    col[pos] = v
    if val is not None:
        val[pos] = w
    return CSRGraph(n=n, row_ptr=row_ptr64.astype(np.int32), col=col, val=val, name=name)


def csr_from_edges(n: int, edges: Sequence, weights=None, name: str = "",
                   val_dtype=np.float64) -> CSRGraph:
    """Symmetric CSR from an undirected edge list. Rejects self-loops and repeats."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if e.size and (e.min() < 0 or e.max() >= n):
        raise ValueError("edge endpoint out of range")
    if np.any(e[:, 0] == e[:, 1]):
        raise ValueError("self-loop in edge list")
    lo = np.minimum(e[:, 0], e[:, 1])
    hi = np.maximum(e[:, 0], e[:, 1])
    key = lo * n + hi
    order = np.argsort(key, kind="stable")
    if np.any(np.diff(key[order]) == 0):
        raise ValueError("repeated edge in edge list")
    w = None
    if weights is not None:
        w = np.asarray(weights, dtype=val_dtype).reshape(-1)[order]
    return _csr_from_unique_pairs(n, lo[order], hi[order], w, name)


# ---------------------------------------------------------------- graph families


def path_graph(n: int, w=None) -> CSRGraph:
    edges = [(i, i + 1) for i in range(n - 1)]
    weights = None if w is None else [w] * len(edges)
    return csr_from_edges(n, edges, weights, name=f"path{n}")


def cycle_graph(n: int, w=None, val_dtype=np.float64) -> CSRGraph:
    """Cycle C_n (n >= 3), every edge of weight ``w`` (None = unit)."""
    i = np.arange(n, dtype=np.int64)
    edges = np.stack([i, (i + 1) % n], axis=1)
    weights = None if w is None else np.full(n, w)
    return csr_from_edges(n, edges, weights, name=f"cycle{n}", val_dtype=val_dtype)


def torus_graph(a: int, b: int, w=None) -> CSRGraph:
    """2-D torus C_a x C_b (a, b >= 3); node (x, y) has index x*b + y."""
    x, y = np.meshgrid(np.arange(a), np.arange(b), indexing="ij")
    idx = (x * b + y).ravel()
    right = (x * b + (y + 1) % b).ravel()
    down = (((x + 1) % a) * b + y).ravel()
    edges = np.concatenate([np.stack([idx, right], 1), np.stack([idx, down], 1)])
    weights = None if w is None else np.full(edges.shape[0], w)
    return csr_from_edges(a * b, edges, weights, name=f"torus{a}x{b}")


def complete_graph(n: int, w=None) -> CSRGraph:
    edges = [(i, j) for i in range(n) for j in range(i + 1, n)]
    weights = None if w is None else [w] * len(edges)
    return csr_from_edges(n, edges, weights, name=f"K{n}")


def random_graph(n: int, p: float, seed: int, weighted: bool = False,
                 wlo: float = 0.5, whi: float = 2.0, val_dtype=np.float64) -> CSRGraph:
    """Erdos-Renyi G(n, p); optional Uniform[wlo, whi] weights."""
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.shape[0]) < p
    edges = np.stack([iu[keep], ju[keep]], 1)
    weights = rng.uniform(wlo, whi, edges.shape[0]) if weighted else None
    return csr_from_edges(n, edges, weights, name=f"gnp{n}", val_dtype=val_dtype)


def barabasi_albert(n: int, m: int, seed: int) -> CSRGraph:
    """Preferential attachment: start from K_{m+1}; each new node links to m
    distinct existing nodes chosen with probability proportional to degree."""
    if n <= m:
        raise ValueError("n must exceed m")
    rng = np.random.default_rng(seed)
    m0 = m + 1
    edges = [(i, j) for i in range(m0) for j in range(i + 1, m0)]
    pool = np.empty(2 * (len(edges) + m * (n - m0)), dtype=np.int64)
    top = 0
    for a, b in edges:
        pool[top] = a
        pool[top + 1] = b
        top += 2
    for t in range(m0, n):
        chosen = set()
        while len(chosen) < m:
            chosen.add(int(pool[rng.integers(0, top)]))
        for c in sorted(chosen):
            edges.append((c, t))
            pool[top] = c
            pool[top + 1] = t
            top += 2
    return csr_from_edges(n, edges, name=f"ba{n}m{m}")


def chung_lu_weights(n: int, gamma: float, mean_deg: float) -> np.ndarray:
    """Expected degrees w_i proportional to (i+1)^(-1/(gamma-1)), capped at
    sqrt(n * mean_deg) and rescaled to mean ``mean_deg`` (cap and rescale are
    repeated until both hold)."""
    w = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (gamma - 1.0))
    cap = np.sqrt(n * mean_deg)
    for _ in range(100):
        w *= mean_deg / w.mean()
        if w.max() <= cap * (1 + 1e-12):
            break
        np.minimum(w, cap, out=w)
    return w


def edge_weight_hash(lo: np.ndarray, hi: np.ndarray, n: int, seed: int,
                     wlo: float, whi: float) -> np.ndarray:
    """float32 weight in [wlo, whi) for each undirected edge (lo, hi), drawn by a
    counter-based generator (SplitMix64 of the edge key mixed with the seed), so
    that both stored directions of an edge get the same value without any
    bookkeeping."""
    with np.errstate(over="ignore"):
        x = (lo.astype(np.uint64) * np.uint64(n) + hi.astype(np.uint64)) ^ np.uint64(
            (seed * 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF)
        x = x + np.uint64(0x9E3779B97F4A7C15)
        x = (x ^ (x >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        x = (x ^ (x >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        x = x ^ (x >> np.uint64(31))
    u = (x >> np.uint64(40)).astype(np.float64) * (1.0 / (1 << 24))
    return (wlo + (whi - wlo) * u).astype(np.float32)


def chung_lu(n: int, gamma: float, mean_deg: float, seed: int, weighted: bool = False,
             wlo: float = 0.5, whi: float = 2.0, name: str = "") -> CSRGraph:
    """Chung-Lu graph: n*mean_deg/2 endpoint pairs drawn i.i.d. proportional to
    the expected degrees; self-loops dropped, repeated pairs merged. All n nodes
    are kept, including isolated ones. Weighted graphs get one float32 weight
    per distinct edge, uniform on [wlo, whi) (see ``edge_weight_hash``).

    The i.i.d. draws are realised as a multinomial count per node followed by a
    uniformly random arrangement of the resulting multiset of endpoints, which
    has the same distribution and is much faster than per-draw inversion."""
    rng = np.random.default_rng(seed)
    w = chung_lu_weights(n, gamma, mean_deg)
    n_pairs = int(round(n * mean_deg / 2))
    counts = rng.multinomial(2 * n_pairs, w / w.sum())
    ends = np.repeat(np.arange(n, dtype=np.int32), counts)
    del counts
    rng.shuffle(ends)
    a = ends[0::2].astype(np.int64)
    b = ends[1::2].astype(np.int64)
    del ends
    keep = a != b
    lo = np.minimum(a[keep], b[keep])
    hi = np.maximum(a[keep], b[keep])
    del a, b, keep
    keys = np.unique(lo * n + hi)
    del lo, hi
    lo = keys // n
    hi = keys - lo * n
    directed = np.concatenate([keys, hi * n + lo])
    del keys
    directed.sort()
    rows = directed // n
    col = (directed - rows * n).astype(np.int32)
    del directed
    row_ptr = np.searchsorted(rows, np.arange(n + 1, dtype=np.int64), side="left")
    val = None
    if weighted:
        c64 = col.astype(np.int64)
        val = edge_weight_hash(np.minimum(rows, c64), np.maximum(rows, c64), n, seed, wlo, whi)
        del c64
    del rows
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32 row pointers")
    return CSRGraph(n=n, row_ptr=row_ptr.astype(np.int32), col=col, val=val,
                    name=name or f"chunglu{n}g{gamma}d{mean_deg}")


# ---------------------------------------------------------------- opinions


def _minmax(x: np.ndarray) -> np.ndarray:
    lo, hi = x.min(), x.max()
    if hi == lo:
        return np.zeros_like(x)
    return (x - lo) / (hi - lo)


def opinions(kind: str, n: int, seed: int) -> np.ndarray:
    """Internal opinions in [0,1], float64.

    kind: 'uniform'        Uniform[0,1]
          'exp'            Exponential(1), min-max scaled
          'pareto'         Pareto(alpha=2, x_min=1), min-max scaled
          'exp_paper'      x_min + Exponential(1) (density e^{x_min} e^{-x}), x_min=1, divided by max
          'powerlaw_paper' density (a-1) x_min^(a-1) x^-a with a=2.5, x_min=1, divided by max
          'constant'       all entries 0.5
    """
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.random(n)
    if kind == "exp":
        return _minmax(rng.exponential(1.0, n))
    if kind == "pareto":
        return _minmax((1.0 - rng.random(n)) ** (-1.0 / 2.0))
    if kind == "exp_paper":
        x = 1.0 + rng.exponential(1.0, n)
        return x / x.max()
    if kind == "powerlaw_paper":
        x = (1.0 - rng.random(n)) ** (-1.0 / 1.5)
        return x / x.max()
    if kind == "constant":
        return np.full(n, 0.5)
    raise ValueError(f"unknown opinion kind {kind!r}")


def opinion_block(n: int, kinds: Sequence[str], seed: int) -> np.ndarray:
    """Node-major n x k block whose column c is ``opinions(kinds[c], n, seed + c)``."""
    cols = [opinions(kd, n, seed + c) for c, kd in enumerate(kinds)]
    return np.ascontiguousarray(np.stack(cols, axis=1))


def log_uniform_weights(g: CSRGraph, span: float, seed: int) -> CSRGraph:
    """The same graph with FP64 weights log-uniform over a factor `span`
    (geometric mean 1, so in [span^-1/2, span^1/2]), equal in both stored
    directions of an edge: u = a 53-bit hash of the edge key, w = span^(u - 1/2)."""
    import dataclasses
    rows = np.repeat(np.arange(g.n, dtype=np.uint64), np.diff(g.row_ptr))
    lo = np.minimum(rows, g.col.astype(np.uint64))
    hi = np.maximum(rows, g.col.astype(np.uint64))
    with np.errstate(over="ignore"):
        h = (lo * np.uint64(g.n) + hi + np.uint64(seed)) * np.uint64(0x9E3779B97F4A7C15)
    u = (h >> np.uint64(11)).astype(np.float64) / 2.0 ** 53
    w = np.exp(np.log(1.0 / np.sqrt(span)) + u * np.log(span))
    return dataclasses.replace(g, val=w.astype(np.float64))


# ---------------------------------------------------------------- named workloads

WORKLOADS = {
    # name: (graph builder, opinion recipe)
    "ba10k": dict(graph=lambda: barabasi_albert(10_000, 3, 1001), s=("uniform", 2001),
                  rtol=1e-10, desc="Barabasi-Albert n=10,000, m=3, unit weights; s~U[0,1]"),
    "cl1m": dict(graph=lambda: chung_lu(1_000_000, 2.5, 10.0, 1002, name="cl1m"), s=("uniform", 2002),
                 rtol=0.0, desc="Chung-Lu n=1,000,000, gamma=2.5, mean degree 10, unit weights; s~U[0,1]"),
    "cl4m": dict(graph=lambda: chung_lu(4_000_000, 2.2, 30.0, 1003, weighted=True, name="cl4m"),
                 s=("exp", 2003), rtol=0.0,
                 desc="Chung-Lu n=4,000,000, gamma=2.2, mean degree 30, weights float32(U[0.5,2]); "
                      "s~Exp(1) min-max scaled"),
    "wide100k": dict(graph=lambda: log_uniform_weights(chung_lu(100_000, 2.5, 10.0, 31), 1e6, 7),
                     s=("uniform", 32), rtol=0.0,
                     desc="Chung-Lu n=100,000, gamma=2.5, mean degree 10, FP64 weights log-uniform over a "
                          "factor 1e6; s~U[0,1]"),
}

def serving_graph_params(count: int = 32, seed0: int = 1100):
    """Graph g of the serving mix: Chung-Lu with n log-uniform in [1e4, 2e6],
    exponent gamma ~ U[2.1, 2.8] and mean degree ~ U[5, 40], drawn from seed
    seed0 + g; unit weights."""
    out = []
    for gi in range(count):
        rng = np.random.default_rng(seed0 + gi)
        n = int(round(np.exp(rng.uniform(np.log(1e4), np.log(2e6)))))
        out.append(dict(n=n, gamma=float(rng.uniform(2.1, 2.8)), mean_deg=float(rng.uniform(5.0, 40.0)),
                        seed=seed0 + gi))
    return out


def serving_graph(params) -> CSRGraph:
    return chung_lu(params["n"], params["gamma"], params["mean_deg"], params["seed"],
                    name=f"serve{params['seed']}")


def serving_requests(count: int, n_graphs: int, seed: int = 3000, kmax: int = 16):
    """(graph, k, first column) per request: graph uniform, k ~ UniformInt[1, kmax],
    columns taken from a per-graph pool of 64 U[0,1] vectors starting at a
    uniform offset."""
    rng = np.random.default_rng(seed)
    g = rng.integers(0, n_graphs, count)
    k = rng.integers(1, kmax + 1, count)
    c0 = rng.integers(0, 64 - k + 1)
    return [(int(a), int(b), int(c)) for a, b, c in zip(g, k, c0)]


_cache: dict = {}


def workload(name: str):
    """Return (graph, s, desc) for a named workload; graphs are cached per process."""
    spec = WORKLOADS[name]
    if name not in _cache:
        _cache[name] = spec["graph"]()
    g = _cache[name]
    kind, seed = spec["s"]
    return g, opinions(kind, g.n, seed), spec
