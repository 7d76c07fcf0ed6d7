"""Dense FP64 oracle (test infrastructure only; see the package docstring).

Every quantity is written as the paper defines it, with a library LAPACK solve
or inverse as the only non-trivial step. Intended for n up to about 10^4.
"""
from __future__ import annotations

import math

import numpy as np

INDEX_NAMES = ("internal_conflict", "disagreement", "polarization", "controversy", "dc_index")


def adjacency_dense(g) -> np.ndarray:
    """Section 2.1: A = (w_ij), w_ij = w_ji = w_e for an edge e = (i, j), else 0."""
    A = np.zeros((g.n, g.n), dtype=np.float64)
    w = g.weights_f64()
    for i in range(g.n):
        for k in range(int(g.row_ptr[i]), int(g.row_ptr[i + 1])):
            A[i, int(g.col[k])] += w[k]
    return A


def laplacian_dense(g) -> np.ndarray:
    """Section 2.1: d_i = sum_j w_ij, D = diag(d), L = D - A."""
    A = adjacency_dense(g)
    return np.diag(A.sum(axis=1)) - A


def incidence_dense(g):
    """Section 2.1: signed incidence B (row b_e = e_i - e_j for edge e=(i,j), i<j)
    and W = diag(w_e); L = B^T W B."""
    lo, hi, w = g.edges()
    m = lo.shape[0]
    B = np.zeros((m, g.n), dtype=np.float64)
    B[np.arange(m), lo] = 1.0
    B[np.arange(m), hi] = -1.0
    return B, np.diag(w)


def forest_matrix(g) -> np.ndarray:
    """Section 2.2: Omega = (I + L)^{-1}."""
    return np.linalg.inv(np.eye(g.n) + laplacian_dense(g))


def equilibrium(g, s) -> np.ndarray:
    """Eq. FJmodel02: z = (I + L)^{-1} s, by an LU solve of (I + L) z = s."""
    return np.linalg.solve(np.eye(g.n) + laplacian_dense(g), np.asarray(s, dtype=np.float64))


def indices_by_definition(g, s, z) -> dict:
    """Section 3.2 definitions evaluated at a given equilibrium z, with exactly
    rounded sums (math.fsum):
      internal conflict  C_I  = sum_i (z_i - s_i)^2
      disagreement       D    = sum over undirected edges (i,j) of w_ij (z_i - z_j)^2
      polarization       P    = sum_i (z_i - mean(z))^2
      controversy        C    = sum_i z_i^2
      dc index           I_dc = D + C, reported through its equal form s^T z
    """
    s = np.asarray(s, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    lo, hi, w = g.edges()
    ci = math.fsum(((z - s) ** 2).tolist())
    d = math.fsum((w * (z[lo] - z[hi]) ** 2).tolist())
    mean_z = math.fsum(z.tolist()) / g.n
    p = math.fsum(((z - mean_z) ** 2).tolist())
    c = math.fsum((z * z).tolist())
    idc = math.fsum((s * z).tolist())
    return dict(internal_conflict=ci, disagreement=d, polarization=p, controversy=c,
                dc_index=idc, dc_sum=d + c, stress=ci + d, polarization_index=c / g.n)


def indices(g, s) -> dict:
    """Exact indices: dense solve of Eq. FJmodel02, then the definitions."""
    return indices_by_definition(g, s, equilibrium(g, s))


def indices_quadratic_forms(g, s) -> dict:
    """Proposition 1: each index as a quadratic form in s through Omega."""
    s = np.asarray(s, dtype=np.float64)
    L = laplacian_dense(g)
    Om = forest_matrix(g)
    sbar = s - s.mean()
    return dict(
        internal_conflict=float(s @ Om @ L @ L @ Om @ s),
        disagreement=float(s @ Om @ L @ Om @ s),
        polarization=float(sbar @ Om @ Om @ sbar),
        controversy=float(s @ Om @ Om @ s),
        dc_index=float(s @ Om @ s),
    )


def indices_l2_norms(g, s) -> dict:
    """Lemma 4.1: the indices as squared l2 norms of vectors built from
    (I+L)^{-1}s and (I+L)^{-1}sbar, with the incidence form for D."""
    s = np.asarray(s, dtype=np.float64)
    L = laplacian_dense(g)
    B, W = incidence_dense(g)
    IpL = np.eye(g.n) + L
    z = np.linalg.solve(IpL, s)
    q = np.linalg.solve(IpL, s - s.mean())
    Whalf = np.sqrt(W)
    dz = Whalf @ B @ z
    return dict(
        internal_conflict=float(np.dot(L @ z, L @ z)),
        disagreement=float(np.dot(dz, dz)),
        polarization=float(np.dot(q, q)),
        controversy=float(np.dot(z, z)),
        dc_index=float(np.dot(dz, dz) + np.dot(z, z)),
    )
