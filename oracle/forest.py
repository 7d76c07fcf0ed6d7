"""Brute-force spanning rooted forests (test infrastructure only).

Section 2.2: the weight of a subgraph is the product of its edge weights (1 with
no edges); Gamma is the set of spanning rooted forests; Gamma_ij those in which
i and j share a tree rooted at i; and omega_ij = eps(Gamma_ij) / eps(Gamma).

Enumeration: every edge subset that is acyclic is a spanning forest; rooting it
means choosing one root per tree, so an unrooted forest F contributes
eps(F) * prod_T |T| to eps(Gamma), and to eps(Gamma_ij) it contributes
eps(F) * prod_{T not containing i} |T| when i and j share a tree (the tree of i
must be rooted at i). Exact rational arithmetic (fractions.Fraction).
Feasible up to about 16 edges.
"""
from __future__ import annotations

from fractions import Fraction
from itertools import combinations


def _components(n, chosen_edges):
    """Union-find over the chosen edges; returns (labels, acyclic?)."""
    parent = list(range(n))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for (a, b) in chosen_edges:
        ra, rb = find(a), find(b)
        if ra == rb:
            return None, False
        parent[ra] = rb
    return [find(a) for a in range(n)], True


def forest_weights(n, edges, weights=None):
    """Return (eps(Gamma), E) where E[i][j] = eps(Gamma_ij), all exact Fractions.

    edges: list of undirected (i, j); weights: matching list (default all 1).
    """
    m = len(edges)
    if weights is None:
        weights = [1] * m
    weights = [Fraction(w) for w in weights]
    total = Fraction(0)
    E = [[Fraction(0)] * n for _ in range(n)]
    for k in range(m + 1):
        for subset in combinations(range(m), k):
            labels, ok = _components(n, [edges[e] for e in subset])
            if not ok:
                continue
            wF = Fraction(1)
            for e in subset:
                wF *= weights[e]
            size = {}
            for lab in labels:
                size[lab] = size.get(lab, 0) + 1
            prod_all = 1
            for sz in size.values():
                prod_all *= sz
            total += wF * prod_all
            for i in range(n):
                others = prod_all // size[labels[i]]
                for j in range(n):
                    if labels[j] == labels[i]:
                        E[i][j] += wF * others
    return total, E


def forest_matrix_exact(n, edges, weights=None):
    """Omega with omega_ij = eps(Gamma_ij)/eps(Gamma), as Fractions."""
    total, E = forest_weights(n, edges, weights)
    return [[E[i][j] / total for j in range(n)] for i in range(n)], total
