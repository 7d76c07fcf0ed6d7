"""Pins for the CPU oracle: checks against values and properties that the paper
or mathematics fix, never against the oracle's own formulas.

Each pin takes the oracle modules it checks as arguments, so that the mutation
tests can run the same pins against deliberately broken copies of the oracle.
A pin raises AssertionError on failure.
"""
from __future__ import annotations

import math
import os
from fractions import Fraction

import numpy as np

from paper_2101_08143_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "p5_forest_matrix.txt")
NAMES = ("internal_conflict", "disagreement", "polarization", "controversy", "dc_index")


def load_p5_golden():
    """The Section 2.2 worked example (path P5): 55 forests, 13 in Gamma_12, 55*Omega."""
    total = in12 = None
    rows = []
    with open(GOLDEN) as f:
        lines = [ln.strip() for ln in f if ln.strip() and not ln.startswith("#")]
    for ln in lines:
        parts = ln.split()
        if parts[0] == "total_rooted_forests":
            total = int(parts[1])
        elif parts[0] == "forests_v2_in_tree_rooted_at_v1":
            in12 = int(parts[1])
        elif parts[0] == "matrix_times_55":
            continue
        else:
            rows.append([int(x) for x in parts])
    return total, in12, np.array(rows, dtype=np.int64)


def _close(a, b, rtol, atol=0.0, what=""):
    if not abs(a - b) <= atol + rtol * abs(b):
        raise AssertionError(f"{what}: {a!r} vs {b!r} (rtol {rtol}, atol {atol})")


def _close_dict(got, want, rtol, atol=0.0, what=""):
    for k in NAMES:
        _close(got[k], want[k], rtol, atol, f"{what} {k}")


# ------------------------------------------------------------------ dense pins


def pin_p5_forest_matrix(dense):
    total, in12, M = load_p5_golden()
    g = W.path_graph(5)
    Om = dense.forest_matrix(g)
    if not np.allclose(Om * total, M, rtol=0, atol=1e-10):
        raise AssertionError(f"P5 forest matrix differs from the printed example:\n{Om * total}")
    z = dense.equilibrium(g, np.eye(5)[:, 1])
    if not np.allclose(z * total, M[:, 1], rtol=0, atol=1e-10):
        raise AssertionError("P5 equilibrium for s = e_2 is not column 2 of the printed Omega")


def pin_p5_forest_enumeration(forest):
    total, in12, M = load_p5_golden()
    t, E = forest.forest_weights(5, [(0, 1), (1, 2), (2, 3), (3, 4)])
    if t != total or E[0][1] != in12:
        raise AssertionError(f"P5 enumeration gave {t} forests and {E[0][1]} in Gamma_12")
    if [[int(x) for x in row] for row in E] != M.tolist():
        raise AssertionError("P5 enumeration matrix differs from the printed example")


def _tiny_graphs():
    rng = np.random.default_rng(77)
    out = []
    for n, p in ((4, 0.8), (5, 0.6), (6, 0.45), (6, 0.5), (7, 0.3)):
        while True:
            iu, ju = np.triu_indices(n, 1)
            keep = rng.random(iu.shape[0]) < p
            if 1 <= keep.sum() <= 12:
                break
        edges = list(zip(iu[keep].tolist(), ju[keep].tolist()))
        weights = rng.integers(1, 4, len(edges)).tolist()
        out.append((n, edges, weights))
    return out


def pin_forest_bruteforce(dense, forest):
    """omega_ij = eps(Gamma_ij)/eps(Gamma) (Section 2.2) against the dense inverse,
    and det(I+L) = eps(Gamma) (the forest form of the matrix-tree theorem)."""
    for n, edges, weights in _tiny_graphs():
        g = W.csr_from_edges(n, edges, weights)
        Om_exact, total = forest.forest_matrix_exact(n, edges, weights)
        Om = dense.forest_matrix(g)
        want = np.array([[float(x) for x in row] for row in Om_exact])
        if not np.allclose(Om, want, rtol=1e-12, atol=1e-14):
            raise AssertionError(f"forest matrix mismatch on n={n} edges={edges}")
        det = np.linalg.det(np.eye(n) + dense.laplacian_dense(g))
        _close(det, float(total), 1e-10, what="det(I+L) vs forest weight")
        s = np.linspace(0.1, 0.9, n)
        z_exact = [float(sum(Om_exact[i][j] * Fraction(float(s[j])) for j in range(n)))
                   for i in range(n)]
        if not np.allclose(dense.equilibrium(g, s), z_exact, rtol=1e-12, atol=1e-14):
            raise AssertionError("equilibrium is not the forest-weighted average of s")


def pin_prop1_and_lemma41(dense):
    """Definitions, Proposition 1 quadratic forms and Lemma 4.1 norms agree."""
    for g in (W.random_graph(30, 0.2, 5, weighted=True), W.barabasi_albert(40, 2, 3)):
        s = W.opinions("uniform", g.n, 9)
        a = dense.indices(g, s)
        b = dense.indices_quadratic_forms(g, s)
        c = dense.indices_l2_norms(g, s)
        _close_dict(b, a, 1e-10, what="Prop. 1")
        _close_dict(c, a, 1e-10, what="Lemma 4.1")


# ------------------------------------------------------- pins on any solver


def pin_closed_forms(indices_fn):
    """Graphs whose equilibrium has a closed form."""
    rng = np.random.default_rng(3)
    # Edgeless graph: z = s.
    n = 7
    s = rng.random(n)
    g = W.csr_from_edges(n, np.zeros((0, 2), dtype=np.int64))
    got = indices_fn(g, s)
    sb = s - s.mean()
    want = dict(internal_conflict=0.0, disagreement=0.0, polarization=float(sb @ sb),
                controversy=float(s @ s), dc_index=float(s @ s))
    _close_dict(got, want, 1e-12, 1e-14, "edgeless")
    # Single edge of weight w.
    for w in (1.0, 0.3, 2.5):
        s = np.array([0.9, 0.2])
        g = W.csr_from_edges(2, [(0, 1)], [w])
        dlt = s[0] - s[1]
        k = 1.0 + 2.0 * w
        z1 = (s.sum() + dlt / k) / 2
        z2 = (s.sum() - dlt / k) / 2
        want = dict(internal_conflict=2 * w * w * dlt * dlt / k ** 2,
                    disagreement=w * dlt * dlt / k ** 2,
                    polarization=dlt * dlt / (2 * k ** 2),
                    controversy=z1 * z1 + z2 * z2,
                    dc_index=s[0] * z1 + s[1] * z2)
        _close_dict(indices_fn(g, s), want, 1e-12, 1e-15, f"single edge w={w}")
    # Complete graph K_n with weight w: z = mean(s) 1 + sbar / (1 + w n).
    for n, w in ((9, None), (12, 0.75)):
        ww = 1.0 if w is None else w
        g = W.complete_graph(n, w)
        s = rng.random(n)
        mu = s.mean()
        sb2 = float(((s - mu) ** 2).sum())
        k = 1.0 + ww * n
        want = dict(internal_conflict=(ww * n) ** 2 * sb2 / k ** 2,
                    disagreement=ww * n * sb2 / k ** 2,
                    polarization=sb2 / k ** 2,
                    controversy=n * mu * mu + sb2 / k ** 2,
                    dc_index=n * mu * mu + sb2 / k)
        _close_dict(indices_fn(g, s), want, 1e-11, 1e-15, f"K_{n}")
    # Constant opinions: z = s, so P = D = C_I = 0.
    g = W.barabasi_albert(300, 3, 8)
    s = np.full(g.n, 0.37)
    got = indices_fn(g, s)
    want = dict(internal_conflict=0.0, disagreement=0.0, polarization=0.0,
                controversy=g.n * 0.37 ** 2, dc_index=g.n * 0.37 ** 2)
    _close_dict(got, want, 1e-12, 1e-18, "constant s")


def pin_circulant(indices_fn, solve_fn, circulant, sizes=((997, 0.7), (1000, None)),
                  torus=((30, 41, 1.3),)):
    """Cycles and tori: spectral closed form (exact up to FFT rounding)."""
    rng = np.random.default_rng(11)
    for n, w in sizes:
        g = W.cycle_graph(n, w)
        ww = 1.0 if w is None else w
        s = rng.random(n)
        z = solve_fn(g, s)
        zf = circulant.cycle_equilibrium(s, ww)
        if not np.allclose(z, zf, rtol=0, atol=1e-11):
            raise AssertionError(f"cycle n={n} equilibrium max err {np.abs(z - zf).max()}")
        v = indices_fn(g, s)
        want = circulant.cycle_indices(s, ww)
        _close_dict(v, want, 1e-9, 0, f"cycle{n}")
        if "lz_norm2" in v:
            _close(v["lz_norm2"], want["internal_conflict"], 1e-9, what=f"cycle{n} ||Lz||^2")
            _close(v["zlz"], want["disagreement"], 1e-9, what=f"cycle{n} z^T L z")
    for a, b, w in torus:
        g = W.torus_graph(a, b, w)
        s = rng.random(a * b)
        z = solve_fn(g, s)
        zf = circulant.torus_equilibrium(s, a, b, w)
        if not np.allclose(z, zf, rtol=0, atol=1e-11):
            raise AssertionError(f"torus {a}x{b} equilibrium max err {np.abs(z - zf).max()}")
        v = indices_fn(g, s)
        want = circulant.torus_indices(s, a, b, w)
        _close_dict(v, want, 1e-9, 0, "torus")
        if "lz_norm2" in v:
            _close(v["lz_norm2"], want["internal_conflict"], 1e-9, what="torus ||Lz||^2")
            _close(v["zlz"], want["disagreement"], 1e-9, what="torus z^T L z")


def _permuted(g, perm):
    lo, hi, w = g.edges()
    edges = np.stack([perm[lo], perm[hi]], 1)
    return W.csr_from_edges(g.n, edges, None if g.val is None else w)


def pin_identities(indices_fn, solve_fn):
    """Conservation sum z = sum s (Section 3.1), ||s||^2 = C + 2D + C_I,
    s^T z = C + D (Section 3.2), P = C - n mean(s)^2, the range
    min s <= z_i <= max s, invariance under relabelling nodes, and invariance of
    P, D and C_I when a constant is added to s."""
    graphs = [W.barabasi_albert(500, 3, 21), W.random_graph(200, 0.05, 22, weighted=True),
              W.chung_lu(3000, 2.3, 8.0, 23, weighted=True)]
    for g in graphs:
        for kind in ("uniform", "exp", "pareto"):
            s = W.opinions(kind, g.n, 31)
            z = solve_fn(g, s)
            v = indices_fn(g, s)
            ss = float(s @ s)
            _close(float(z.sum()), float(s.sum()), 1e-12, 1e-12, "sum z = sum s")
            _close(v["controversy"] + 2 * v["disagreement"] + v["internal_conflict"], ss, 1e-11,
                   what="||s||^2 = C + 2D + C_I")
            _close(v["dc_index"], v["controversy"] + v["disagreement"], 1e-11, what="s^T z = C + D")
            _close(v["polarization"], v["controversy"] - g.n * s.mean() ** 2, 1e-8, 1e-12,
                   what="P = C - n mean(s)^2")
            if z.min() < s.min() - 1e-12 or z.max() > s.max() + 1e-12:
                raise AssertionError("z leaves [min s, max s]")
            if "lz_norm2" in v:  # Lemma 4.1 and Proposition 1 forms, where the oracle reports them
                _close(v["lz_norm2"], v["internal_conflict"], 1e-9, 1e-14 * ss, "||Lz||^2 = C_I")
                _close(v["zlz"], v["disagreement"], 1e-9, 1e-14 * ss, "z^T L z = D")
        perm = np.random.default_rng(5).permutation(g.n)
        gp = _permuted(g, perm)
        sp = np.empty_like(s)
        sp[perm] = s
        _close_dict(indices_fn(gp, sp), v, 1e-10, what="relabelled")
        shifted = indices_fn(g, s + 0.25)
        for k in ("polarization", "disagreement", "internal_conflict"):
            _close(shifted[k], v[k], 1e-8, 1e-12, f"shift invariance {k}")


def pin_fj_dynamics(fj_iterate_fn, solve_fn):
    """The FJ update rule (Eq. FJmodel) converges to the equilibrium of
    Eq. FJmodel02; on P5 with s = e_1 that is column 1 of the printed Omega."""
    total, in12, M = load_p5_golden()
    g = W.path_graph(5)
    z = fj_iterate_fn(g, np.eye(5)[:, 0])
    if not np.allclose(z * total, M[:, 0], rtol=0, atol=1e-9):
        raise AssertionError("FJ dynamics on P5 do not reach column 1 of the printed Omega")
    for g in (W.barabasi_albert(400, 2, 41), W.random_graph(150, 0.06, 42, weighted=True)):
        s = W.opinions("uniform", g.n, 43)
        if not np.allclose(fj_iterate_fn(g, s), solve_fn(g, s), rtol=0, atol=1e-10):
            raise AssertionError("FJ dynamics fixed point differs from the solve")


def pin_p5_sparse(solve_fn):
    total, in12, M = load_p5_golden()
    g = W.path_graph(5)
    for j in range(5):
        z = solve_fn(g, np.eye(5)[:, j])
        if not np.allclose(z * total, M[:, j], rtol=0, atol=1e-10):
            raise AssertionError(f"P5 solve for s = e_{j + 1} differs from the printed Omega")


# ------------------------------------------------ the oracle's certificate


def _closed_form_cases():
    """(name, graph, s, exact z, exact indices) for graphs whose equilibrium has
    a closed form: no solver is involved, so these are the truth."""
    rng = np.random.default_rng(17)
    cases = []
    for w in (0.001, 0.5, 2.5):  # single edge of weight w
        s = np.array([0.9, 0.2])
        dlt = s[0] - s[1]
        k = 1.0 + 2.0 * w
        z = np.array([(s.sum() + dlt / k) / 2, (s.sum() - dlt / k) / 2])
        want = dict(internal_conflict=2 * w * w * dlt * dlt / k ** 2, disagreement=w * dlt * dlt / k ** 2,
                    polarization=dlt * dlt / (2 * k ** 2), controversy=float(z @ z), dc_index=float(s @ z))
        cases.append((f"edge w={w}", W.csr_from_edges(2, [(0, 1)], [w]), s, z, want))
    for n, w in ((9, 1.0), (12, 0.75)):  # K_n: z = mean(s) 1 + sbar / (1 + w n)
        s = rng.random(n)
        mu = s.mean()
        sb = s - mu
        k = 1.0 + w * n
        z = mu + sb / k
        sb2 = float(sb @ sb)
        want = dict(internal_conflict=(w * n) ** 2 * sb2 / k ** 2, disagreement=w * n * sb2 / k ** 2,
                    polarization=sb2 / k ** 2, controversy=n * mu * mu + sb2 / k ** 2,
                    dc_index=n * mu * mu + sb2 / k)
        cases.append((f"K_{n}", W.complete_graph(n, None if w == 1.0 else w), s, z, want))
    n = 7  # edgeless: z = s
    s = rng.random(n)
    sb = s - s.mean()
    cases.append(("edgeless", W.csr_from_edges(n, np.zeros((0, 2), dtype=np.int64)), s, s.copy(),
                  dict(internal_conflict=0.0, disagreement=0.0, polarization=float(sb @ sb),
                       controversy=float(s @ s), dc_index=float(s @ s))))
    g = W.barabasi_albert(300, 3, 8)  # constant opinions: z = s
    s = np.full(g.n, 0.37)
    cases.append(("constant s", g, s, s.copy(),
                  dict(internal_conflict=0.0, disagreement=0.0, polarization=0.0,
                       controversy=g.n * 0.37 ** 2, dc_index=g.n * 0.37 ** 2)))
    return cases


def _perturbations(z, s, rng):
    u = rng.standard_normal(z.shape[0])
    u /= np.linalg.norm(u)
    sb = s - s.mean()
    dirs = [z, -z, np.ones_like(z), np.linalg.norm(z) * u]
    if np.linalg.norm(sb) > 0:
        dirs += [sb, -sb]
    for t in (1e-2, 1e-4, 1e-7):
        for d in dirs:
            yield t, t * d


def pin_error_bounds(sparse):
    """The oracle's certificate (reading of Algorithm 1's guarantee through the
    Section 4 ordering I <= I + L) at perturbed points z~ = z + e of graphs
    with a closed-form equilibrium, where the true error of every index is
    known: each bound is at least the actual relative error, certifies
    nothing (>= 1/2) where the true index is 0, and is within a stated
    factor of the actual error where the perturbation attains the bound."""
    rng = np.random.default_rng(23)
    for name, g, s, z, want in _closed_form_cases():
        for t, e in _perturbations(z, s, rng):
            vals = sparse.indices_at(g, s, z + e)
            bnd = sparse.error_bounds(vals)
            for k in NAMES:
                if want[k] == 0.0:
                    # no relative bound exists; any value >= 1/2 certifies nothing for an
                    # admissible eps (Algorithm 1 takes eps in (0, 1/2)). At the boundary
                    # sqrt(X~) = rho rounding may give a huge finite value instead of inf.
                    if not bnd[k] >= 0.5:
                        raise AssertionError(f"{name}: relative bound {bnd[k]} for a zero {k}")
                    continue
                actual = abs(vals[k] - want[k]) / want[k]
                if not actual <= bnd[k] * (1 + 1e-9) + 1e-13:
                    raise AssertionError(f"{name} t={t}: {k} error {actual} above its bound {bnd[k]}")
    # Perturbations that attain the bound to first order (factor 1 + O(t)).
    t = 1e-4

    def ratio(g, s, z, zt, want, k):
        vals = sparse.indices_at(g, s, zt)
        return sparse.error_bounds(vals)[k] / (abs(vals[k] - want[k]) / want[k])

    cases = {c[0]: c[1:] for c in _closed_form_cases()}
    g, s, z, want = cases["constant s"]
    # e = -t z is constant, (I + L) e = e: rho = t ||z|| = |sqrt(C) - sqrt(C~)|
    for k, hi in (("controversy", 1.001), ("dc_index", 1.001)):
        r = ratio(g, s, z, (1 - t) * z, want, k)
        if not 1.0 <= r <= hi:
            raise AssertionError(f"constant s: {k} bound / error = {r}, expected in [1, {hi}]")
    g, s, z, want = cases["edgeless"]  # L = 0: e = t sbar gives rho = sqrt(P~) - sqrt(P)
    r = ratio(g, s, z, z + t * (s - s.mean()), want, "polarization")
    if not 1.0 <= r <= 1.001:
        raise AssertionError(f"edgeless: polarization bound / error = {r}")
    # single edge: e along z - s (eigenvalue 2w of L): rho = (1 + 2w) |sqrt(C_I~) - sqrt(C_I)|,
    # and at w = 1/2 the disagreement form sees half of rho (hence a factor 2 at best)
    g, s, z, want = cases["edge w=0.001"]
    r = ratio(g, s, z, z + t * (z - s), want, "internal_conflict")
    if not 1.0 <= r <= 1.01:
        raise AssertionError(f"edge: internal conflict bound / error = {r}")
    g, s, z, want = cases["edge w=0.5"]
    r = ratio(g, s, z, z + t * np.array([1.0, -1.0]), want, "disagreement")
    if not 1.0 <= r <= 2.01:
        raise AssertionError(f"edge: disagreement bound / error = {r}")


def pin_certified_flag(sparse):
    """indices() certifies only when every index meets the requested bound:
    nearly constant opinions make P, D and C_I tiny, so a residual that
    certifies C and I_dc to 1e-9 does not certify them."""
    g = W.barabasi_albert(400, 3, 51)
    s = 0.5 + 1e-6 * W.opinions("uniform", g.n, 52)
    _, _, loose = sparse.indices(g, s, rtol=1e-9, certify=1e-9)
    if loose["certified"]:
        raise AssertionError(f"certified although some bound exceeds 1e-9: {loose['bounds']}")
    if not min(loose["bounds"].values()) <= 1e-9:
        raise AssertionError("case does not separate 'every index' from 'some index'")
    _, _, tight = sparse.indices(g, W.opinions("uniform", g.n, 52))
    if not tight["certified"]:
        raise AssertionError(f"not certified at the oracle tolerance: {tight['bounds']}")


def pin_sparse_forms(indices_at_fn, solve_fn):
    """Lemma 4.1 (C_I = ||L z||^2) and Proposition 1 (D = z^T L z) against the
    definitions: at the closed-form equilibria exactly, and at the solved z of
    larger graphs to within the solve's residual."""
    for name, g, s, z, want in _closed_form_cases():
        v = indices_at_fn(g, s, z)
        scale = float(s @ s)
        _close(v["lz_norm2"], want["internal_conflict"], 1e-11, 1e-15 * scale, f"{name} ||Lz||^2")
        _close(v["zlz"], want["disagreement"], 1e-11, 1e-15 * scale, f"{name} z^T L z")
    graphs = [W.barabasi_albert(500, 3, 21), W.random_graph(200, 0.05, 22, weighted=True),
              W.chung_lu(3000, 2.3, 8.0, 23, weighted=True)]
    for g in graphs:
        s = W.opinions("exp", g.n, 33)
        v = indices_at_fn(g, s, solve_fn(g, s))
        _close(v["lz_norm2"], v["internal_conflict"], 1e-9, what="Lemma 4.1 ||Lz||^2 = C_I")
        _close(v["zlz"], v["disagreement"], 1e-9, what="Prop. 1 z^T L z = D")
