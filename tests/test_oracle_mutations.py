"""Planted mistakes: each test copies an oracle source file, plants one
plausible mistake (a dropped term, a wrong sign, a wrong index, a swapped
operand), and checks that at least one pin from tests/oracle_pins.py fails on
the broken copy. Mistakes are planted on the CPU only, in temporary copies."""
import os
import types

import numpy as np
import pytest

import oracle_pins as P
from oracle import circulant, dense, forest, sparse

ORACLE_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")


def _mutate(path, old, new):
    src = open(path).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {old!r}"
    return src.replace(old, new, 1)


def _module_from(src, name):
    mod = types.ModuleType(name)
    exec(compile(src, name, "exec"), mod.__dict__)
    return mod


def _some_pin_fails(pins):
    for pin in pins:
        try:
            pin()
        except (AssertionError, np.linalg.LinAlgError, ZeroDivisionError, ValueError,
                FloatingPointError, OverflowError):
            return True
    return False


# ---------------------------------------------------------------- C oracle

C_MUTANTS = {
    "apply drops identity": ("y[i] = x[i] + nval(deg) * x[i] - nval(ax);",
                             "y[i] = nval(deg) * x[i] - nval(ax);"),
    "apply adjacency sign": ("y[i] = x[i] + nval(deg) * x[i] - nval(ax);",
                             "y[i] = x[i] + nval(deg) * x[i] + nval(ax);"),
    "apply wrong weight index": ("nadd(&ax, weight(w, k) * x[col[k]]);",
                                 "nadd(&ax, weight(w, rp[i]) * x[col[k]]);"),
    "apply own value for neighbour": ("nadd(&ax, weight(w, k) * x[col[k]]);",
                                      "nadd(&ax, weight(w, k) * x[i]);"),
    "residual sign": ("for (int32_t i = 0; i < n; ++i) r[i] = s[i] - r[i];",
                      "for (int32_t i = 0; i < n; ++i) r[i] = s[i] + r[i];"),
    "cg residual update uses p": ("r[i] -= alpha * q[i];", "r[i] -= alpha * p[i];"),
    "cg beta inverted": ("double beta = rz_new / rz;", "double beta = rz / rz_new;"),
    "disagreement counts both directions": ("if (j > i) {", "if (j != i) {"),
    "disagreement drops weight": ("nadd(&d, weight(w, k) * e * e);", "nadd(&d, e * e);"),
    "conflict wrong index": ("double dz = z[i] - s[i];", "double dz = z[i] - s[(i + 1) % n];"),
    "polarization mean over n-1": ("double mean = sumz / (double)n;",
                                   "double mean = sumz / (double)(n - 1);"),
    "controversy uses s": ("nadd(&cc, z[i] * z[i]);", "nadd(&cc, s[i] * z[i]);"),
    "dc index uses s twice": ("nadd(&idc, s[i] * z[i]);", "nadd(&idc, s[i] * s[i]);"),
    "fj update drops self weight": ("nadd(&den, 1.0);", ";"),
    "fj update drops internal opinion": ("nadd(&num, s[i]);", ";"),
    "Lemma 4.1 form drops the degree": ("lz[i] = nval(deg) * z[i] - nval(az);", "lz[i] = z[i] - nval(az);"),
    "Lemma 4.1 norm not squared": ("nadd(&l2, lz[i] * lz[i]);", "nadd(&l2, lz[i]);"),
    "Prop. 1 form uses s": ("nadd(&zlz, z[i] * lz[i]);", "nadd(&zlz, s[i] * lz[i]);"),
    "residual norm squared": ("return sqrt(dot(n, r, r));", "return dot(n, r, r);"),
}


def _sparse_pins():
    def ind(g, s):
        vals, _, info = sparse.indices(g, s)
        assert info["status"] == 0, "not converged"
        return vals

    def sol(g, s):
        z, info = sparse.solve(g, s)
        assert info["status"] == 0, "not converged"
        return z

    def fj(g, s):
        z, info = sparse.fj_iterate(g, s, max_sweeps=20000, tol=1e-15)
        assert info["status"] == 0, "not converged"
        return z

    return [lambda: P.pin_p5_sparse(sol),
            lambda: P.pin_closed_forms(ind),
            lambda: P.pin_circulant(ind, sol, circulant),
            lambda: P.pin_identities(ind, sol),
            lambda: P.pin_fj_dynamics(fj, sol),
            lambda: P.pin_sparse_forms(sparse.indices_at, sol),
            lambda: P.pin_error_bounds(sparse),
            lambda: P.pin_certified_flag(sparse)]


def test_unmutated_c_oracle_passes_every_pin(tmp_path):
    lib = sparse.build(os.path.join(ORACLE_DIR, "fj_oracle.c"), str(tmp_path / "ok.so"))
    with sparse.swapped(lib):
        assert not _some_pin_fails(_sparse_pins())


@pytest.mark.parametrize("name", sorted(C_MUTANTS))
def test_c_oracle_mutant_is_caught(name, tmp_path):
    old, new = C_MUTANTS[name]
    src = tmp_path / "mutant.c"
    src.write_text(_mutate(os.path.join(ORACLE_DIR, "fj_oracle.c"), old, new))
    lib = sparse.build(str(src), str(tmp_path / "mutant.so"))
    with np.errstate(all="ignore"), sparse.swapped(lib):
        assert _some_pin_fails(_sparse_pins()), f"no pin caught: {name}"


# ---------------------------------------------------------------- Python oracle

DENSE_MUTANTS = {
    "laplacian adjacency sign": ("return np.diag(A.sum(axis=1)) - A", "return np.diag(A.sum(axis=1)) + A"),
    "laplacian unweighted degree": ("return np.diag(A.sum(axis=1)) - A",
                                    "return np.diag((A > 0).sum(axis=1)) - A"),
    "adjacency ignores weights": ("A[i, int(g.col[k])] += w[k]", "A[i, int(g.col[k])] += 1.0"),
    "forest matrix drops identity": ("return np.linalg.inv(np.eye(g.n) + laplacian_dense(g))",
                                     "return np.linalg.pinv(laplacian_dense(g))"),
    "equilibrium sign": ("np.linalg.solve(np.eye(g.n) + laplacian_dense(g), np.asarray",
                         "np.linalg.solve(np.eye(g.n) - laplacian_dense(g), np.asarray"),
    "disagreement not squared": ("(w * (z[lo] - z[hi]) ** 2)", "(w * (z[lo] - z[hi]))"),
    "conflict against mean": ("((z - s) ** 2)", "((z - s.mean()) ** 2)"),
    "polarization mean over n-1": ("mean_z = math.fsum(z.tolist()) / g.n",
                                   "mean_z = math.fsum(z.tolist()) / (g.n - 1)"),
    "incidence head sign": ("B[np.arange(m), hi] = -1.0", "B[np.arange(m), hi] = 1.0"),
    "prop1 polarization uncentred": ("polarization=float(sbar @ Om @ Om @ sbar)",
                                     "polarization=float(s @ Om @ Om @ s)"),
    "prop1 conflict single L": ("internal_conflict=float(s @ Om @ L @ L @ Om @ s)",
                                "internal_conflict=float(s @ Om @ L @ Om @ s)"),
}


def _dense_pins(D):
    return [lambda: P.pin_p5_forest_matrix(D),
            lambda: P.pin_forest_bruteforce(D, forest),
            lambda: P.pin_prop1_and_lemma41(D),
            lambda: P.pin_closed_forms(D.indices),
            lambda: P.pin_circulant(D.indices, D.equilibrium, circulant)]


@pytest.mark.parametrize("name", sorted(DENSE_MUTANTS))
def test_dense_oracle_mutant_is_caught(name):
    old, new = DENSE_MUTANTS[name]
    D = _module_from(_mutate(dense.__file__, old, new), "dense_mutant")
    with np.errstate(all="ignore"):
        assert _some_pin_fails(_dense_pins(D)), f"no pin caught: {name}"


FOREST_MUTANTS = {
    "root of i's tree not fixed": ("others = prod_all // size[labels[i]]", "others = prod_all"),
    "forests left unrooted": ("prod_all *= sz", "prod_all *= 1"),
    "edge weights ignored": ("wF *= weights[e]", "wF *= 1"),
}


@pytest.mark.parametrize("name", sorted(FOREST_MUTANTS))
def test_forest_mutant_is_caught(name):
    old, new = FOREST_MUTANTS[name]
    Fm = _module_from(_mutate(forest.__file__, old, new), "forest_mutant")
    assert _some_pin_fails([lambda: P.pin_p5_forest_enumeration(Fm),
                            lambda: P.pin_forest_bruteforce(dense, Fm)])


CIRCULANT_MUTANTS = {
    "eigenvalue factor": ("return 2.0 * w * (1.0 - np.cos(2.0 * np.pi * k / n))",
                          "return w * (1.0 - np.cos(2.0 * np.pi * k / n))"),
    "polarization keeps mean mode": ("p = c - float((shat2 * g * g).flat[0]) / n", "p = c"),
    "dc index squared kernel": ("idc = float(np.sum(shat2 * g)) / n", "idc = float(np.sum(shat2 * g * g)) / n"),
}


@pytest.mark.parametrize("name", sorted(CIRCULANT_MUTANTS))
def test_circulant_mutant_is_caught(name):
    old, new = CIRCULANT_MUTANTS[name]
    Cm = _module_from(_mutate(circulant.__file__, old, new), "circulant_mutant")
    assert _some_pin_fails([lambda: P.pin_circulant(dense.indices, dense.equilibrium, Cm)])


# ------------------------------------------------ the oracle's certificate (sparse.py)

# Not listed, because each still bounds the error:
#  - dropping rho^2 from the numerator: rho (2 rx - rho) / (rx - rho)^2 is the exact worst
#    case of |X - X~| / X given |sqrt(X) - sqrt(X~)| <= rho (the oracle's form is looser);
#  - ||z~|| rho instead of (||z~|| + rho) rho for I_dc: the difference is of order rho^2,
#    and the relative form a / (I_dc~ - a) over-covers it by more than that.
SPARSE_MUTANTS = {
    "bound denominator (rx + rho)^2": ("/ (rx - rho) ** 2", "/ (rx + rho) ** 2"),
    "bound drops the factor 2": ("rho * (2 * rx + rho)", "rho * (rx + rho)"),
    "residual norm squared": ('rho = vals["residual_norm"]', 'rho = vals["residual_norm"] ** 2'),
    "certified when any index meets": ("all(b <= certify", "any(b <= certify"),
}


def _sparse_module_from(src):
    mod = types.ModuleType("sparse_mutant")
    mod.__dict__["__file__"] = sparse.__file__  # same C library
    exec(compile(src, "sparse_mutant", "exec"), mod.__dict__)
    return mod


def test_unmutated_sparse_module_passes_certificate_pins():
    S = _sparse_module_from(open(sparse.__file__).read())
    assert not _some_pin_fails([lambda: P.pin_error_bounds(S), lambda: P.pin_certified_flag(S)])


@pytest.mark.parametrize("name", sorted(SPARSE_MUTANTS))
def test_sparse_certificate_mutant_is_caught(name):
    old, new = SPARSE_MUTANTS[name]
    S = _sparse_module_from(_mutate(sparse.__file__, old, new))
    with np.errstate(all="ignore"):
        assert _some_pin_fails([lambda: P.pin_error_bounds(S), lambda: P.pin_certified_flag(S)]), \
            f"no pin caught: {name}"
