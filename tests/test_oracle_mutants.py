"""Plants plausible mistakes in copies of the CPU oracle and shows the pins catch each.

Every mutant is a one-token change to `oracle/tableau_simplex.c`, compiled to a
temporary library. The battery below reuses the independent pins (hand-worked
example, vertex enumeration, exact-rational pivot sequence, closed forms,
certificates, the iteration cap); a mutant is caught when any of them fails.
"""

import os
import tempfile
from fractions import Fraction

import numpy as np
import pytest

import oracle
from exact_ref import brute_force_optimum, exact_simplex
from goldens import read_fixture
from paper_2211_10979_amd import lpgen

SRC = os.path.join(os.path.dirname(oracle.__file__), "tableau_simplex.c")
GENERAL_MARK = "/* ------------------------------------------------------------------------\n * General form:"

MUTANTS = {
    "update_sign": ("row[j] = fma(mf, R[j], row[j]);", "row[j] = fma(-mf, R[j], row[j]);"),
    "pricing_tie_high": ("if (v < best) {", "if (v <= best) {"),
    "ratio_tie_high": ("if (r < 0 || ratio < best) {", "if (r < 0 || ratio <= best) {"),
    "rhs_not_updated": ("for (int j = 0; j < W; ++j) row[j] = fma(", "for (int j = 0; j < W - 1; ++j) row[j] = fma("),
    "normalise_multiplies": ("o->R[j] = TAB(o, r, j) / p;", "o->R[j] = TAB(o, r, j) * p;"),
    "basis_not_updated": ("o->basis[r - 1] = q;", "(void)q;"),
    "eligible_nonzero": ("if (a > o->eps_p) {", "if (a != 0.0) {"),
    "cost_sign": ("TAB(o, 0, j) = -c[j];", "TAB(o, 0, j) = c[j];"),
    "dual_index": ("y[i - 1] = TAB(o, 0, n + i - 1);", "y[i - 1] = TAB(o, 0, i - 1);"),
    "ratio_wrong_column": ("double rhs = TAB(o, i, W - 1);", "double rhs = TAB(o, i, W - 2);"),
    "pricing_skips_slacks": ("for (int j = 0; j < o->n + o->m; ++j) {", "for (int j = 0; j < o->n; ++j) {"),
    "ratio_skips_last_row": ("for (int i = 1; i <= o->m; ++i) {\n        double a", "for (int i = 1; i < o->m; ++i) {\n        double a"),
    "cap_off_by_one": ("if (o->pivots >= o->max_pivots)", "if (o->pivots > o->max_pivots)"),
    "pivot_row_not_normalised": ("for (int j = 0; j < W; ++j) row[j] = R[j];", "for (int j = 0; j < W; ++j) row[j] = row[j];"),
    "x_from_wrong_row": ("x[o->basis[i - 1]] = TAB(o, i, W - 1);", "x[o->basis[i - 1]] = TAB(o, i - 1, W - 1);"),
    "step1_nan_ignored": ("if (isnan(v)) return -2;", "(void)0;"),
    "step1_neg_inf_ignored": ("if (best == -INFINITY) return -2;", "(void)0;"),
    "step2_inf_column_ignored": ("if (!isfinite(a) || isnan(rhs)) return -2;", "if (isnan(a) || isnan(rhs)) return -2;"),
    "step2_nan_rhs_ignored": ("if (!isfinite(a) || isnan(rhs)) return -2;", "if (!isfinite(a)) return -2;"),
    "step2_nan_rhs_eligible_rows_only": ("if (!isfinite(a) || isnan(rhs)) return -2;\n        if (a > o->eps_p) {",
                                         "if (!isfinite(a)) return -2;\n        if (a > o->eps_p) {\n            if (isnan(rhs)) return -2;"),
}

NONFINITE_FIXTURES = ["nonfinite_step2_nan_rhs.txt", "nonfinite_step1_neg_inf.txt",
                      "nonfinite_step2_inf_column.txt", "nonfinite_step1_nan.txt"]


def _battery(lib):
    """Runs the pins against the library at `lib`; returns the first failure or None."""

    def solve(A, b, c, **kw):
        return oracle.solve(A, b, c, library=lib, threads=2, **kw)

    fx = read_fixture("hand_example.txt")
    r = solve(fx["A"], fx["b"], fx["c"])
    if list(zip(r["rows"].tolist(), r["cols"].tolist())) != fx["pivot"]:
        return "hand example pivots"
    if abs(r["objective"] - fx["objective"]) > 1e-12 or not np.allclose(r["y"], fx["y"]) \
            or not np.allclose(r["x"], fx["x"]):
        return "hand example solution"
    for name in NONFINITE_FIXTURES:
        nf = read_fixture(name)
        r = solve(nf["A"], nf["b"], nf["c"])
        if oracle.STATUS_NAMES[r["status"]] != nf["status"] or r["pivots"] != nf["pivots"] \
                or list(zip(r["rows"].tolist(), r["cols"].tolist())) != nf["pivot"]:
            return f"non-finite fixture {name}"
    rng = np.random.default_rng(5)
    for t in range(12):
        m, n = int(rng.integers(1, 6)), int(rng.integers(1, 6))
        A = rng.integers(1, 20, size=(m, n)).astype(float)
        b = rng.integers(1, 20, size=m).astype(float)
        c = rng.integers(1, 20, size=n).astype(float)
        best, _ = brute_force_optimum(A, b, c)
        r = solve(A, b, c)
        if r["status"] != 0 or abs(r["objective"] - float(best)) > 1e-9 * max(1, abs(float(best))):
            return f"vertex enumeration {t}"
    for t in range(6):
        m, n = int(rng.integers(3, 15)), int(rng.integers(3, 15))
        A = rng.integers(1, 5, size=(m, n)).astype(float)
        b = rng.integers(1, 5, size=m).astype(float)
        c = rng.integers(1, 5, size=n).astype(float)
        ex = exact_simplex(A, b, c, 1e-9, 1e-9)
        r = solve(A, b, c)
        if list(zip(r["rows"].tolist(), r["cols"].tolist())) != ex.log:
            return f"exact pivot sequence {t}"
    # a signed LP whose optimal path re-enters a slack column (pivot (5, 12))
    srng = np.random.default_rng(4)
    m, n = int(srng.integers(3, 10)), int(srng.integers(3, 10))
    A = srng.integers(1, 10, size=(m, n)).astype(float) * srng.choice([-1.0, 1.0], size=(m, n), p=[0.3, 0.7])
    b = srng.integers(1, 10, size=m).astype(float)
    c = srng.integers(1, 10, size=n).astype(float)
    ex = exact_simplex(A, b, c, 1e-9, 1e-9)
    assert any(q >= n for _, q in ex.log)
    r = solve(A, b, c)
    if list(zip(r["rows"].tolist(), r["cols"].tolist())) != ex.log:
        return "exact pivot sequence, slack re-entry"
    d = np.array([3.0, 5.0, 2.0, 7.0])
    c = np.array([2.0, 4.0, 4.0, 1.0])
    b = np.array([9.0, 10.0, 4.0, 14.0])
    r = solve(np.diag(d), b, c)
    if r["cols"].tolist() != [1, 2, 0, 3] or not np.allclose(r["y"], c / d):
        return "diagonal closed form"
    a = np.array([[2.0], [3.0], [1.0], [3.0]])
    bb = np.array([8.0, 6.0, 5.0, 6.0])
    r = solve(a, bb, np.array([1.0]))
    if r["rows"].tolist() != [2]:
        return "single-variable ratio tie"
    lp = lpgen.dense_lp(1, 60, 60)
    r = solve(lp.A, lp.b, lp.c)
    if not oracle.certificates(lp.A, lp.b, lp.c, r["x"], r["y"], r["objective"])["ok"]:
        return "certificates"
    r1 = solve(lp.A, lp.b, lp.c, max_pivots=1)
    if r1["status"] != oracle.ITER_LIMIT or r1["pivots"] != 1:
        return "iteration cap"
    return None


def test_battery_passes_on_the_oracle():
    assert _battery(None) is None


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    # these mutants target the standard form; the general form's section
    # (after GENERAL_MARK) has its own battery in test_oracle_general.py
    cut = src.index(GENERAL_MARK)
    head, tail = src[:cut], src[cut:]
    assert head.count(old) == 1, f"mutation site for {name} not found exactly once"
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "mutant.c")
        with open(path, "w") as f:
            f.write(head.replace(old, new) + tail)
        lib = oracle.build(src=path, out=os.path.join(d, f"lib_{name}.so"))
        caught = _battery(lib)
    assert caught is not None, f"mutant {name} survived every pin"
