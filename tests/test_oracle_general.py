"""Pins of the CPU oracle's general form (rows <=, >= or =, any sign of b; the
two-phase method), none of them the oracle itself:

* on <= rows with b >= 0 it must reproduce the standard method bit for bit
  (Phase I is empty there and the extra rows and columns change no value);
* an exact-rational run of the same two-phase construction and rules
  (tests/exact_ref.py) fixes the pivot sequence and the status;
* brute-force vertex enumeration of the equality form fixes the optimum and
  infeasibility without any simplex logic;
* scipy's HiGHS fixes status and objective on larger LPs;
* closed forms (identity equality systems, contradictory rows, a row that
  forces a drive-out on a negative entry, redundant rows);
* general optimality certificates (primal and dual feasibility with the sign
  rules of each row type, zero duality gap);
* planted mistakes in a copy of the general section are each caught.
"""

import os
import tempfile
from fractions import Fraction

import numpy as np
import pytest

import oracle
from exact_ref import EQ, GE, LE, brute_force_general, exact_general


def random_general(rng, m, n, lo=-5, hi=9, bound=None):
    A = rng.integers(lo, hi + 1, size=(m, n)).astype(float)
    b = rng.integers(-6, 12, size=m).astype(float)
    c = rng.integers(-3, 8, size=n).astype(float)
    sense = rng.integers(0, 3, size=m)
    if bound is not None:  # a <= row that bounds every variable
        A = np.vstack([A, np.ones(n)])
        b = np.append(b, bound)
        sense = np.append(sense, LE)
    return A, b, c, sense


def test_reduces_to_the_standard_form_bit_for_bit():
    rng = np.random.default_rng(1)
    for t in range(30):
        m, n = int(rng.integers(1, 30)), int(rng.integers(1, 30))
        A = rng.integers(1 if t % 2 else -4, 20, size=(m, n)).astype(float)
        b = rng.integers(0, 30, size=m).astype(float)
        c = rng.integers(-5, 20, size=n).astype(float)
        g = oracle.solve_general(A, b, c, np.full(m, LE), threads=2)
        s = oracle.solve(A, b, c, threads=2)
        assert g["status"] == s["status"] and g["pivots"] == s["pivots"]
        assert g["rows"].tolist() == s["rows"].tolist() and g["cols"].tolist() == s["cols"].tolist()
        assert np.array_equal(g["x"], s["x"]) and np.array_equal(g["y"], s["y"])
        assert g["objective"] == s["objective"]
        # the standard tableau is rows 0..m of the general one without the
        # carried row's own column (n + m)
        o = oracle.OracleLP(A, b, c, threads=2)
        o.step(-1)
        T = g["tableau"]
        W = T.shape[1]
        keep = [j for j in range(W) if j != n + m]
        assert np.array_equal(T[: m + 1][:, keep], o.tableau())
        o.close()


def test_exact_two_phase_pivot_sequence():
    rng = np.random.default_rng(2)
    eps = Fraction(1, 10**9)
    compared = skipped = 0
    statuses = set()
    for t in range(120):
        m, n = int(rng.integers(1, 7)), int(rng.integers(1, 7))
        A, b, c, sense = random_general(rng, m, n)
        g = oracle.solve_general(A, b, c, sense, threads=1)
        e = exact_general(A, b, c, sense, eps_d=eps, eps_p=eps)
        same = (list(zip(g["rows"].tolist(), g["cols"].tolist())) == e.log
                and oracle.STATUS_NAMES[g["status"]] == e.status)
        if not same:
            assert min(e.near_ties, default=1.0) < 1e-9, (t, e.log, g["rows"], g["cols"], e.status)
            skipped += 1
            continue
        compared += 1
        statuses.add(e.status)
        if e.status == "OPTIMAL":
            ex = [float(v) for v in e.x()]
            ey = [float(v) for v in e.y()]
            assert np.allclose(g["x"], ex, rtol=1e-9, atol=1e-9)
            assert np.allclose(g["y"], ey, rtol=1e-9, atol=1e-9)
            assert abs(g["objective"] - float(e.objective())) <= 1e-9 * max(1.0, abs(float(e.objective())))
    assert compared >= 110 and {"OPTIMAL", "INFEASIBLE", "UNBOUNDED"} <= statuses, (compared, statuses)


def test_brute_force_optimum_and_infeasibility():
    rng = np.random.default_rng(3)
    seen = {"OPTIMAL": 0, "INFEASIBLE": 0}
    for t in range(80):
        m, n = int(rng.integers(1, 4)), int(rng.integers(1, 4))
        A, b, c, sense = random_general(rng, m, n, bound=40.0)
        S = np.hstack([A, np.array([[1.0 if sense[i] == LE else -1.0 if sense[i] == GE else 0.0]
                                     for i in range(len(b))]) * np.eye(len(b))])
        if np.linalg.matrix_rank(S) < len(b):
            continue
        best, _ = brute_force_general(A, b, c, sense)
        g = oracle.solve_general(A, b, c, sense, threads=1)
        if best is None:
            assert g["status"] == oracle.INFEASIBLE, t
            seen["INFEASIBLE"] += 1
        else:
            assert g["status"] == oracle.OPTIMAL, t
            assert abs(g["objective"] - float(best)) <= 1e-9 * max(1.0, abs(float(best))), t
            seen["OPTIMAL"] += 1
    assert seen["OPTIMAL"] >= 20 and seen["INFEASIBLE"] >= 5, seen


def feasible_general(rng, m, n, bound=None):
    """Mixed rows around a known nonnegative integer point x0, so the LP is
    feasible; with `bound`, also bounded."""
    A = rng.integers(-5, 10, size=(m, n)).astype(float)
    x0 = rng.integers(0, 4, size=n).astype(float)
    sense = rng.integers(0, 3, size=m)
    slack = rng.integers(0, 5, size=m).astype(float)
    b = A @ x0 + np.where(sense == LE, slack, np.where(sense == GE, -slack, 0.0))
    c = rng.integers(-3, 8, size=n).astype(float)
    if bound is not None:
        A = np.vstack([A, np.ones(n)])
        b = np.append(b, bound)
        sense = np.append(sense, LE)
    return A, b, c, sense


def test_highs_status_and_objective():
    scipy_opt = pytest.importorskip("scipy.optimize")
    rng = np.random.default_rng(4)
    counts = {}
    for t in range(45):
        m, n = int(rng.integers(2, 40)), int(rng.integers(2, 40))
        if t % 3 == 0:
            A, b, c, sense = random_general(rng, m, n, lo=-3, hi=9)
        elif t % 3 == 1:
            A, b, c, sense = feasible_general(rng, m, n, bound=200.0)
        else:
            A, b, c, sense = feasible_general(rng, m, n)
        ub, eq = sense != EQ, sense == EQ
        A_ub = np.where((sense == GE)[:, None], -A, A)[ub]
        b_ub = np.where(sense == GE, -b, b)[ub]
        h = scipy_opt.linprog(-c, A_ub=A_ub if ub.any() else None, b_ub=b_ub if ub.any() else None,
                              A_eq=A[eq] if eq.any() else None, b_eq=b[eq] if eq.any() else None,
                              bounds=(0, None), method="highs")
        g = oracle.solve_general(A, b, c, sense, threads=2)
        want = {0: oracle.OPTIMAL, 2: oracle.INFEASIBLE, 3: oracle.UNBOUNDED}[h.status]
        assert g["status"] == want, (t, h.status, g["status"])
        counts[want] = counts.get(want, 0) + 1
        if want == oracle.OPTIMAL:
            assert abs(g["objective"] + h.fun) <= 1e-9 * max(1.0, abs(h.fun)), t
            cert = oracle.certificates_general(A, b, c, sense, g["x"], g["y"], g["objective"])
            assert cert["ok"], (t, cert)
    assert counts.get(oracle.OPTIMAL, 0) >= 10 and counts.get(oracle.INFEASIBLE, 0) >= 3, counts


def test_closed_forms():
    # contradictory rows: x1 <= 1 and x1 >= 2
    g = oracle.solve_general([[1.0], [1.0]], [1.0, 2.0], [1.0], [LE, GE])
    assert g["status"] == oracle.INFEASIBLE and g["pivots"] >= 1
    # a <= row with b < 0 and nonnegative coefficients: infeasible
    g = oracle.solve_general([[1.0, 1.0]], [-1.0], [1.0, 1.0], [LE])
    assert g["status"] == oracle.INFEASIBLE
    # -x1 >= -3 is x1 <= 3: max x1 = 3, dual of the original row -1
    g = oracle.solve_general([[-1.0]], [-3.0], [1.0], [GE])
    assert g["status"] == oracle.OPTIMAL and g["x"].tolist() == [3.0] and g["objective"] == 3.0
    assert g["y"].tolist() == [-1.0]
    # x1 - x2 >= 1 with max x1: unbounded
    g = oracle.solve_general([[1.0, -1.0]], [1.0], [1.0, 0.0], [GE])
    assert g["status"] == oracle.UNBOUNDED
    # identity equality system: x = b, objective c.b, duals y = c
    rng = np.random.default_rng(5)
    k = 7
    b = rng.integers(0, 9, size=k).astype(float)
    c = rng.integers(-4, 9, size=k).astype(float)
    g = oracle.solve_general(np.eye(k), b, c, np.full(k, EQ))
    assert g["status"] == oracle.OPTIMAL
    assert np.array_equal(g["x"], b) and g["objective"] == float(c @ b) and np.array_equal(g["y"], c)
    # a row that forces a drive-out on a negative entry: -x1 - x2 = 0 keeps
    # its artificial variable basic at zero after Phase I; Phase II must keep
    # x1 = x2 = 0
    g = oracle.solve_general([[-1.0, -1.0], [1.0, 0.0]], [0.0, 5.0], [1.0, 1.0], [EQ, LE])
    assert g["status"] == oracle.OPTIMAL and g["objective"] == 0.0 and g["x"].tolist() == [0.0, 0.0]
    assert (2, 0) in list(zip(g["rows"].tolist(), g["cols"].tolist()))  # the drive-out pivot
    # a redundant equality (a duplicated row) stays with its artificial
    # variable basic; the optimum is unaffected
    A = np.array([[1.0, 2.0], [1.0, 2.0], [1.0, 0.0]])
    g = oracle.solve_general(A, [4.0, 4.0, 3.0], [1.0, 1.0], [EQ, EQ, LE])
    assert g["status"] == oracle.OPTIMAL and abs(g["objective"] - 3.5) <= 1e-12
    cert = oracle.certificates_general(A, [4.0, 4.0, 3.0], [1.0, 1.0], [EQ, EQ, LE], g["x"], g["y"], g["objective"])
    assert cert["ok"], cert


def test_basic_columns_stay_unit_vectors():
    rng = np.random.default_rng(6)
    for t in range(25):
        m, n = int(rng.integers(2, 15)), int(rng.integers(2, 15))
        A, b, c, sense = random_general(rng, m, n, lo=-2, hi=9, bound=60.0)
        g = oracle.solve_general(A, b, c, sense, threads=2)
        if g["status"] != oracle.OPTIMAL:
            continue
        T, basis = g["tableau"], g["basis"]
        M = len(basis)
        for row, j in enumerate(basis[:-1], start=1):
            col = T[:, j]
            unit = np.zeros(M + 1)
            unit[row] = 1.0
            assert np.array_equal(col, unit), (t, row, j)


def test_certificate_checker_rejects_bad_points():
    A = np.array([[1.0, 1.0], [1.0, -1.0]])
    b = np.array([4.0, 1.0])
    c = np.array([1.0, 2.0])
    sense = np.array([EQ, GE])
    good = oracle.certificates_general(A, b, c, sense, [2.5, 1.5], [1.5, -0.5], 5.5)
    assert good["ok"]
    assert not oracle.certificates_general(A, b, c, sense, [3.0, 1.0], [1.5, -0.5], 5.0)["ok"]  # gap
    assert not oracle.certificates_general(A, b, c, sense, [2.5, 1.5], [1.5, 0.5], 5.5)["ok"]  # y sign on >=
    assert not oracle.certificates_general(A, b, c, sense, [2.0, 1.5], [1.5, -0.5], 5.0)["ok"]  # primal


# ---------------------------------------------------------------- planted mistakes

SRC = os.path.join(os.path.dirname(oracle.__file__), "tableau_simplex.c")

MUTANTS = {
    "negative_rows_not_flipped": ("if (b[i] < 0.0 && k != 2) k = 1 - k;", "(void)0;"),
    "surplus_sign": ("TAB(o, t1, surplus++) = -1.0;", "TAB(o, t1, surplus++) = 1.0;"),
    "phase1_row_added": ("TAB(o, 0, j) = TAB(o, 0, j) - TAB(o, t1, j);", "TAB(o, 0, j) = TAB(o, 0, j) + TAB(o, t1, j);"),
    "no_drive_out": ("if (q < 0) continue; /* redundant row */", "if (1) continue;"),
    "drive_out_positive_only": ("if (fabs(TAB(o, t, j)) > o->eps_p) {", "if (TAB(o, t, j) > o->eps_p) {"),
    "artificials_enter_phase2": ("o->bar = allowed;", "o->bar = np + m;"),
    "no_feasibility_check": ("if (w < -OR_FEAS_TOL * o->feas_scale) {", "if (w < -1e300) {"),
    "no_row_swap": ("TAB(o, 0, j) = TAB(o, m + 1, j);\n        TAB(o, m + 1, j) = v;", "(void)v;"),
    "dual_sign_ignored": ("y[o->perm[t - 1]] = o->sign[t - 1] == 1.0 ? v : -v;", "y[o->perm[t - 1]] = v;"),
    "carried_cost_sign": ("for (int j = 0; j < n; ++j) TAB(o, M, j) = -c[j];",
                          "for (int j = 0; j < n; ++j) TAB(o, M, j) = c[j];"),
    "leaving_bar_ignored": ("if (a > o->eps_p && o->basis[i - 1] < o->bar) {", "if (a > o->eps_p) {"),
    "entering_bar_ignored": ("for (int j = 0; j < o->bar; ++j) {", "for (int j = 0; j < o->n + o->m; ++j) {"),
    "negated_rhs_kept": ("TAB(o, t1, W - 1) = s == 1.0 ? b[k] : -b[k];", "TAB(o, t1, W - 1) = b[k];"),
}


def _general_battery(lib):
    """The pins above on a library built from a variant; the first failure or None."""

    def solve(A, b, c, sense):
        return oracle.solve_general(A, b, c, sense, threads=1, library=lib)

    g = solve([[1.0], [1.0]], [1.0, 2.0], [1.0], [LE, GE])
    if g["status"] != oracle.INFEASIBLE:
        return "contradictory rows"
    g = solve([[-1.0]], [-3.0], [1.0], [GE])
    if g["status"] != oracle.OPTIMAL or g["x"].tolist() != [3.0] or g["y"].tolist() != [-1.0]:
        return "negated >= row"
    g = solve([[-1.0, -1.0], [1.0, 0.0]], [0.0, 5.0], [1.0, 1.0], [EQ, LE])
    if g["status"] != oracle.OPTIMAL or g["x"].tolist() != [0.0, 0.0]:
        return "drive-out on a negative entry"
    rng = np.random.default_rng(7)
    eps = Fraction(1, 10**9)
    for t in range(40):
        m, n = int(rng.integers(1, 6)), int(rng.integers(1, 6))
        A, b, c, sense = random_general(rng, m, n)
        g = solve(A, b, c, sense)
        e = exact_general(A, b, c, sense, eps_d=eps, eps_p=eps)
        if oracle.STATUS_NAMES[g["status"]] != e.status or \
                list(zip(g["rows"].tolist(), g["cols"].tolist())) != e.log:
            if min(e.near_ties, default=1.0) >= 1e-9:
                return f"exact two-phase {t}"
        if e.status == "OPTIMAL":
            ey = [float(v) for v in e.y()]
            if not np.allclose(g["y"], ey, rtol=1e-9, atol=1e-9) or \
                    abs(g["objective"] - float(e.objective())) > 1e-9 * max(1.0, abs(float(e.objective()))):
                return f"exact two-phase solution {t}"
    return None


def test_planted_mistakes_are_caught():
    src = open(SRC).read()
    assert _general_battery(None) is None
    with tempfile.TemporaryDirectory() as d:
        for name, (old, new) in MUTANTS.items():
            assert src.count(old) == 1, name
            path = os.path.join(d, f"{name}.c")
            with open(path, "w") as f:
                f.write(src.replace(old, new))
            lib = oracle.build(src=path, out=os.path.join(d, f"{name}.so"))
            assert _general_battery(lib) is not None, f"mutant {name} survived"
