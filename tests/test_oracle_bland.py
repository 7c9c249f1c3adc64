"""Pins of the oracle's anti-cycling fallback (bland_after = k: Bland's rule
after k degenerate pivots in a row, until a pivot that is not degenerate).

* a textbook instance cycles under the plain rule (the cycle re-derived in
  exact rational arithmetic) and reaches its optimum (vertex enumeration,
  HiGHS) with the fallback, for every k;
* an exact-rational run of the same switching rule fixes the pivot sequence
  on degenerate batteries, standard and general form;
* with the fallback off the oracle is bit-identical to the plain method;
* planted mistakes in the fallback are each caught.
"""

import os
import tempfile
from fractions import Fraction

import numpy as np
import pytest

import oracle
from exact_ref import brute_force_optimum, exact_general, exact_simplex
from goldens import read_fixture
from test_oracle_general import random_general


def cycling():
    fx = read_fixture("cycling_example.txt")
    return fx, fx["A"], fx["b"], fx["c"]


def test_the_plain_rule_cycles_on_the_textbook_instance():
    fx, A, b, c = cycling()
    o = oracle.solve(A, b, c, max_pivots=60, threads=1)
    assert o["status"] == oracle.ITER_LIMIT
    log = list(zip(o["rows"].tolist(), o["cols"].tolist()))
    assert log[:6] == fx["pivot"] and log == (fx["pivot"] * 10)[:60]
    e = exact_simplex(A, b, c, max_pivots=12)
    assert e.status == "ITER_LIMIT" and e.log == fx["pivot"] * 2
    # after six pivots the exact tableau is the starting one again
    e6 = exact_simplex(A, b, c, max_pivots=6)
    e0 = exact_simplex(A, b, c, max_pivots=0)
    assert e6.T == e0.T and e6.basis == e0.basis


def test_the_fallback_reaches_the_optimum():
    fx, A, b, c = cycling()
    best, bx = brute_force_optimum(A, b, c)
    assert best == Fraction(1) and [float(v) for v in bx] == fx["x"].tolist()
    scipy_opt = pytest.importorskip("scipy.optimize")
    h = scipy_opt.linprog(-c, A_ub=A, b_ub=b, bounds=(0, None), method="highs")
    assert h.status == 0 and abs(-h.fun - fx["objective"]) < 1e-12
    for k in range(1, 9):
        o = oracle.solve(A, b, c, max_pivots=60, threads=1, bland_after=k)
        assert o["status"] == oracle.OPTIMAL and o["objective"] == fx["objective"], k
        assert o["x"].tolist() == fx["x"].tolist(), k
        e = exact_simplex(A, b, c, bland_after=k)
        assert e.status == "OPTIMAL" and list(zip(o["rows"].tolist(), o["cols"].tolist())) == e.log, k


def degenerate(rng, m, n):
    A = rng.integers(-3, 5, size=(m, n)).astype(float)
    b = np.where(rng.random(m) < 0.6, 0.0, rng.integers(0, 6, size=m).astype(float))
    c = rng.integers(-2, 6, size=n).astype(float)
    return A, b, c


def test_exact_switching_rule_standard_form():
    rng = np.random.default_rng(21)
    eps = Fraction(1, 10**9)
    compared = switched = 0
    for t in range(150):
        m, n = int(rng.integers(2, 9)), int(rng.integers(2, 9))
        A, b, c = degenerate(rng, m, n)
        k = 1 + t % 3
        o = oracle.solve(A, b, c, threads=1, bland_after=k)
        e = exact_simplex(A, b, c, eps_d=eps, eps_p=eps, bland_after=k)
        plain = exact_simplex(A, b, c, eps_d=eps, eps_p=eps)
        if list(zip(o["rows"].tolist(), o["cols"].tolist())) != e.log or oracle.STATUS_NAMES[o["status"]] != e.status:
            assert min(e.near_ties, default=1.0) < 1e-9 or e.exact_ties, t
            continue
        compared += 1
        switched += e.log != plain.log
    assert compared >= 140 and switched >= 20, (compared, switched)


def test_exact_switching_rule_general_form():
    rng = np.random.default_rng(22)
    eps = Fraction(1, 10**9)
    compared = 0
    for t in range(100):
        m, n = int(rng.integers(1, 7)), int(rng.integers(1, 7))
        A, b, c, sense = random_general(rng, m, n)
        b = np.where(rng.random(len(b)) < 0.5, 0.0, b)
        k = 1 + t % 2
        o = oracle.solve_general(A, b, c, sense, threads=1, bland_after=k)
        e = exact_general(A, b, c, sense, eps_d=eps, eps_p=eps, bland_after=k)
        if list(zip(o["rows"].tolist(), o["cols"].tolist())) != e.log or oracle.STATUS_NAMES[o["status"]] != e.status:
            assert min(e.near_ties, default=1.0) < 1e-9 or e.exact_ties, t
            continue
        compared += 1
    assert compared >= 90


def test_off_is_the_plain_method():
    rng = np.random.default_rng(23)
    for t in range(20):
        A, b, c = degenerate(rng, int(rng.integers(2, 30)), int(rng.integers(2, 30)))
        o1 = oracle.solve(A, b, c, threads=2)
        o2 = oracle.solve(A, b, c, threads=2, bland_after=0)
        assert o1["rows"].tolist() == o2["rows"].tolist() and np.array_equal(o1["x"], o2["x"])


def test_terminates_and_agrees_with_highs_on_degenerate_lps():
    scipy_opt = pytest.importorskip("scipy.optimize")
    rng = np.random.default_rng(24)
    for t in range(30):
        m, n = int(rng.integers(5, 40)), int(rng.integers(5, 40))
        A, b, c = degenerate(rng, m, n)
        A = np.vstack([A, np.ones(n)])
        b = np.append(b, 50.0)  # bounded
        o = oracle.solve(A, b, c, threads=2, bland_after=2, max_pivots=5000)
        h = scipy_opt.linprog(-c, A_ub=A, b_ub=b, bounds=(0, None), method="highs")
        assert o["status"] == oracle.OPTIMAL and h.status == 0, t
        assert abs(o["objective"] + h.fun) <= 1e-9 * max(1.0, abs(h.fun)), t


# ---------------------------------------------------------------- planted mistakes

SRC = os.path.join(os.path.dirname(oracle.__file__), "tableau_simplex.c")

MUTANTS = {
    "entering_most_negative": ("if (q < 0 && v < -o->eps_d) q = j;", "if (v < -o->eps_d && (q < 0 || v < TAB(o, 0, q))) q = j;"),
    "leaving_tie_by_row": ("(ratio == best && o->basis[i - 1] < o->basis[r - 1])", "(0)"),
    "zero_step_not_degenerate": ("o->degen_run = theta <= o->eps_p ? o->degen_run + 1 : 0;",
                                 "o->degen_run = theta < 0.0 ? o->degen_run + 1 : 0;"),
    "count_never_reset": ("o->degen_run = theta <= o->eps_p ? o->degen_run + 1 : 0;",
                          "o->degen_run = theta <= o->eps_p ? o->degen_run + 1 : o->degen_run;"),
    "switch_off_by_one": ("return o->bland_after > 0 && o->degen_run >= o->bland_after;",
                          "return o->bland_after > 0 && o->degen_run > o->bland_after;"),
}


def _battery(lib):
    fx, A, b, c = cycling()
    for k in (1, 3, 5):
        o = oracle.solve(A, b, c, max_pivots=60, threads=1, bland_after=k, library=lib)
        e = exact_simplex(A, b, c, bland_after=k)
        if o["status"] != oracle.OPTIMAL or list(zip(o["rows"].tolist(), o["cols"].tolist())) != e.log:
            return f"cycling example k={k}"
    rng = np.random.default_rng(25)
    eps = Fraction(1, 10**9)
    for t in range(160):
        A, b, c = degenerate(rng, int(rng.integers(3, 12)), int(rng.integers(3, 12)))
        k = 1 + t % 2
        o = oracle.solve(A, b, c, threads=1, bland_after=k, library=lib)
        e = exact_simplex(A, b, c, eps_d=eps, eps_p=eps, bland_after=k)
        if list(zip(o["rows"].tolist(), o["cols"].tolist())) != e.log and min(e.near_ties, default=1.0) >= 1e-9 \
                and not e.exact_ties:
            return f"exact switching {t}"
    return None


def test_planted_mistakes_are_caught():
    src = open(SRC).read()
    assert _battery(None) is None
    with tempfile.TemporaryDirectory() as d:
        for name, (old, new) in MUTANTS.items():
            assert src.count(old) == 1, name
            path = os.path.join(d, f"{name}.c")
            with open(path, "w") as f:
                f.write(src.replace(old, new))
            lib = oracle.build(src=path, out=os.path.join(d, f"{name}.so"))
            assert _battery(lib) is not None, f"mutant {name} survived"
