"""Exact-rational references used to pin the CPU oracle (tests only).

Both work in Python `fractions.Fraction`, so they carry no rounding at all:

* `exact_simplex` runs the same full-tableau method (Section III, Table I and
  Steps 1-3) with the same decision rules (most negative row-0 entry, lowest
  index on ties; minimum ratio over rows with a positive pivot-column entry,
  lowest row on ties), but in exact arithmetic. It pins the pivot sequence and
  the tableau values for small LPs.
* `brute_force_optimum` enumerates every basis of [A | I] and keeps the best
  feasible basic solution. It pins the optimum without any simplex logic.
"""

from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np


def _frac_matrix(a):
    return [[Fraction(float(v)) for v in row] for row in np.atleast_2d(a)]


class ExactTableau:
    def __init__(self, A, b, c, eps_d=0.0, eps_p=0.0):
        A = _frac_matrix(A)
        m, n = len(A), len(A[0])
        b = [Fraction(float(v)) for v in b]
        c = [Fraction(float(v)) for v in c]
        self.m, self.n, self.W = m, n, n + m + 1
        W = self.W
        T = [[Fraction(0)] * W for _ in range(m + 1)]
        for j in range(n):
            T[0][j] = -c[j]
        for i in range(1, m + 1):
            for j in range(n):
                T[i][j] = A[i - 1][j]
            T[i][n + i - 1] = Fraction(1)
            T[i][W - 1] = b[i - 1]
        self.T = T
        self.basis = [n + i for i in range(m)]
        self.eps_d = Fraction(eps_d)
        self.eps_p = Fraction(eps_p)
        self.log = []
        self.status = None
        # smallest relative gaps between the winner and the runner-up of every
        # decision; a gap below 1e-9 flags a near-tie that binary64 may flip.
        self.near_ties = []

    def entering(self):
        row0 = self.T[0][: self.n + self.m]
        order = sorted(range(len(row0)), key=lambda j: (row0[j], j))
        q = order[0]
        if not row0[q] < -self.eps_d:
            return None
        if len(order) > 1:
            a, b = row0[order[0]], row0[order[1]]
            if a != b:
                gap = abs(b - a) / max(abs(a), abs(b), Fraction(1))
                self.near_ties.append(float(gap))
            else:
                self.exact_ties += 1  # broken by the lower index; binary64 may see a rounding apart
        return q

    def leaving(self, q):
        W = self.W
        cand = []
        for i in range(1, self.m + 1):
            a = self.T[i][q]
            if a > self.eps_p:
                cand.append((self.T[i][W - 1] / a, i))
        if not cand:
            return None
        cand.sort()
        if len(cand) > 1 and cand[0][0] != cand[1][0]:
            a, b = cand[0][0], cand[1][0]
            self.near_ties.append(float(abs(b - a) / max(abs(a), abs(b), Fraction(1))))
        elif len(cand) > 1 and cand[0][0] != 0:
            # an exact tie of two nonzero ratios, broken by the lower row;
            # binary64 may see them a rounding apart (a zero ratio, 0 / a,
            # is exact on both sides)
            self.exact_ties += 1
        return cand[0][1]

    exact_ties = 0

    def pivot(self, r, q):
        T, W = self.T, self.W
        p = T[r][q]
        F = [T[i][q] for i in range(self.m + 1)]
        R = [T[r][j] / p for j in range(W)]
        for i in range(self.m + 1):
            if i == r:
                T[i] = list(R)
            else:
                T[i] = [T[i][j] - F[i] * R[j] for j in range(W)]
        self.basis[r - 1] = q
        self.log.append((r, q))

    # The anti-cycling fallback: after `bland_after` degenerate pivots in a
    # row (ratio <= 0), Bland's rule (lowest eligible column; among the rows
    # with the smallest ratio, the lowest basic variable) until a pivot that
    # is not degenerate.
    bland_after = 0
    degen_run = 0

    def bland(self):
        return self.bland_after > 0 and self.degen_run >= self.bland_after

    def entering_bland(self, limit):
        for j in range(limit):
            if self.T[0][j] < -self.eps_d:
                return j
        return None

    def leaving_bland(self, q, bar):
        W = self.W
        cand = [(self.T[i][W - 1] / self.T[i][q], self.basis[i - 1], i) for i in range(1, self.m + 1)
                if self.T[i][q] > self.eps_p and self.basis[i - 1] < bar]
        if not cand:
            return None
        best = min(cand)
        if sum(1 for v in cand if v[0] == best[0]) > 1 and best[0] != 0:
            # an exact tie that Bland's rule breaks by the basic variable;
            # binary64 may see the two ratios a rounding apart
            self.exact_ties += 1
        return best[2]

    def step_rules(self, limit, bar):
        """(q, r) of the next pivot under the rule in force; None parts end."""
        if self.bland():
            q = self.entering_bland(limit)
            return q, (None if q is None else self.leaving_bland(q, bar))
        q = self.entering()
        return q, (None if q is None else self.leaving(q))

    def count(self, r, q):
        theta = self.T[r][self.W - 1] / self.T[r][q]
        if self.bland_after and theta != 0 and abs(theta - self.eps_p) <= Fraction(1, 10**6) * self.eps_p:
            self.near_ties.append(float(abs(theta - self.eps_p) / self.eps_p))  # at the degeneracy threshold
        self.degen_run = self.degen_run + 1 if theta <= self.eps_p else 0

    def solve(self, max_pivots=10_000):
        while True:
            q, r = self.step_rules(self.n + self.m, self.n + self.m)
            if q is None:
                self.status = "OPTIMAL"
                return self
            if r is None:
                self.status = "UNBOUNDED"
                return self
            if len(self.log) >= max_pivots:
                self.status = "ITER_LIMIT"
                return self
            self.count(r, q)
            self.pivot(r, q)

    def objective(self):
        return self.T[0][self.W - 1]


def exact_simplex(A, b, c, eps_d=0.0, eps_p=0.0, max_pivots=10_000, bland_after=0):
    t = ExactTableau(A, b, c, eps_d, eps_p)
    t.bland_after = bland_after
    return t.solve(max_pivots)


def _solve_exact(M, rhs):
    """Gauss-Jordan in Fractions; returns None when M is singular."""
    k = len(M)
    aug = [list(M[i]) + [rhs[i]] for i in range(k)]
    for col in range(k):
        piv = next((i for i in range(col, k) if aug[i][col] != 0), None)
        if piv is None:
            return None
        aug[col], aug[piv] = aug[piv], aug[col]
        pv = aug[col][col]
        aug[col] = [v / pv for v in aug[col]]
        for i in range(k):
            if i != col and aug[i][col] != 0:
                f = aug[i][col]
                aug[i] = [a - f * bb for a, bb in zip(aug[i], aug[col])]
    return [aug[i][k] for i in range(k)]


def brute_force_optimum(A, b, c):
    """Best objective over all basic feasible solutions of [A | I] z = b, z >= 0.

    Returns (objective, x) as Fractions, or (None, None) when no basis is
    feasible. The caller must know the LP is bounded (e.g. A > 0).
    """
    A = _frac_matrix(A)
    m, n = len(A), len(A[0])
    b = [Fraction(float(v)) for v in b]
    c = [Fraction(float(v)) for v in c] + [Fraction(0)] * m
    cols = [[A[i][j] for i in range(m)] for j in range(n)]
    cols += [[Fraction(1) if i == j else Fraction(0) for i in range(m)] for j in range(m)]
    best, best_x = None, None
    for S in itertools.combinations(range(n + m), m):
        M = [[cols[j][i] for j in S] for i in range(m)]
        z = _solve_exact(M, b)
        if z is None or any(v < 0 for v in z):
            continue
        obj = sum(c[j] * v for j, v in zip(S, z))
        if best is None or obj > best:
            best = obj
            x = [Fraction(0)] * n
            for j, v in zip(S, z):
                if j < n:
                    x[j] = v
            best_x = x
    return best, best_x


# ---------------------------------------------------------------- general form

LE, GE, EQ = 0, 1, 2


class ExactGeneral(ExactTableau):
    """The two-phase method for rows <=, >= or = (any sign of b) in exact
    arithmetic, with the construction and decision rules of the oracle's
    general form: rows with b < 0 negated (<= and >= swap); tableau rows
    ordered <=, >=, =; surplus columns for >= rows; one identity column per
    row (slack or artificial) plus one for the carried objective row m+1;
    Phase I maximises minus the sum of the artificial variables; after it,
    artificial variables still basic are driven out on the lowest
    non-artificial column with |entry| > eps_p; Phase II runs on the carried
    objective with artificial columns barred."""

    def __init__(self, A, b, c, sense, eps_d=0.0, eps_p=0.0, feas_tol=Fraction(1, 10**9)):
        A = _frac_matrix(A)
        m, n = len(A), len(A[0])
        b = [Fraction(float(v)) for v in b]
        c = [Fraction(float(v)) for v in c]
        kinds = []
        for i in range(m):
            k = int(sense[i])
            if b[i] < 0 and k != EQ:
                k = GE if k == LE else LE
            kinds.append(k)
        order = [i for want in (LE, GE, EQ) for i in range(m) if kinds[i] == want]
        self.n_le = sum(k == LE for k in kinds)
        n_ge = sum(k == GE for k in kinds)
        self.m_in, self.n_in = m, n
        self.perm = order
        self.sgn = [Fraction(-1) if b[i] < 0 else Fraction(1) for i in order]
        np_ = n + n_ge
        self.nprime = np_
        M = m + 1
        self.m, self.n, self.W = M, np_, np_ + M + 1
        W = self.W
        T = [[Fraction(0)] * W for _ in range(M + 1)]
        surplus = n
        for t, i in enumerate(order, start=1):
            s = self.sgn[t - 1]
            for j in range(n):
                T[t][j] = s * A[i][j]
            if kinds[i] == GE:
                T[t][surplus] = Fraction(-1)
                surplus += 1
            T[t][np_ + t - 1] = Fraction(1)
            T[t][W - 1] = s * b[i]
        for j in range(n):
            T[M][j] = -c[j]
        T[M][np_ + m] = Fraction(1)
        art = range(self.n_le + 1, m + 1)
        T[0] = [Fraction(1) if np_ + self.n_le <= j < np_ + m else Fraction(0) for j in range(W)]
        for t in art:
            T[0] = [T[0][j] - T[t][j] for j in range(W)]
        self.feas_scale = max(Fraction(1), sum((T[t][W - 1] for t in art), Fraction(0)))
        self.feas_tol = feas_tol
        self.T = T
        self.basis = [np_ + t for t in range(M)]
        self.eps_d = Fraction(eps_d)
        self.eps_p = Fraction(eps_p)
        self.log = []
        self.status = None
        self.near_ties = []
        self.bar = np_ + m

    def entering(self):
        row0 = self.T[0][: self.bar]
        order = sorted(range(len(row0)), key=lambda j: (row0[j], j))
        q = order[0]
        if not row0[q] < -self.eps_d:
            return None
        if len(order) > 1 and row0[order[0]] != row0[order[1]]:
            a, b = row0[order[0]], row0[order[1]]
            self.near_ties.append(float(abs(b - a) / max(abs(a), abs(b), Fraction(1))))
        elif len(order) > 1:
            self.exact_ties += 1  # broken by the lower index; binary64 may see a rounding apart
        return q

    def leaving(self, q):
        W = self.W
        cand = [(self.T[i][W - 1] / self.T[i][q], i) for i in range(1, self.m + 1)
                if self.T[i][q] > self.eps_p and self.basis[i - 1] < self.bar]
        if not cand:
            return None
        cand.sort()
        if len(cand) > 1 and cand[0][0] != cand[1][0]:
            a, b = cand[0][0], cand[1][0]
            self.near_ties.append(float(abs(b - a) / max(abs(a), abs(b), Fraction(1))))
        return cand[0][1]

    def _phase(self, max_pivots):
        self.degen_run = 0
        while True:
            q, r = self.step_rules(self.bar, self.bar)
            if q is None:
                return "OPTIMAL"
            if r is None:
                return "UNBOUNDED"
            if len(self.log) >= max_pivots:
                return "ITER_LIMIT"
            self.count(r, q)
            self.pivot(r, q)

    def solve(self, max_pivots=10_000):
        st = self._phase(max_pivots)
        if st != "OPTIMAL":
            self.status = st
            return self
        if self.T[0][self.W - 1] < -self.feas_tol * self.feas_scale:
            self.status = "INFEASIBLE"
            return self
        allowed = self.nprime + self.n_le
        for t in range(1, self.m_in + 1):
            if self.basis[t - 1] < allowed:
                continue
            q = next((j for j in range(allowed) if abs(self.T[t][j]) > self.eps_p), None)
            if q is None:
                continue
            if len(self.log) >= max_pivots:
                self.status = "ITER_LIMIT"
                return self
            self.pivot(t, q)
        M = self.m
        self.T[0], self.T[M] = self.T[M], self.T[0]
        self.bar = allowed
        self.status = self._phase(max_pivots)
        return self

    def x(self):
        x = [Fraction(0)] * self.n_in
        for t in range(1, self.m_in + 1):
            if self.basis[t - 1] < self.n_in:
                x[self.basis[t - 1]] = self.T[t][self.W - 1]
        return x

    def y(self):
        y = [Fraction(0)] * self.m_in
        for t in range(1, self.m_in + 1):
            y[self.perm[t - 1]] = self.sgn[t - 1] * self.T[0][self.nprime + t - 1]
        return y


def exact_general(A, b, c, sense, eps_d=0.0, eps_p=0.0, max_pivots=10_000, bland_after=0):
    t = ExactGeneral(A, b, c, sense, eps_d, eps_p)
    t.bland_after = bland_after
    return t.solve(max_pivots)


def brute_force_general(A, b, c, sense):
    """Best objective over the basic feasible solutions of the equality form
    [A | S] z = b, z >= 0 (S: +e_i for a <= row, -e_i for a >= row, nothing
    for a = row), without any simplex logic. Needs [A | S] of full row rank
    and a bounded LP. Returns (objective, x) as Fractions, or (None, None)
    when no basic solution is feasible (the LP is infeasible)."""
    A = _frac_matrix(A)
    m, n = len(A), len(A[0])
    b = [Fraction(float(v)) for v in b]
    cols = [[A[i][j] for i in range(m)] for j in range(n)]
    for i in range(m):
        if int(sense[i]) != EQ:
            cols.append([Fraction(1 if int(sense[i]) == LE else -1) if k == i else Fraction(0) for k in range(m)])
    cost = [Fraction(float(v)) for v in c] + [Fraction(0)] * (len(cols) - n)
    best, best_x = None, None
    for S in itertools.combinations(range(len(cols)), m):
        Mx = [[cols[j][i] for j in S] for i in range(m)]
        z = _solve_exact(Mx, b)
        if z is None or any(v < 0 for v in z):
            continue
        obj = sum(cost[j] * v for j, v in zip(S, z))
        if best is None or obj > best:
            best = obj
            x = [Fraction(0)] * n
            for j, v in zip(S, z):
                if j < n:
                    x[j] = v
            best_x = x
    return best, best_x
