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
        return cand[0][1]

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

    def solve(self, max_pivots=10_000):
        while True:
            q = self.entering()
            if q is None:
                self.status = "OPTIMAL"
                return self
            r = self.leaving(q)
            if r is None:
                self.status = "UNBOUNDED"
                return self
            if len(self.log) >= max_pivots:
                self.status = "ITER_LIMIT"
                return self
            self.pivot(r, q)

    def objective(self):
        return self.T[0][self.W - 1]


def exact_simplex(A, b, c, eps_d=0.0, eps_p=0.0, max_pivots=10_000):
    return ExactTableau(A, b, c, eps_d, eps_p).solve(max_pivots)


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
