"""Optimality certificates of a returned solution, from the original data.

A primal-dual pair (x, y) of max c^T x s.t. Ax <= b, x >= 0 is optimal when x
is primal feasible, y is dual feasible (A^T y >= c, y >= 0) and the objectives
agree (c^T x = b^T y, strong duality). The check is independent of how the
solution was found; it uses only A, b, c and the returned x, y and objective.
Each residual is scaled by the magnitude of the terms it compares.
"""

from __future__ import annotations

import numpy as np


def residuals(A, b, c, x, y, objective):
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    out = {}
    lhs = A @ x
    mag = np.abs(A) @ np.abs(x)
    out["primal"] = float(np.max((lhs - b) / np.maximum(1.0, np.maximum(np.abs(b), mag)), initial=0.0))
    out["x_sign"] = float(max(0.0, -float(x.min(initial=0.0))) / max(1.0, float(np.abs(x).max(initial=0.0))))
    red = A.T @ y
    magd = np.abs(A).T @ np.abs(y)
    out["dual"] = float(np.max((c - red) / np.maximum(1.0, np.maximum(np.abs(c), magd)), initial=0.0))
    out["y_sign"] = float(max(0.0, -float(y.min(initial=0.0))) / max(1.0, float(np.abs(y).max(initial=0.0))))
    px, dy = float(c @ x), float(b @ y)
    out["gap"] = abs(px - dy) / max(1.0, abs(px))
    out["objective"] = abs(float(objective) - px) / max(1.0, abs(px))
    return out


def certify(A, b, c, x, y, objective, tol=1e-9):
    """Returns (ok, residuals); ok when every scaled residual is <= tol."""
    r = residuals(A, b, c, x, y, objective)
    return all(v <= tol for v in r.values()), r
