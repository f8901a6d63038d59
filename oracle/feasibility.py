"""Feasibility of the constraint set and infeasibility certificates (plain FP64; test
infrastructure only).

Every decision period of the single-period (paper Section 2.1, eq. 2-3) and
multi-period (Section 2.2, eq. 5-6) models has the same feasible set

    X = { w : L <= A w <= U,  ||w||_1 <= 1 }.

min_budget() returns min { ||w||_1 : L <= A w <= U } by linear programming (HiGHS), so X
is empty exactly when that minimum exceeds 1 (or the box alone is empty).

certificate_value(y) = sum_j max(U_j y_j, L_j y_j) + ||A^T y||_inf.  For any w in X,
y^T A w <= sum_j max(U_j y_j, L_j y_j) (the box) and y^T A w >= -||A^T y||_inf ||w||_1
>= -||A^T y||_inf (the budget), so a negative value for some y proves X empty; by LP
duality such a y exists whenever X is empty.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import linprog

__all__ = ["min_budget", "certificate_value", "is_feasible"]


def _box(inst):
    A = np.asarray(inst["A"], dtype=np.float64)
    n = np.atleast_2d(np.asarray(inst["alpha"])).shape[1]
    A = A.reshape(-1, n)
    L = np.asarray(inst["L"], dtype=np.float64).reshape(A.shape[0])
    U = np.asarray(inst["U"], dtype=np.float64).reshape(A.shape[0])
    return A, L, U


def min_budget(inst: dict) -> float:
    """min ||w||_1 subject to L <= A w <= U (inf if the box is empty)."""
    A, L, U = _box(inst)
    m, n = A.shape
    if m == 0:
        return 0.0
    # w = p - r with p, r >= 0; minimise sum(p + r)
    c = np.ones(2 * n)
    AA = np.hstack([A, -A])
    rows, rhs = [], []
    for j in range(m):
        if np.isfinite(U[j]):
            rows.append(AA[j]); rhs.append(U[j])
        if np.isfinite(L[j]):
            rows.append(-AA[j]); rhs.append(-L[j])
    if not rows:
        return 0.0
    res = linprog(c, A_ub=np.array(rows), b_ub=np.array(rhs), bounds=[(0, None)] * (2 * n), method="highs")
    if res.status == 2:
        return float("inf")
    if res.status != 0:
        raise RuntimeError(f"linprog failed: {res.message}")
    return float(res.fun)


def certificate_value(inst: dict, y) -> float:
    """sum_j max(U_j y_j, L_j y_j) + ||A^T y||_inf, with 0 * inf = 0."""
    A, L, U = _box(inst)
    y = np.asarray(y, dtype=np.float64).reshape(A.shape[0])
    sup = 0.0
    for j in range(A.shape[0]):
        if y[j] > 0:
            sup += U[j] * y[j]
        elif y[j] < 0:
            sup += L[j] * y[j]
    return float(sup + (np.abs(A.T @ y).max() if A.shape[0] else 0.0))


def is_feasible(inst: dict, slack: float = 1e-9) -> bool:
    return min_budget(inst) <= 1.0 + slack
