"""Exact active-set enumeration for small instances (test infrastructure only).

An independent pin of the optimum W* of paper eq. 1-3 (single-period) and eq. 4-6
(multi-period), built only from the problem's definition: Sigma = F Omega F^T +
diag(delta^2) is formed explicitly, and nothing here uses the oracle's splitting, dual,
prox maps, PDHG or polish.

The objective, in the oracle's scaled minimisation form (the paper's objective divided by
-GMV, g1 = lambda1 GMV, g2 = lambda2, g3 = lambda3), is

    Phi(W) = sum_t [ -a_t^T w_t + g1 (w_t - c)^T Sigma (w_t - c) ]
             + sum_k [ g2 s_k |u_k| + g3 q_k |u_k|^d ],      u = D vec(W) + e,

subject to L <= A w_t <= U and ||w_t||_1 <= 1 (c = 0 single-period, w_T multi-period;
u_k runs over the trades w_t - w_{t-1}, t = 1..T', with w_0 and w_T fixed).

Every point of the feasible set lies on a piece fixed by
* a sign state tau_k in {-1, 0, +1} for every trade (0: u_k = 0),
* per period, the budget slack or tight and, when tight, a sign state omega_ti in
  {-1, 0, +1} for every weight (0: w_ti = 0),
* a state in {lower, free, upper} for every exposure row of every period (a row with
  L = U is always active).
On a piece the objective is smooth (|u_k| = tau_k u_k, |w_ti| = omega_ti w_ti) and the
piece's zero states and active bounds are equality constraints, so its minimiser solves
the equality-constrained KKT system

    grad f(x) + E^T nu = 0,    E x = r.

At d = 2 the system is linear and solved directly; otherwise it is solved by Newton's
method on the same system.  The piece's solution is the optimum of the whole problem iff
it satisfies the optimality conditions of the original nonsmooth problem (convexity makes
them sufficient, and strict convexity makes W* unique):
* free trades keep their sign (tau_k u_k >= 0), free weights theirs (omega w >= 0);
* a zero trade's multiplier lies in [-g2 s_k, g2 s_k] (the subdifferential of the
  spread term at 0);
* a tight budget's multiplier mu_t >= 0, and a zero weight's multiplier lies in
  [-mu_t, mu_t] (the subdifferential of mu_t |w| at 0);
* an upper-active row has a nonnegative multiplier, a lower-active one a nonpositive one
  (Lagrangian f + nu (A_j w - bound)), a free row lies within its bounds;
* a slack budget has ||w_t||_1 <= 1.
The function enumerates every piece (slack budgets first; tight ones only when no slack
piece is consistent, skipping the combinations that contradict the fixed end points w_0
and w_T), solves each, and returns the consistent solution together with the number of
consistent pieces and the spread of their solutions (degenerate problems, with a
multiplier exactly at its limit, have several pieces with the same W*).  Cost: 3^(T' n)
trade states times the row and budget states, so up to n = 8 single-period with a slack
budget, n = 5 with a tight one, and two-decision multi-period problems of two assets.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

__all__ = ["EnumResult", "active_set_enumeration"]


@dataclass
class EnumResult:
    W: np.ndarray          # (P, n) the optimum
    phi: float             # its scaled objective
    pieces: int            # pieces solved
    consistent: int        # pieces whose solution met every optimality condition
    spread: float          # max |W_piece - W| over the consistent pieces
    budget_tight: tuple    # per period, whether the optimum's budget is tight


def _data(inst):
    T = int(inst.get("T", 0) or 0)
    alpha = np.atleast_2d(np.asarray(inst["alpha"], dtype=np.float64))
    P, n = alpha.shape
    Tp = 1 if T == 0 else T
    F = np.asarray(inst["F"], dtype=np.float64).reshape(n, -1)
    Om = np.asarray(inst["Omega"], dtype=np.float64)
    Sigma = F @ Om @ F.T + np.diag(np.asarray(inst["delta"], dtype=np.float64) ** 2)
    g1 = float(inst["lambda1"]) * float(inst["GMV"])
    s = np.atleast_2d(np.asarray(inst["s"], dtype=np.float64)).reshape(-1) * float(inst["lambda2"])
    q = np.atleast_2d(np.asarray(inst["q"], dtype=np.float64)).reshape(-1) * float(inst["lambda3"])
    A = np.asarray(inst["A"], dtype=np.float64).reshape(-1, n)
    L = np.asarray(inst["L"], dtype=np.float64).reshape(-1)
    U = np.asarray(inst["U"], dtype=np.float64).reshape(-1)
    w0 = np.asarray(inst["w0"], dtype=np.float64)
    wT = np.asarray(inst["w_target"], dtype=np.float64) if T else None
    nv, nt = P * n, Tp * n
    # trades u = D x + e, x = vec(W) (period-major)
    D = np.zeros((nt, nv))
    e = np.zeros(nt)
    I = np.eye(n)
    if T == 0:
        D[:, :] = I
        e[:] = -w0
    else:
        for t in range(Tp):
            if t < P:
                D[t * n:(t + 1) * n, t * n:(t + 1) * n] += I
            if t >= 1:
                D[t * n:(t + 1) * n, (t - 1) * n:t * n] -= I
        e[:n] = -w0
        e[P * n:] = wT
    c = np.zeros(n) if T == 0 else wT
    return dict(P=P, n=n, nv=nv, nt=nt, alpha=alpha.reshape(-1), Sigma=Sigma, g1=g1, s=s, q=q,
                d=float(inst["d"]), A=A, L=L, U=U, D=D, e=e, c=c)


def _objective(dd, x):
    P, n = dd["P"], dd["n"]
    val = -dd["alpha"] @ x
    for t in range(P):
        xc = x[t * n:(t + 1) * n] - dd["c"]
        val += dd["g1"] * xc @ dd["Sigma"] @ xc
    u = dd["D"] @ x + dd["e"]
    return float(val + np.sum(dd["s"] * np.abs(u) + dd["q"] * np.abs(u) ** dd["d"]))


def _solve_piece(dd, tau, rows_eq, rhs_eq):
    """Minimiser of the piece's objective, with |u_k| written as tau_k u_k for the free
    trades (zero trades and the other zero states are the equality rows), subject to
    rows_eq x = rhs_eq.  Returns (x, nu) or None when the rows are dependent.

    The function minimised, f(x) = sum_t[-a_t^T w_t + g1 (w_t - c)^T Sigma (w_t - c)]
    + sum_free [g2 s_k tau_k u_k + g3 q_k |u_k|^d], is convex on the whole space and equals
    Phi on the piece's sign region, so its constrained minimiser is the optimum whenever
    the piece is the optimum's (the optimality conditions coincide)."""
    P, n, nv, d = dd["P"], dd["n"], dd["nv"], dd["d"]
    D, e, q, s = dd["D"], dd["e"], dd["q"], dd["s"]
    free = tau != 0
    E = np.asarray(rows_eq, dtype=np.float64).reshape(-1, nv)
    r = np.asarray(rhs_eq, dtype=np.float64).reshape(-1)
    ne = E.shape[0]
    if ne > nv or (ne and np.linalg.matrix_rank(E) < ne):
        return None
    Hr = np.zeros((nv, nv))
    g0 = -dd["alpha"].copy()
    for t in range(P):
        Hr[t * n:(t + 1) * n, t * n:(t + 1) * n] = 2.0 * dd["g1"] * dd["Sigma"]
        g0[t * n:(t + 1) * n] -= 2.0 * dd["g1"] * dd["Sigma"] @ dd["c"]
    Df, ef, qf = D[free], e[free], q[free]
    g0 = g0 + Df.T @ (s[free] * tau[free])

    def kkt_step(H, g, rr):
        M = np.zeros((nv + ne, nv + ne))
        M[:nv, :nv] = H
        M[:nv, nv:] = E.T
        M[nv:, :nv] = E
        sol = np.linalg.solve(M, np.concatenate([-g, rr]))
        return sol[:nv], sol[nv:]

    # d = 2: one linear solve.  Otherwise the same solve is the starting point (it meets
    # the equality rows) and Newton steps follow, with a backtracking line search on f.
    H2 = Hr + 2.0 * (Df.T * qf) @ Df
    x, nu = kkt_step(H2, g0 + 2.0 * Df.T @ (qf * ef), r)
    if d == 2.0:
        return x, nu

    def fval(x):
        u = Df @ x + ef
        return 0.5 * x @ Hr @ x + g0 @ x + float(np.sum(qf * np.abs(u) ** d))

    def grad(x):
        u = Df @ x + ef
        return Hr @ x + g0 + Df.T @ (qf * d * np.sign(u) * np.abs(u) ** (d - 1.0))

    for _ in range(200):
        u = Df @ x + ef
        curv = qf * d * (d - 1.0) * np.maximum(np.abs(u), 1e-14) ** (d - 2.0)
        g = grad(x)
        dx, _ = kkt_step(Hr + (Df.T * curv) @ Df, g, np.zeros(ne))
        f0, slope = fval(x), float(g @ dx)
        if slope >= 0.0:
            break
        step = 1.0
        while step > 1e-14 and fval(x + step * dx) > f0 + 1e-4 * step * slope:
            step *= 0.5
        x = x + step * dx
        if np.max(np.abs(step * dx)) <= 1e-16 * max(1.0, float(np.max(np.abs(x)))):
            break
    g = grad(x)
    if ne:
        nu = np.linalg.lstsq(E.T, -g, rcond=None)[0]
        res = np.max(np.abs(E.T @ nu + g))
    else:
        nu = np.zeros(0)
        res = float(np.max(np.abs(g)))
    # a stationary point of the convex piece problem, or none found
    if res > 1e-9 * max(1e-3, float(np.max(np.abs(g0)))):
        return None
    return x, nu


def active_set_enumeration(inst: dict, tol: float = 1e-10, max_pieces: int = 200000) -> EnumResult:
    dd = _data(inst)
    P, n, nv, nt = dd["P"], dd["n"], dd["nv"], dd["nt"]
    A, L, U, D, e, s = dd["A"], dd["L"], dd["U"], dd["D"], dd["e"], dd["s"]
    m = A.shape[0]
    scale = 1.0   # weights are O(1) by the budget

    def row_states(j):
        if L[j] == U[j]:
            return (2,)                      # equality row: always active
        st = [0]
        if np.isfinite(L[j]):
            st.append(-1)
        if np.isfinite(U[j]):
            st.append(1)
        return tuple(st)

    row_choices = [row_states(j) for _ in range(P) for j in range(m)]

    def pieces(tight_allowed):
        budget_opts = (0, 1) if tight_allowed else (0,)
        for tau in itertools.product((-1, 0, 1), repeat=nt):
            for bud in itertools.product(budget_opts, repeat=P):
                omega_sets = [itertools.product((-1, 0, 1), repeat=n) if b else [None] for b in bud]
                for om in itertools.product(*[list(o) for o in omega_sets]):
                    for rs in itertools.product(*row_choices):
                        yield np.array(tau), bud, om, rs

    T = P + 1 if nt > n else 0
    w0 = -e[:n]
    wT = e[P * n:] if T else None

    def admissible(tau, bud, om):
        """Combinations that contradict the fixed end points are skipped without a solve:
        a zero first trade fixes w_1 = w_0 (so its sign), a zero weight in period 1 fixes
        the first trade to -w_0; likewise the last trade against w_T."""
        for i in range(n):
            if bud[0]:
                o = om[0][i]
                if tau[i] == 0 and o != np.sign(w0[i]):
                    return False
                if o == 0 and tau[i] != -np.sign(w0[i]):
                    return False
            if T and bud[P - 1]:
                o = om[P - 1][i]
                k = P * n + i
                if tau[k] == 0 and o != np.sign(wT[i]):
                    return False
                if o == 0 and tau[k] != np.sign(wT[i]):
                    return False
        return True

    count = consistent = 0
    sols = []
    for tight_allowed in (False, True):
        for tau, bud, om, rs in pieces(tight_allowed):
            if tight_allowed and not any(bud):
                continue   # slack pieces were done in the first pass
            if tight_allowed and not admissible(tau, bud, om):
                continue
            count += 1
            if count > max_pieces:
                raise ValueError("instance too large for the enumeration")
            rows, rhs, kinds = [], [], []
            for k in np.nonzero(tau == 0)[0]:
                rows.append(D[k]); rhs.append(-e[k]); kinds.append(("trade", k))
            for t in range(P):
                if bud[t]:
                    sg = np.array(om[t], dtype=np.float64)
                    for i in np.nonzero(sg == 0)[0]:
                        r = np.zeros(nv); r[t * n + i] = 1.0
                        rows.append(r); rhs.append(0.0); kinds.append(("zero_w", t))
                    r = np.zeros(nv); r[t * n:(t + 1) * n] = sg
                    rows.append(r); rhs.append(1.0); kinds.append(("budget", t))
                for j in range(m):
                    stj = rs[t * m + j]
                    if stj != 0:
                        r = np.zeros(nv); r[t * n:(t + 1) * n] = A[j]
                        rows.append(r)
                        rhs.append(U[j] if stj in (1, 2) else L[j])
                        kinds.append(("row", stj))
            res = _solve_piece(dd, tau, rows, rhs)
            if res is None:
                continue
            x, nu = res
            W = x.reshape(P, n)
            u = D @ x + e
            ok = bool(np.all(tau[tau != 0] * u[tau != 0] >= -tol * scale))
            bmu = {}
            for (kind, a), v in zip(kinds, nu):
                if kind == "budget":
                    bmu[a] = v
            for (kind, a), v in zip(kinds, nu):
                if not ok:
                    break
                if kind == "trade":
                    ok = abs(v) <= s[a] * (1.0 + 1e-9) + tol
                elif kind == "budget":
                    ok = v >= -tol
                elif kind == "zero_w":
                    ok = abs(v) <= bmu[a] * (1.0 + 1e-9) + tol
                elif kind == "row":
                    ok = (a == 2) or (a == 1 and v >= -tol) or (a == -1 and v <= tol)
            for t in range(P):
                if not ok:
                    break
                if bud[t]:
                    sg = np.array(om[t], dtype=np.float64)
                    ok = bool(np.all(sg * W[t] >= -tol * scale))
                else:
                    ok = np.abs(W[t]).sum() <= 1.0 + tol
                if ok and m:
                    aw = A @ W[t]
                    ok = bool(np.all(aw >= L - tol) and np.all(aw <= U + tol))
            if not ok:
                continue
            consistent += 1
            sols.append((W.copy(), tuple(bool(b) for b in bud)))
        if sols:
            break
    if not sols:
        raise RuntimeError("no piece satisfies the optimality conditions")
    W, bt = sols[0]
    spread = max(float(np.max(np.abs(Wi - W))) for Wi, _ in sols)
    return EnumResult(W=W, phi=_objective(dd, W.reshape(-1)), pieces=count, consistent=consistent,
                      spread=spread, budget_tight=bt)
