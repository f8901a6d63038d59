"""Reference gradient of a loss of the optimal weights (plain FP64, dense; test
infrastructure only).

For a loss l(W*) of the solution W*(theta) of the paper's single- or multi-period
problem (Section 2, eq. 1-6, risk model of Section 3.2), with theta one of the expected
returns a_t, the spread coefficients s_t or the factor loadings F (A, L, U, Omega held
fixed), this module applies the implicit function theorem to the optimality conditions
of the smooth piece that contains W*:

* trades u_ti = w_ti - w_{t-1,i} that are zero at W* stay zero (the spread term's kink),
* weights that are zero in a period whose budget ||w_t||_1 <= 1 is tight stay zero,
* exposure rows at a bound stay there, tight budgets stay tight with the signs of W*.

On that piece Phi is twice differentiable; with E W = e collecting the equalities above,
the conditions grad Phi(W) + E^T nu = 0, E W = e give, for a change of theta,
[H E^T; E 0] [dW; dnu] = -[d_theta grad Phi; 0].  One symmetric solve with the
right-hand side (dl/dW, 0) yields lambda, and dl/dtheta = -lambda^T d_theta grad Phi:

* alpha_ti enters grad Phi as -alpha_ti:                 dl/dalpha = lambda;
* s_ti enters through g2 s_ti sign(u_ti) on a nonzero trade, pushing w_t and pulling
  w_{t-1}:                                               dl/ds_ti = -g2 sign(u_ti) (lambda_ti - lambda_{t-1,i});
* F enters the risk term g1 (w_t - c)^T (F Omega F^T + diag(delta^2)) (w_t - c):
                                                         dl/dF = -2 g1 sum_t [lambda_t x_t^T + x_t lambda_t^T] F Omega,
  x_t = w_t - c (Omega symmetric).

The matrix is dense in the P*n weights (the factor term couples all assets), so this is
meant for the small instances of the tests.  The pieces are read off the certified
oracle solution with relative thresholds; a directional central difference of the
oracle's own solve pins the result.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .problem import Problem, normalize, trades
from .solve import solve

__all__ = ["reference_gradient", "Gradient", "piece_of"]


@dataclass
class Gradient:
    alpha: np.ndarray    # (P, n)
    s: np.ndarray        # (T', n)
    F: np.ndarray        # (n, k)
    W: np.ndarray        # (P, n) the solution the gradient is taken at
    loss: float


@dataclass
class Piece:
    zero_trade: np.ndarray   # (T', n) bool
    sgn_u: np.ndarray        # (T', n)
    tight: np.ndarray        # (P,) bool
    zero_w: np.ndarray       # (P, n) bool (only in tight periods)
    sgn_w: np.ndarray        # (P, n)
    rows: list               # per period: (row indices, bound values)


def piece_of(pb: Problem, W: np.ndarray, eps: float = 1e-9) -> Piece:
    """Active pieces of a (certified) solution, thresholds relative to max |W|."""
    W = np.atleast_2d(W)
    scale = max(1e-300, float(np.abs(W).max()))
    U = trades(pb, W)
    zero_trade = np.abs(U) <= eps * scale
    sgn_u = np.where(zero_trade, 0.0, np.sign(U))
    tight = np.abs(W).sum(axis=1) >= 1.0 - 1e-9
    zero_w = (np.abs(W) <= eps * scale) & tight[:, None]
    sgn_w = np.where(zero_w, 0.0, np.sign(W))
    rows = []
    for t in range(pb.P):
        aw = pb.A @ W[t]
        span = np.where(np.isfinite(pb.U - pb.L), np.maximum(pb.U - pb.L, 0.0), 1.0)
        tol = 1e-9 * np.maximum(1.0, span)
        at_u = np.isfinite(pb.U) & (pb.U - aw <= tol)
        at_l = np.isfinite(pb.L) & (aw - pb.L <= tol) & ~at_u
        idx = np.nonzero(at_u | at_l)[0]
        rows.append((idx, np.where(at_u[idx], pb.U[idx], pb.L[idx])))
    return Piece(zero_trade, sgn_u, tight, zero_w, sgn_w, rows)


def _index(pb: Problem):
    """Flat index of w_ti, and the left / right decision of trade t (-1 = w_0, P = w_T)."""
    return lambda t, i: t * pb.n + i


def _system(pb: Problem, W: np.ndarray, pc: Piece):
    """H (P n x P n) and the equality rows E (list of dense rows over the P n weights)."""
    P, n = pb.P, pb.n
    N = P * n
    ix = _index(pb)
    Sigma = pb.G @ pb.G.T + np.diag(pb.delta2)
    H = np.zeros((N, N))
    for t in range(P):
        H[t * n:(t + 1) * n, t * n:(t + 1) * n] += 2.0 * pb.g1 * Sigma
    U = trades(pb, W)
    E = []
    for t in range(pb.Tp):
        left, right = t - 1, t          # trade t moves w_{t-1} (or w_0) to w_t (or w_T)
        for i in range(n):
            lv = ix(left, i) if 0 <= left < P else None
            rv = ix(right, i) if 0 <= right < P else None
            if pc.zero_trade[t, i]:
                row = np.zeros(N)
                if rv is not None:
                    row[rv] += 1.0
                if lv is not None:
                    row[lv] -= 1.0
                if row.any():
                    E.append(row)
            else:
                au = abs(U[t, i])
                curv = pb.cb[t, i] * pb.d * (pb.d - 1.0) * au ** (pb.d - 2.0) if au > 0 else 0.0
                for a in (lv, rv):
                    if a is not None:
                        H[a, a] += curv
                if lv is not None and rv is not None:
                    H[lv, rv] -= curv
                    H[rv, lv] -= curv
    for t in range(P):
        for i in np.nonzero(pc.zero_w[t])[0]:
            row = np.zeros(N)
            row[ix(t, i)] = 1.0
            E.append(row)
        idx, _ = pc.rows[t]
        for r in idx:
            row = np.zeros(N)
            row[t * n:(t + 1) * n] = pb.A[r]
            E.append(row)
        if pc.tight[t]:
            row = np.zeros(N)
            row[t * n:(t + 1) * n] = pc.sgn_w[t]
            E.append(row)
    E = np.array(E) if E else np.zeros((0, N))
    return H, E


def reference_gradient(inst: dict, grad_W: np.ndarray, sol=None, eps: float = 1e-9) -> Gradient:
    """Gradient of l(W*) = <grad_W, W*> + const (grad_W: (P, n)) with respect to alpha,
    s and F at the oracle's certified solution of ``inst``."""
    pb = normalize(inst)
    if sol is None:
        sol = solve(inst, tol=1e-11)
    W = np.atleast_2d(sol.W)
    P, n = pb.P, pb.n
    pc = piece_of(pb, W, eps)
    H, E = _system(pb, W, pc)
    N = P * n
    ne = E.shape[0]
    KKT = np.zeros((N + ne, N + ne))
    KKT[:N, :N] = H
    KKT[:N, N:] = E.T
    KKT[N:, :N] = E
    rhs = np.concatenate([np.asarray(grad_W, dtype=np.float64).reshape(N), np.zeros(ne)])
    # dependent equality rows leave nu non-unique; lambda is unique because H is
    # positive definite on the null space of E
    sol_kkt = np.linalg.lstsq(KKT, rhs, rcond=None)[0]
    lam = sol_kkt[:N].reshape(P, n)
    g_alpha = lam.copy()
    g_s = np.zeros((pb.Tp, n))
    for t in range(pb.Tp):
        left, right = t - 1, t
        lr = lam[right] if 0 <= right < P else np.zeros(n)
        ll = lam[left] if 0 <= left < P else np.zeros(n)
        g_s[t] = -pb.g2 * pc.sgn_u[t] * (lr - ll)
    g_F = np.zeros((n, pb.k))
    if pb.k:
        Om = 0.5 * (pb.Omega + pb.Omega.T)
        for t in range(P):
            x = W[t] - pb.c
            g_F -= 2.0 * pb.g1 * (np.outer(lam[t], x) + np.outer(x, lam[t])) @ pb.F @ Om
    loss = float(np.sum(np.asarray(grad_W).reshape(P, n) * W))
    return Gradient(alpha=g_alpha, s=g_s, F=g_F, W=W, loss=loss)
