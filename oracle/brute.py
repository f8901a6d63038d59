"""Brute-force minimiser for tiny instances (independent of pdhg/polish).

On every orthant of the signs of the weights w_ti and of the trades u_ti the scaled
objective of paper eq. 1 / eq. 4 is smooth and convex: |u| = s_u u and |w| = s_w w
are linear there, so the budget ||w_t||_1 <= 1 becomes the linear inequality
sum_i s_w,ti w_ti <= 1 together with the sign constraints s_w w >= 0, s_u u >= 0.
The union of these closed pieces is the whole feasible set, so the optimum is the
smallest of the per-piece minima.  Each piece is solved with SciPy's SLSQP from a
dense, explicitly formed Sigma = F Omega F^T + diag(delta^2); nothing here reuses
the oracle's factorisation, dual or proximal maps.  Cost: 2^(P n + T' n) pieces, so
only for n <= 4 (single-period) or P n + T' n <= 8.
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy.optimize import minimize

__all__ = ["brute_force"]


def brute_force(inst: dict, max_pieces: int = 4096):
    T = int(inst.get("T", 0) or 0)
    alpha = np.atleast_2d(np.asarray(inst["alpha"], dtype=np.float64))
    P, n = alpha.shape
    Tp = 1 if T == 0 else T
    F = np.asarray(inst["F"], dtype=np.float64).reshape(n, -1)
    Om = np.asarray(inst["Omega"], dtype=np.float64)
    Sigma = F @ Om @ F.T + np.diag(np.asarray(inst["delta"], dtype=np.float64) ** 2)
    GMV = float(inst["GMV"])
    l1, l2, l3 = float(inst["lambda1"]), float(inst["lambda2"]), float(inst["lambda3"])
    s = np.atleast_2d(np.asarray(inst["s"], dtype=np.float64))
    q = np.atleast_2d(np.asarray(inst["q"], dtype=np.float64))
    d = float(inst["d"])
    A = np.asarray(inst["A"], dtype=np.float64).reshape(-1, n)
    L = np.asarray(inst["L"], dtype=np.float64)
    U = np.asarray(inst["U"], dtype=np.float64)
    w0 = np.asarray(inst["w0"], dtype=np.float64)
    wT = np.asarray(inst["w_target"], dtype=np.float64) if T else None
    nv = P * n
    npieces = 2 ** (nv + Tp * n)
    if npieces > max_pieces:
        raise ValueError("instance too large for brute force")

    def weights(x):
        return x.reshape(P, n)

    def trade_mat():
        """u = D x + e with D (Tp*n, P*n)."""
        D = np.zeros((Tp * n, nv))
        e = np.zeros(Tp * n)
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
        return D, e

    D, e = trade_mat()
    cen = np.zeros(n) if T == 0 else wT
    sv = (l2 * s).reshape(-1)
    qv = (l3 * q).reshape(-1)
    g1 = l1 * GMV

    def obj_piece(x, su):
        W = weights(x)
        val = 0.0
        grad = np.zeros(nv)
        for t in range(P):
            xc = W[t] - cen
            val += -alpha[t] @ W[t] + g1 * xc @ Sigma @ xc
            grad[t * n:(t + 1) * n] = -alpha[t] + 2.0 * g1 * Sigma @ xc
        u = D @ x + e
        au = np.maximum(su * u, 0.0)
        val += float(np.sum(sv * au + qv * au ** d))
        gu = su * (sv + qv * d * au ** (d - 1.0))
        grad += D.T @ gu
        return val, grad

    best = (np.inf, None)
    for sw in itertools.product((-1.0, 1.0), repeat=nv):
        sw = np.array(sw)
        for su in itertools.product((-1.0, 1.0), repeat=Tp * n):
            su = np.array(su)
            cons = [
                {"type": "ineq", "fun": lambda x, sw=sw: sw * x, "jac": lambda x, sw=sw: np.diag(sw)},
                {"type": "ineq", "fun": lambda x, su=su: su * (D @ x + e), "jac": lambda x, su=su: su[:, None] * D},
            ]
            for t in range(P):
                row = np.zeros(nv)
                row[t * n:(t + 1) * n] = sw[t * n:(t + 1) * n]
                cons.append({"type": "ineq", "fun": lambda x, row=row: 1.0 - row @ x, "jac": lambda x, row=row: -row[None, :]})
                if A.shape[0]:
                    At = np.zeros((A.shape[0], nv))
                    At[:, t * n:(t + 1) * n] = A
                    fl = np.isfinite(L)
                    fu = np.isfinite(U)
                    if fl.any():
                        cons.append({"type": "ineq", "fun": lambda x, At=At, fl=fl: (At @ x - L)[fl],
                                     "jac": lambda x, At=At, fl=fl: At[fl]})
                    if fu.any():
                        cons.append({"type": "ineq", "fun": lambda x, At=At, fu=fu: (U - At @ x)[fu],
                                     "jac": lambda x, At=At, fu=fu: -At[fu]})
            x0 = np.tile(w0, P)
            res = minimize(lambda x: obj_piece(x, su), x0, jac=True, method="SLSQP", constraints=cons,
                           options={"ftol": 1e-16, "maxiter": 500})
            x = res.x
            # feasibility of the piece (tolerant): reject points that violate its constraints
            viol = 0.0
            for c in cons:
                viol = max(viol, float(np.max(-np.asarray(c["fun"](x)), initial=0.0)))
            if viol > 1e-9:
                continue
            val = obj_piece(x, su)[0]
            if val < best[0]:
                best = (val, x.copy())
    if best[1] is None:
        raise RuntimeError("no feasible piece")
    return best[1].reshape(P, n), best[0]
