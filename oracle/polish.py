"""Active-set polish and exact optimality certificate (plain FP64 NumPy).

Given an approximate primal-dual point, guess which nonsmooth pieces are active at
the optimum (paper eq. 1-6):

* zero trades u_ti = 0 (the spread term's kink),
* zero weights w_ti = 0 in periods whose budget ||w_t||_1 <= 1 is tight,
* exposure rows at L or U, and the tight budgets themselves.

On that piece the problem is smooth: merge each asset's consecutive periods joined
by zero trades into one variable (fixed to w_0, w_T or 0 where a member is fixed),
give every nonzero trade and weight its sign, and minimise the smooth objective
subject to the active linear equalities by Newton's method.  The factor part of the
risk is lifted (v_t = G^T (w_t - c), cost g1 ||v_t||^2), so the Hessian in the asset
variables is block diagonal with one small block per asset and the equality
constraints are handled through a dense Schur complement of size
(k + active rows + tight budgets) per period.

The result is then CERTIFIED, independently of how it was found: multipliers are
recovered (exposure rows, budgets, and the spread subgradients of zero trades by
interval propagation along each asset's trade chain), every sign and interval
condition of the KKT system is checked, the dual point is assembled and the duality
gap Phi(W) - Psi(Y) is evaluated with the closed-form dual.  A gap at rounding level
with W feasible proves W is the optimum up to the strong-convexity bound.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .problem import Problem, objective, trades, dual_objective, kkt

__all__ = ["polish", "PolishResult", "certify_dual"]


@dataclass
class PolishResult:
    ok: bool
    W: np.ndarray | None
    yA: np.ndarray | None
    yF: np.ndarray | None
    yC: np.ndarray | None
    gap: float
    rel_gap: float
    newton_iters: int
    reason: str


class _Piece:
    """Identified active set in array form."""

    def __init__(self, pb: Problem, W, yA, eps_u, eps_w, eps_e, eps_b):
        P, n, Tp = pb.P, pb.n, pb.Tp
        W = np.atleast_2d(W)
        scale = max(1e-300, float(np.abs(W).max()))
        U = trades(pb, W)
        self.zero_trade = np.abs(U) <= eps_u * scale                 # (Tp, n)
        self.sgn_u = np.where(self.zero_trade, 0.0, np.sign(U))
        l1 = np.abs(W).sum(axis=1)
        self.tight = l1 >= 1.0 - eps_b                                # (P,)
        self.zero_w = (np.abs(W) <= eps_w * scale) & self.tight[:, None]
        self.sgn_w = np.where(self.zero_w, 0.0, np.sign(W)) * self.tight[:, None]
        AW = W @ pb.A.T
        span = np.maximum(pb.U - pb.L, 0.0)
        tol_e = eps_e * np.maximum(1.0, np.where(np.isfinite(span), span, 1.0))
        eq = np.isfinite(pb.L) & (pb.U == pb.L)
        self.at_U = (pb.U[None, :] - AW <= tol_e[None, :]) & np.isfinite(pb.U)[None, :]
        self.at_L = (AW - pb.L[None, :] <= tol_e[None, :]) & np.isfinite(pb.L)[None, :] & ~self.at_U
        self.at_U |= eq[None, :]
        self.eq = np.broadcast_to(eq[None, :], AW.shape)
        # groups along each asset's chain of nodes 0..P (+ node T for multi-period)
        nn = P + 2 if pb.multi else P + 1
        self.grp = -np.ones((P, n), dtype=np.int64)
        self.fv = np.zeros((P, n))
        self.ng = np.zeros(n, dtype=np.int64)
        self.bad = False
        for i in range(n):
            parent = list(range(nn))

            def find(a):
                while parent[a] != a:
                    parent[a] = parent[parent[a]]
                    a = parent[a]
                return a
            for t in range(Tp):            # trade t+1 joins nodes t and t+1
                if self.zero_trade[t, i]:
                    ra, rb = find(t), find(t + 1)
                    if ra != rb:
                        parent[ra] = rb
            fixed = {}
            vals = {0: pb.w0[i]}
            if pb.multi:
                vals[P + 1] = pb.wT[i]
            for t in range(P):
                if self.zero_w[t, i]:
                    vals[t + 1] = 0.0
            for node, v in vals.items():
                r = find(node)
                if r in fixed and abs(fixed[r] - v) > 1e-15 * max(1.0, abs(v)):
                    self.bad = True
                fixed.setdefault(r, v)
            gid = {}
            for t in range(P):
                r = find(t + 1)
                if r in fixed:
                    self.fv[t, i] = fixed[r]
                else:
                    if r not in gid:
                        gid[r] = len(gid)
                    self.grp[t, i] = gid[r]
            self.ng[i] = len(gid)
        self.free = self.grp >= 0


def _expand(pb, pc: _Piece, X):
    """W(X): free entries from the per-asset variables X (n, P), fixed ones from fv."""
    P, n = pb.P, pb.n
    cols = np.arange(n)[None, :].repeat(P, axis=0)
    g = np.where(pc.free, pc.grp, 0)
    return np.where(pc.free, X[cols, g], pc.fv)


def _gather(pb, pc: _Piece, D):
    """Adjoint of _expand restricted to free entries: sum period values into groups."""
    P, n = pb.P, pb.n
    out = np.zeros((n, P))
    t_idx, i_idx = np.nonzero(pc.free)
    np.add.at(out, (i_idx, pc.grp[t_idx, i_idx]), D[t_idx, i_idx])
    return out


def _trade_nodes(pb):
    """For trade t (0-based) the left and right period indices (-1 = w_0, P = w_T)."""
    left = np.arange(pb.Tp) - 1
    right = np.arange(pb.Tp)
    return left, right


def _smooth_parts(pb, pc: _Piece, W):
    """Objective (without the lifted factor term), its W-gradient, and the per-trade
    curvature phi'' for the identified piece."""
    P, n = pb.P, pb.n
    x = W - pb.c[None, :]
    f = float(np.sum(-pb.alpha * W) + pb.g1 * np.sum(pb.delta2[None, :] * x * x))
    gW = -pb.alpha + 2.0 * pb.g1 * pb.delta2[None, :] * x
    U = trades(pb, W)
    su = pc.sgn_u
    au = su * U                                     # |u| on nonzero trades
    nz = su != 0
    d = pb.d
    auz = np.where(nz, np.maximum(au, 0.0), 0.0)
    f += float(np.sum(np.where(nz, pb.ca * auz + pb.cb * auz ** d, 0.0)))
    dphi = np.where(nz, su * (pb.ca + pb.cb * d * auz ** (d - 1.0)), 0.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        ddphi = np.where(nz & (auz > 0), pb.cb * d * (d - 1.0) * auz ** (d - 2.0), 0.0)
    left, right = _trade_nodes(pb)
    for t in range(pb.Tp):
        if 0 <= right[t] < P:
            gW[right[t]] += dphi[t]
        if 0 <= left[t] < P:
            gW[left[t]] -= dphi[t]
    return f, gW, dphi, ddphi, au


def _hessian(pb, pc: _Piece, ddphi):
    P, n = pb.P, pb.n
    H = np.zeros((n, P, P))
    ar = np.arange(n)
    for t in range(P):
        fr = pc.free[t]
        g = pc.grp[t]
        H[ar[fr], g[fr], g[fr]] += 2.0 * pb.g1 * pb.delta2[fr]
    left, right = _trade_nodes(pb)
    for t in range(pb.Tp):
        c = ddphi[t]
        lf = pc.free[left[t]] if 0 <= left[t] < P else np.zeros(n, bool)
        rf = pc.free[right[t]] if 0 <= right[t] < P else np.zeros(n, bool)
        gl = pc.grp[left[t]] if 0 <= left[t] < P else np.zeros(n, np.int64)
        gr = pc.grp[right[t]] if 0 <= right[t] < P else np.zeros(n, np.int64)
        m = rf
        H[ar[m], gr[m], gr[m]] += c[m]
        m = lf
        H[ar[m], gl[m], gl[m]] += c[m]
        m = lf & rf & (gl != gr)
        H[ar[m], gl[m], gr[m]] -= c[m]
        H[ar[m], gr[m], gl[m]] -= c[m]
    # pad unused groups with the identity
    for g in range(P):
        pad = pc.ng <= g
        H[pad, g, g] = 1.0
    return H


def _rows(pb, pc: _Piece):
    """Equality rows per period: lifted factor rows, active exposure rows, tight budget."""
    rows = []
    for t in range(pb.P):
        act = np.nonzero(pc.at_U[t] | pc.at_L[t])[0]
        bnd = np.where(pc.at_U[t, act], pb.U[act], pb.L[act])
        rows.append((act, bnd, bool(pc.tight[t])))
    return rows


def _coef(pb, pc: _Piece, rows, t):
    """Coefficient matrix (n, nr_t) of period t's rows on w_t (lift rows carry -G)."""
    act, _, tight = rows[t]
    blocks = []
    if pb.k and pb.g1 > 0:
        blocks.append(-pb.G)
    if act.size:
        blocks.append(pb.A[act].T)
    if tight:
        blocks.append(pc.sgn_w[t][:, None])
    if not blocks:
        return np.zeros((pb.n, 0))
    C = np.concatenate(blocks, axis=1)
    return C * pc.free[t][:, None]


def _newton(pb, pc: _Piece, W_init, max_iter=60):
    P, n = pb.P, pb.n
    lift = pb.k > 0 and pb.g1 > 0
    rows = _rows(pb, pc)
    # initial X: mean of the period values in each group
    X = np.zeros((n, P))
    cnt = np.zeros((n, P))
    t_idx, i_idx = np.nonzero(pc.free)
    np.add.at(X, (i_idx, pc.grp[t_idx, i_idx]), W_init[t_idx, i_idx])
    np.add.at(cnt, (i_idx, pc.grp[t_idx, i_idx]), 1.0)
    X = np.where(cnt > 0, X / np.maximum(cnt, 1.0), 0.0)
    W = _expand(pb, pc, X)
    V = (W - pb.c[None, :]) @ pb.G if lift else np.zeros((P, 0))
    coefs = [_coef(pb, pc, rows, t) for t in range(P)]
    nr = [c.shape[1] for c in coefs]
    off = np.concatenate([[0], np.cumsum(nr)]).astype(int)
    Nr = int(off[-1])
    kk = pb.k if lift else 0
    lam = np.zeros(Nr)

    def residual(W, V):
        r = np.zeros(Nr)
        for t in range(P):
            act, bnd, tight = rows[t]
            o = off[t]
            if lift:
                r[o:o + kk] = pb.G.T @ (W[t] - pb.c) - V[t]
                o += kk
            if act.size:
                r[o:o + act.size] = bnd - pb.A[act] @ W[t]
                o += act.size
            if tight:
                r[o] = 1.0 - float(pc.sgn_w[t] @ W[t])
        return r

    def in_region(W):
        U = trades(pb, W)
        ok_u = np.all((pc.sgn_u == 0) | (pc.sgn_u * U > 0))
        ok_w = np.all((pc.sgn_w == 0) | (pc.sgn_w * W > 0) | ~pc.free)
        return bool(ok_u and ok_w)

    def merit(W, V):
        f, _, _, _, _ = _smooth_parts(pb, pc, W)
        return f + (pb.g1 * float(np.sum(V * V)) if lift else 0.0)

    it = 0
    for it in range(1, max_iter + 1):
        f, gW, dphi, ddphi, _ = _smooth_parts(pb, pc, W)
        gX = _gather(pb, pc, gW)
        gV = 2.0 * pb.g1 * V if lift else None
        H = _hessian(pb, pc, ddphi)
        Hinv = np.linalg.inv(H)
        # period-space inverse blocks M[i, t, t'] for free entries
        ar = np.arange(n)
        Mt = np.zeros((n, P, P))
        for t in range(P):
            for s in range(P):
                both = pc.free[t] & pc.free[s]
                Mt[both, t, s] = Hinv[ar[both], pc.grp[t, both], pc.grp[s, both]]
        S = np.zeros((Nr, Nr))
        for t in range(P):
            if nr[t] == 0:
                continue
            for s in range(P):
                if nr[s] == 0:
                    continue
                S[off[t]:off[t + 1], off[s]:off[s + 1]] = coefs[t].T @ (Mt[:, t, s][:, None] * coefs[s])
        if lift:
            for t in range(P):
                idx = np.arange(off[t], off[t] + kk)
                S[idx, idx] += 1.0 / (2.0 * pb.g1)
        hx = np.einsum("igh,ih->ig", Hinv, gX)
        HW = _expand(pb, pc, hx) * pc.free
        CHg = np.zeros(Nr)
        for t in range(P):
            if nr[t]:
                CHg[off[t]:off[t + 1]] = coefs[t].T @ HW[t]
                if lift:
                    CHg[off[t]:off[t] + kk] += gV[t] / (2.0 * pb.g1)
        rp = residual(W, V)
        rhs = -CHg - rp
        if Nr:
            try:
                lam = np.linalg.solve(S, rhs)
            except np.linalg.LinAlgError:
                lam = np.linalg.lstsq(S, rhs, rcond=None)[0]
        CtW = np.zeros((P, n))
        for t in range(P):
            if nr[t]:
                CtW[t] = coefs[t] @ lam[off[t]:off[t + 1]]
        CtX = _gather(pb, pc, CtW)
        dX = -np.einsum("igh,ih->ig", Hinv, gX + CtX)
        dX[np.arange(P)[None, :] >= pc.ng[:, None]] = 0.0
        if lift:
            lam_lift = np.stack([lam[off[t]:off[t] + kk] for t in range(P)])
            dV = -(gV + lam_lift) / (2.0 * pb.g1)
        else:
            dV = np.zeros_like(V)
        scale = max(1e-300, float(np.abs(W).max()))
        step = 1.0
        base = merit(W, V)
        first = it == 1
        accepted = False
        for _ in range(60):
            Xn = X + step * dX
            Wn = _expand(pb, pc, Xn)
            Vn = V + step * dV
            if in_region(Wn):
                if first or merit(Wn, Vn) <= base + 1e-14 * abs(base) + 1e-30:
                    accepted = True
                    break
            step *= 0.5
        if not accepted:
            return None, None, lam, it, rows, off, "line search left the piece"
        X, W, V = Xn, Wn, Vn
        if float(np.abs(dX).max(initial=0.0)) * step <= 1e-15 * scale and \
                float(np.abs(residual(W, V)).max(initial=0.0)) <= 1e-15 * max(1.0, scale):
            break
    return X, W, lam, it, rows, off, ""


def _chain_duals(pb, pc: _Piece, W, yA, yF, mu, tol):
    """Spread subgradients xi (= y_C) and budget subgradients zeta that satisfy
    g_t + zeta_t + xi_t - xi_{t+1} = 0 along each asset's trade chain, chosen inside
    their intervals; returns (xi, ok)."""
    P, n, Tp = pb.P, pb.n, pb.Tp
    R = yA @ pb.A + yF @ pb.G.T
    gsm = -pb.alpha + 2.0 * pb.g1 * pb.delta2[None, :] * (W - pb.c[None, :]) + R    # (P, n)
    U = trades(pb, W)
    d = pb.d
    au = np.abs(U)
    pt = np.where(pc.sgn_u != 0, pc.sgn_u * (pb.ca + pb.cb * d * au ** (d - 1.0)), 0.0)
    Ilo = np.where(pc.sgn_u != 0, pt, -pb.ca)
    Ihi = np.where(pc.sgn_u != 0, pt, pb.ca)
    zw = pc.zero_w
    Jlo = np.where(zw, -mu[:, None], mu[:, None] * pc.sgn_w)
    Jhi = np.where(zw, mu[:, None], mu[:, None] * pc.sgn_w)
    # forward interval propagation
    Xlo = np.zeros((Tp + 1, n)); Xhi = np.zeros((Tp + 1, n))
    Xlo[0], Xhi[0] = Ilo[0] - tol, Ihi[0] + tol
    ok = np.ones(n, bool)
    for t in range(P):
        ylo = Xlo[t] + gsm[t] + Jlo[t]
        yhi = Xhi[t] + gsm[t] + Jhi[t]
        if pb.multi:
            lo = np.maximum(ylo, Ilo[t + 1] - tol)
            hi = np.minimum(yhi, Ihi[t + 1] + tol)
        else:
            lo = np.maximum(ylo, -tol)
            hi = np.minimum(yhi, tol)
        ok &= lo <= hi
        Xlo[t + 1], Xhi[t + 1] = lo, np.maximum(hi, lo)
    # backward choice
    xi = np.zeros((Tp + 1, n))
    if pb.multi:
        xi[P] = np.clip(0.5 * (Ilo[P] + Ihi[P]), Xlo[P], Xhi[P])
    else:
        xi[1] = 0.0
    for t in range(P - 1, -1, -1):
        lo = np.maximum(Xlo[t], xi[t + 1] - gsm[t] - Jhi[t])
        hi = np.minimum(Xhi[t], xi[t + 1] - gsm[t] - Jlo[t])
        ok &= lo <= hi + tol
        mid = 0.5 * (np.maximum(Ilo[t], lo) + np.minimum(Ihi[t], hi))
        xi[t] = np.clip(mid, lo, np.maximum(hi, lo))
    return xi[:Tp], ok


def certify_dual(pb: Problem, W, yA, yF, yC):
    """Duality gap of a primal-dual pair and the implied bound on ||W - W*||_F."""
    po = objective(pb, W)
    do = dual_objective(pb, yA, yF, yC)
    gap = po - do
    mind = float(pb.delta2.min()) if pb.n else 0.0
    bound = np.sqrt(max(gap, 0.0) / (pb.g1 * mind)) if pb.g1 > 0 and mind > 0 else np.inf
    return po, do, gap, bound


def polish(pb: Problem, W, yA, yF, yC, eps=(1e-7, 1e-6, 1e-5, 1e-8, 1e-4, 1e-9, 1e-10, 1e-11)) -> PolishResult:
    if pb.g1 <= 0 or float(pb.delta2.min(initial=1.0)) <= 0:
        return PolishResult(False, None, None, None, None, np.inf, np.inf, 0,
                            "polish needs g1 > 0 and delta > 0")
    W = np.atleast_2d(np.asarray(W, dtype=np.float64))
    last = "no attempt"
    for e in eps:
        pc = _Piece(pb, W, yA, eps_u=e, eps_w=e, eps_e=e, eps_b=1e-9)
        if pc.bad:
            last = f"eps {e}: inconsistent fixed values"
            continue
        X, Wn, lam, its, rows, off, why = _newton(pb, pc, W)
        if X is None:
            last = f"eps {e}: {why}"
            continue
        # multipliers: exposure rows and budgets from lam
        lift = pb.k > 0 and pb.g1 > 0
        kk = pb.k if lift else 0
        yA_n = np.zeros((pb.P, pb.m))
        mu = np.zeros(pb.P)
        for t in range(pb.P):
            act, _, tight = rows[t]
            o = off[t] + kk
            yA_n[t, act] = lam[o:o + act.size]
            if tight:
                mu[t] = lam[o + act.size]
        yF_n = 2.0 * pb.g1 * (Wn - pb.c[None, :]) @ pb.G
        scale = max(float(np.abs(pb.ca).max(initial=0.0)), float(np.abs(mu).max(initial=0.0)),
                    float(np.abs(pb.alpha).max(initial=0.0)), 1e-300)
        tol = 1e-10 * scale
        # sign conditions
        sgn_ok = np.all(yA_n[pc.at_U & ~pc.eq] >= -tol) and np.all(yA_n[pc.at_L] <= tol) and np.all(mu >= -tol)
        if not sgn_ok:
            last = f"eps {e}: multiplier sign"
            continue
        yA_n = np.where(pc.at_U & ~pc.eq, np.maximum(yA_n, 0.0), yA_n)
        yA_n = np.where(pc.at_L, np.minimum(yA_n, 0.0), yA_n)
        mu = np.maximum(mu, 0.0)
        xi, ok = _chain_duals(pb, pc, Wn, yA_n, yF_n, mu, tol)
        if not np.all(ok):
            last = f"eps {e}: subgradient chain infeasible for {int((~ok).sum())} assets"
            continue
        # primal feasibility of inactive pieces
        K = kkt(pb, Wn, yA_n, yF_n, xi)
        if K.rel_pri > 1e-12 or K.budget_excess > 1e-13:
            last = f"eps {e}: primal infeasible (rel_pri {K.rel_pri:.2e})"
            continue
        po, do, gap, _ = certify_dual(pb, Wn, yA_n, yF_n, xi)
        rel = abs(gap) / max(abs(po) + abs(do), 1e-300)
        if rel > 1e-11:
            last = f"eps {e}: gap {rel:.2e}"
            continue
        return PolishResult(True, Wn, yA_n, yF_n, xi, gap, rel, its, "")
    return PolishResult(False, None, None, None, None, np.inf, np.inf, 0, last)
