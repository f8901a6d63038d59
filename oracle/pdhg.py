"""Restarted, averaged, diagonally preconditioned PDHG (plain FP64 NumPy).

Solves min_W g(W) + h(K W - b) for the splitting documented in ``problem``:
K W = (A w_t, G^T w_t, D W), b = (0, G^T c, b_C), h = box + g1||.||^2 + trade costs.

Iteration (Chambolle-Pock with diagonal step matrices, Pock-Chambolle 2011, alpha=1):

    x+ = prox_{tau g}(x - tau K^T y)
    y+ = prox_{sigma h~*}(y + sigma K (2 x+ - x)),   h~(z) = h(z - b),

with tau_i = theta / (omega * sum_j |K_ji|) and sigma_j = theta * omega / sum_i |K_ji|,
which keeps ||Sigma^(1/2) K T^(1/2)|| <= theta < 1 for every primal weight omega.
Convergence is measured on the running averages of the iterates; every
``check_every`` iterations the average or the current point (whichever has the
smaller relative KKT error) becomes a restart candidate, and the method restarts
from it when the error has dropped by a sufficient factor, or by a smaller factor
with no further progress, or when the current epoch is long compared to the total
(the adaptive restart rule of PDLP, Applegate et al. 2021).  At each restart the
primal weight is moved halfway (in log scale) to ||dy||_Sigma^-1 / ||dx||_T^-1,
by at most a factor ``omega_cap``.

This is deliberately a different PDHG variant from the one the GPU solver runs.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .problem import Problem, K_apply, KT_apply, K_offset, kkt
from .prox import l1_ball_quadratic, prox_cost

__all__ = ["pdhg", "PdhgResult"]


@dataclass
class PdhgResult:
    W: np.ndarray
    yA: np.ndarray
    yF: np.ndarray
    yC: np.ndarray
    rel_kkt: float
    iters: int
    restarts: int
    history: list = field(default_factory=list)


def _diag_steps(pb: Problem):
    """Row sums (dual) and column sums (primal) of |K| for the stacked operator."""
    absA = np.abs(pb.A)
    absG = np.abs(pb.G)
    rA = absA.sum(axis=1) if pb.m else np.zeros(0)
    rF = absG.sum(axis=0) if pb.k else np.zeros(0)
    colA = absA.sum(axis=0) if pb.m else np.zeros(pb.n)
    colF = absG.sum(axis=1) if pb.k else np.zeros(pb.n)
    if pb.g1 <= 0:
        rF = np.zeros_like(rF)
        colF = np.zeros(pb.n)
    if not pb.multi:
        rC = np.ones((1, pb.n))
        colC = np.ones(pb.n)
    else:
        rC = np.full((pb.Tp, pb.n), 2.0)
        rC[0] = 1.0
        rC[pb.P] = 1.0
        colC = np.full(pb.n, 2.0)
    col = colA + colF + colC
    return rA, rF, rC, col


def _safe_inv(x):
    return np.where(x > 0, 1.0 / np.where(x > 0, x, 1.0), 0.0)


def pdhg(pb: Problem, tol: float = 1e-10, max_iter: int = 200000, check_every: int = 64,
         theta: float = 0.99, W0=None, Y0=None, verbose: bool = False,
         omega_cap: float = 2.0) -> PdhgResult:
    P, n, m, k, Tp = pb.P, pb.n, pb.m, pb.k, pb.Tp
    rA, rF, rC, col = _diag_steps(pb)
    tau0 = theta * _safe_inv(col)                  # (n,)
    sA0 = theta * _safe_inv(rA)                    # (m,)
    sF0 = theta * _safe_inv(rF)                    # (k,)
    sC0 = theta * _safe_inv(rC)                    # (Tp, n)
    bA, bF, bC = K_offset(pb)
    a_risk = 2.0 * pb.g1 * pb.delta2

    x = np.tile(pb.w0, (P, 1)) if W0 is None else np.array(W0, dtype=np.float64).reshape(P, n)
    if Y0 is None:
        yA = np.zeros((P, m)); yF = np.zeros((P, k)); yC = np.zeros((Tp, n))
    else:
        yA, yF, yC = (np.array(v, dtype=np.float64) for v in Y0)
    omega = 1.0

    def primal_step(x, R, tau):
        v = x - tau[None, :] * R
        out = np.empty_like(x)
        a = 1.0 / tau + a_risk
        for t in range(P):
            b = v[t] / tau + pb.alpha[t] + a_risk * pb.c
            out[t], _ = l1_ball_quadratic(b, a)
        return out

    def dual_step(yA, yF, yC, xbar, sA, sF, sC):
        zA, zF, zC = K_apply(pb, xbar)
        vA = yA + sA[None, :] * zA
        nA = vA - sA[None, :] * np.clip(vA / np.where(sA > 0, sA, 1.0)[None, :], pb.L[None, :], pb.U[None, :])
        nA = np.where(sA[None, :] > 0, nA, 0.0)
        if k and pb.g1 > 0:
            vF = yF + sF[None, :] * zF
            nF = 2.0 * pb.g1 * (vF - sF[None, :] * bF) / (sF[None, :] + 2.0 * pb.g1)
        else:
            nF = np.zeros_like(yF)
        vC = yC + sC * zC
        z = vC / sC - bC
        nC = vC - sC * bC - sC * prox_cost(z, 1.0 / sC, pb.ca, pb.cb, pb.d)
        return nA, nF, nC

    def err(xx, ya, yf, yc):
        return kkt(pb, xx, ya, yf, yc).rel_kkt

    # restart bookkeeping
    last = (x.copy(), yA.copy(), yF.copy(), yC.copy())
    e_last = err(x, yA, yF, yC)
    e_prev_cand = np.inf
    sum_x = np.zeros_like(x); sum_yA = np.zeros_like(yA); sum_yF = np.zeros_like(yF); sum_yC = np.zeros_like(yC)
    cnt = 0
    it_epoch = 0
    restarts = 0
    history = []
    best = (e_last, x.copy(), yA.copy(), yF.copy(), yC.copy())
    it = 0
    while it < max_iter:
        tau = tau0 / omega
        sA, sF, sC = sA0 * omega, sF0 * omega, sC0 * omega
        R = KT_apply(pb, yA, yF, yC)
        xn = primal_step(x, R, tau)
        yAn, yFn, yCn = dual_step(yA, yF, yC, 2.0 * xn - x, sA, sF, sC)
        x, yA, yF, yC = xn, yAn, yFn, yCn
        sum_x += x; sum_yA += yA; sum_yF += yF; sum_yC += yC
        cnt += 1
        it += 1
        it_epoch += 1
        if it % check_every:
            continue
        ax, ayA, ayF, ayC = sum_x / cnt, sum_yA / cnt, sum_yF / cnt, sum_yC / cnt
        e_avg = err(ax, ayA, ayF, ayC)
        e_cur = err(x, yA, yF, yC)
        if e_avg < e_cur:
            cand, e_c = (ax, ayA, ayF, ayC), e_avg
        else:
            cand, e_c = (x.copy(), yA.copy(), yF.copy(), yC.copy()), e_cur
        if e_c < best[0]:
            best = (e_c,) + tuple(v.copy() for v in cand)
        history.append((it, e_c, omega))
        if verbose:
            print(f"[oracle pdhg] it {it} err {e_c:.3e} omega {omega:.3e}")
        if e_c <= tol:
            break
        do_restart = (e_c <= 0.2 * e_last) or (e_c <= 0.8 * e_last and e_c > e_prev_cand) \
            or (it_epoch >= 0.36 * it)
        e_prev_cand = e_c
        if do_restart:
            cx, cyA, cyF, cyC = cand
            lx, lyA, lyF, lyC = last
            dx = np.sqrt(np.sum((cx - lx) ** 2 / tau0[None, :]))
            dy2 = np.sum((cyA - lyA) ** 2 * _safe_inv(sA0)[None, :]) + \
                np.sum((cyF - lyF) ** 2 * _safe_inv(sF0)[None, :]) + np.sum((cyC - lyC) ** 2 / sC0)
            dy = np.sqrt(dy2)
            if dx > 1e-300 and dy > 1e-300:
                new = float(np.exp(0.5 * np.log(dy / dx) + 0.5 * np.log(omega)))
                omega = min(max(new, omega / omega_cap), omega * omega_cap)
            x, yA, yF, yC = (v.copy() for v in cand)
            last = (x.copy(), yA.copy(), yF.copy(), yC.copy())
            e_last = e_c
            e_prev_cand = np.inf
            sum_x[:] = 0; sum_yA[:] = 0; sum_yF[:] = 0; sum_yC[:] = 0
            cnt = 0
            it_epoch = 0
            restarts += 1
    e_b, bx, byA, byF, byC = best
    return PdhgResult(W=bx, yA=byA, yF=byF, yC=byC, rel_kkt=float(e_b), iters=it, restarts=restarts,
                      history=history)
