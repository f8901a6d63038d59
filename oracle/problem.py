"""Problem data, primal objective, closed-form dual and relative KKT (plain FP64).

Notation (paper Section 2): n assets, k factors, m exposure rows.  Single-period has
one decision vector w (P = 1) and one trade u = w - w0 (T' = 1).  Multi-period with
horizon T has decisions w_1..w_{T-1} (P = T-1) and trades u_t = w_t - w_{t-1},
t = 1..T (T' = T) with w_0 and w_T given.  Risk is measured against c = 0
(single-period) or c = w_T (multi-period, paper eq. 4).

Splitting used for the dual.  With G any n x k matrix with G G^T = F Omega F^T
(here G = F V diag(sqrt(lambda)) from the eigendecomposition of Omega),

    Phi(W) = g(W) + sum_t h_A(A w_t) + sum_t h_F(G^T (w_t - c)) + sum_t cost_t(u_t),
    g(W)   = sum_t [ -a_t^T w_t + g1 sum_i delta_i^2 (w_ti - c_i)^2 + I{||w_t||_1 <= 1} ],
    h_A    = indicator of [L, U],  h_F(v) = g1 ||v||^2,
    cost_t(u) = sum_i g2 s_ti |u_i| + g3 q_ti |u_i|^d.

Fenchel duality gives, for duals y_A (P x m), y_F (P x k), y_C (T' x n):

    Psi(Y) = sum_t min_{||w||_1<=1} [ g1 sum_i delta_i^2 (w_i - c_i)^2 + (R_t - a_t)^T w ]
             - sum_t y_F,t^T G^T c - y_C,1^T w_0 + y_C,T^T w_T
             - sum_t supp_[L,U](y_A,t) - sum_t ||y_F,t||^2 / (4 g1) - sum_t cost_t^*(y_C,t),
    R_t    = A^T y_A,t + G y_F,t + y_C,t - y_C,t+1    (single-period: + y_C),

and Psi(Y) <= Phi(W) for every feasible W.  Because Phi is strongly convex with
modulus at least 2 g1 min delta^2 (per coordinate), any feasible W satisfies
||W - W*||_F^2 <= (Phi(W) - Psi(Y)) / (g1 min_i delta_i^2).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .prox import conj_cost, l1_ball_quadratic

__all__ = ["Problem", "normalize", "trades", "objective", "dual_objective", "kkt",
           "project_dual_domain", "K_apply", "KT_apply", "risk_factor"]


def risk_factor(Omega: np.ndarray) -> np.ndarray:
    """C with C C^T = Omega for a symmetric PSD Omega (eigendecomposition)."""
    Om = 0.5 * (Omega + Omega.T)
    lam, V = np.linalg.eigh(Om)
    if lam.size and lam.min() < -1e-12 * max(1.0, abs(lam).max()):
        raise ValueError("Omega is not positive semidefinite")
    return V * np.sqrt(np.maximum(lam, 0.0))[None, :]


@dataclass
class Problem:
    n: int
    k: int
    m: int
    T: int           # 0 for single-period, else the horizon
    P: int           # decision periods
    Tp: int          # trades
    alpha: np.ndarray   # (P, n)
    F: np.ndarray       # (n, k)
    Omega: np.ndarray   # (k, k)
    G: np.ndarray       # (n, k)  G G^T = F Omega F^T
    delta2: np.ndarray  # (n,)
    ca: np.ndarray      # (Tp, n) g2 * s
    cb: np.ndarray      # (Tp, n) g3 * q
    d: float
    A: np.ndarray       # (m, n)
    L: np.ndarray
    U: np.ndarray
    w0: np.ndarray
    wT: np.ndarray | None
    c: np.ndarray       # (n,) risk centre
    g1: float
    g2: float
    g3: float
    GMV: float

    @property
    def multi(self) -> bool:
        return self.T > 0


def normalize(inst: dict, factor: np.ndarray | None = None) -> Problem:
    """Scale the paper's maximisation (eq. 1 / eq. 4) to the minimisation form Phi.

    ``factor``: optional k x k matrix C with C C^T = Omega fixing the coordinates of the
    factor dual y_F (G = F C); default: the eigendecomposition of Omega.  Phi, W* and
    Psi's value do not depend on this choice, only the meaning of y_F does."""
    T = int(inst.get("T", 0) or 0)
    alpha = np.atleast_2d(np.asarray(inst["alpha"], dtype=np.float64))
    n = alpha.shape[1]
    P = 1 if T == 0 else T - 1
    Tp = 1 if T == 0 else T
    if alpha.shape[0] != P:
        raise ValueError("alpha must have P rows")
    F = np.asarray(inst["F"], dtype=np.float64).reshape(n, -1)
    k = F.shape[1]
    Omega = np.asarray(inst["Omega"], dtype=np.float64).reshape(k, k)
    delta = np.asarray(inst["delta"], dtype=np.float64)
    s = np.atleast_2d(np.asarray(inst["s"], dtype=np.float64))
    q = np.atleast_2d(np.asarray(inst["q"], dtype=np.float64))
    if s.shape != (Tp, n) or q.shape != (Tp, n):
        raise ValueError("s and q must have T' rows")
    d = float(inst["d"])
    if not (1.0 < d <= 2.0):
        raise ValueError("d must lie in (1, 2]")
    A = np.asarray(inst["A"], dtype=np.float64).reshape(-1, n)
    m = A.shape[0]
    L = np.asarray(inst["L"], dtype=np.float64).reshape(m)
    U = np.asarray(inst["U"], dtype=np.float64).reshape(m)
    w0 = np.asarray(inst["w0"], dtype=np.float64).reshape(n)
    GMV = float(inst["GMV"])
    g1 = float(inst["lambda1"]) * GMV
    g2 = float(inst["lambda2"])
    g3 = float(inst["lambda3"])
    if T > 0:
        wT = np.asarray(inst["w_target"], dtype=np.float64).reshape(n)
        c = wT.copy()
    else:
        wT = None
        c = np.zeros(n)
    if k > 0 and factor is not None:
        C = np.asarray(factor, dtype=np.float64).reshape(k, k)
        if not np.allclose(C @ C.T, 0.5 * (Omega + Omega.T), rtol=1e-10, atol=1e-14 * max(1.0, np.abs(Omega).max())):
            raise ValueError("factor does not satisfy C C^T = Omega")
    else:
        C = risk_factor(Omega) if k > 0 else None
    G = F @ C if k > 0 else np.zeros((n, 0))
    return Problem(n=n, k=k, m=m, T=T, P=P, Tp=Tp, alpha=alpha, F=F, Omega=Omega, G=G,
                   delta2=delta * delta, ca=g2 * s, cb=g3 * q, d=d, A=A, L=L, U=U, w0=w0,
                   wT=wT, c=c, g1=g1, g2=g2, g3=g3, GMV=GMV)


def trades(pb: Problem, W: np.ndarray) -> np.ndarray:
    """u_t = w_t - w_{t-1} for t = 1..T' (w_0 and, multi-period, w_T given)."""
    W = np.atleast_2d(W)
    if not pb.multi:
        return W - pb.w0[None, :]
    Uo = np.empty((pb.Tp, pb.n))
    Uo[0] = W[0] - pb.w0
    if pb.P > 1:
        Uo[1:pb.P] = W[1:] - W[:-1]
    Uo[pb.P] = pb.wT - W[pb.P - 1]
    return Uo


def objective(pb: Problem, W: np.ndarray) -> float:
    """Phi(W): scaled minimisation objective of paper eq. 1 (P=1) or eq. 4."""
    W = np.atleast_2d(W)
    val = 0.0
    for t in range(pb.P):
        x = W[t] - pb.c
        fx = pb.F.T @ x
        val += -pb.alpha[t] @ W[t] + pb.g1 * (fx @ pb.Omega @ fx + np.sum(pb.delta2 * x * x))
    u = np.abs(trades(pb, W))
    val += float(np.sum(pb.ca * u) + np.sum(pb.cb * u ** pb.d))
    return float(val)


def paper_objective(pb: Problem, W: np.ndarray) -> float:
    """The paper's reported objective (maximisation, eq. 1/eq. 4) without the constant
    GMV a_T^T w_T of the multi-period sum."""
    return -pb.GMV * objective(pb, W)


def K_apply(pb: Problem, W: np.ndarray):
    """(A w_t, G^T w_t, D W): D W stacks w_1, w_t - w_{t-1}, -w_{T-1} (multi-period)."""
    W = np.atleast_2d(W)
    zA = W @ pb.A.T
    zF = W @ pb.G
    if not pb.multi:
        zC = W.copy()
    else:
        zC = np.empty((pb.Tp, pb.n))
        zC[0] = W[0]
        if pb.P > 1:
            zC[1:pb.P] = W[1:] - W[:-1]
        zC[pb.P] = -W[pb.P - 1]
    return zA, zF, zC


def K_offset(pb: Problem):
    """b with K W - b = (A w_t, G^T (w_t - c), u_t)."""
    bA = np.zeros((pb.P, pb.m))
    bF = np.tile(pb.G.T @ pb.c, (pb.P, 1))
    bC = np.zeros((pb.Tp, pb.n))
    bC[0] = pb.w0
    if pb.multi:
        bC[pb.P] = -pb.wT
    return bA, bF, bC


def KT_apply(pb: Problem, yA, yF, yC) -> np.ndarray:
    """R_t = A^T y_A,t + G y_F,t + y_C,t - y_C,t+1 (single-period: + y_C)."""
    R = yA @ pb.A + yF @ pb.G.T
    if not pb.multi:
        return R + yC
    return R + yC[:pb.P] - yC[1:pb.P + 1]


def _support_box(y, L, U):
    """sum_j max(U_j y_j, L_j y_j), with 0 * inf = 0."""
    y = np.asarray(y, dtype=np.float64)
    pos = y > 0
    neg = y < 0
    return float(np.sum(U[pos] * y[pos]) + np.sum(L[neg] * y[neg]))


def project_dual_domain(pb: Problem, yA, yF, yC):
    """Nearest point of dom(h*): sign limits for infinite bounds, y_F = 0 if g1 = 0,
    |y_C| <= g2 s where the impact weight vanishes."""
    yA = np.array(yA, dtype=np.float64, copy=True)
    yF = np.array(yF, dtype=np.float64, copy=True)
    yC = np.array(yC, dtype=np.float64, copy=True)
    yA = np.where(np.isneginf(pb.L)[None, :], np.maximum(yA, 0.0), yA)
    yA = np.where(np.isposinf(pb.U)[None, :], np.minimum(yA, 0.0), yA)
    if pb.g1 <= 0:
        yF[:] = 0.0
    lin = pb.cb <= 0
    yC = np.where(lin, np.clip(yC, -pb.ca, pb.ca), yC)
    return yA, yF, yC


def dual_objective(pb: Problem, yA, yF, yC) -> float:
    """Psi(Y) of the module docstring (assumes Y in dom(h*); project first if unsure)."""
    yA = np.atleast_2d(yA); yF = np.atleast_2d(yF); yC = np.atleast_2d(yC)
    R = KT_apply(pb, yA, yF, yC)
    a = 2.0 * pb.g1 * pb.delta2
    val = 0.0
    for t in range(pb.P):
        b = pb.alpha[t] + a * pb.c - R[t]
        w, _ = l1_ball_quadratic(b, a)
        val += float(np.sum(0.5 * a * w * w - b * w)) + pb.g1 * float(np.sum(pb.delta2 * pb.c * pb.c))
        val -= _support_box(yA[t], pb.L, pb.U)
    Gc = pb.G.T @ pb.c
    val -= float(np.sum(yF @ Gc))
    if pb.g1 > 0:
        val -= float(np.sum(yF * yF)) / (4.0 * pb.g1)
    val -= float(yC[0] @ pb.w0)
    if pb.multi:
        val += float(yC[pb.P] @ pb.wT)
    val -= float(np.sum(conj_cost(yC, pb.ca, pb.cb, pb.d)))
    return float(val)


@dataclass
class KKT:
    rel_pri: float
    rel_dual: float
    rel_gap: float
    primal_obj: float
    dual_obj: float
    budget_excess: float

    @property
    def rel_kkt(self) -> float:
        return max(self.rel_pri, self.rel_dual, self.rel_gap)


def kkt(pb: Problem, W, yA, yF, yC) -> KKT:
    """Relative KKT error of a primal-dual pair.

    rel_pri  = ||[A W - clip(A W, L, U); (||w_t||_1 - 1)_+]|| / (1 + ||clip(A W, L, U)||)
    rel_dual = ||Y - proj_dom(Y)|| / (1 + ||Y||)
    rel_gap  = |Phi(W) - Psi(proj_dom(Y))| / (|Phi| + |Psi|)
    """
    W = np.atleast_2d(W)
    AW = W @ pb.A.T
    cl = np.clip(AW, pb.L[None, :], pb.U[None, :])
    bex = np.maximum(np.abs(W).sum(axis=1) - 1.0, 0.0)
    rp = np.sqrt(np.sum((AW - cl) ** 2) + np.sum(bex ** 2)) / (1.0 + np.linalg.norm(cl))
    pA, pF, pC = project_dual_domain(pb, yA, yF, yC)
    dres = np.sqrt(np.sum((pA - yA) ** 2) + np.sum((pF - yF) ** 2) + np.sum((pC - yC) ** 2))
    ynorm = np.sqrt(np.sum(np.square(yA)) + np.sum(np.square(yF)) + np.sum(np.square(yC)))
    rd = dres / (1.0 + ynorm)
    po = objective(pb, W)
    do = dual_objective(pb, pA, pF, pC)
    den = abs(po) + abs(do)
    rg = abs(po - do) / den if den > 0 else 0.0
    return KKT(rel_pri=float(rp), rel_dual=float(rd), rel_gap=float(rg), primal_obj=po,
               dual_obj=do, budget_excess=float(bex.max(initial=0.0)))
