"""One-dimensional building blocks of the oracle (plain FP64 NumPy).

Cost of a trade u (paper Section 2.1, eq. 1: the bid-offer term s|u| and the market
impact term q|u|^d, 1 < d <= 2), after scaling by the penalty weights:

    c(u) = a |u| + b |u|^d,  a = g2 s >= 0,  b = g3 q >= 0.

Proximal map of t c:   prox(v) = argmin_x 1/2 (x - v)^2 + t c(x).
Shrinking by t a first, the magnitude rho = |x| solves rho + t b d rho^(d-1) = r with
r = max(|v| - t a, 0); x = sign(v) rho.  At d = 2 that is linear; at d = 3/2 it is a
quadratic in sqrt(rho); any other d is solved by bisection (rho lies in [0, r]).

Conjugate of c:  c*(e) = sup_u e u - c(u) = 0 for |e| <= a, otherwise with
r = |e| - a the maximiser is u = (r/(b d))^(1/(d-1)) and c*(e) = ((d-1)/d) r u
(+inf when b = 0 and |e| > a).

Budget (paper eq. 3) with a diagonal quadratic: minimise sum_i (a_i/2 w_i^2 - b_i w_i)
over ||w||_1 <= 1, a_i > 0.  The solution is w_i = sign(b_i) max(|b_i| - mu, 0)/a_i with
mu = 0 if sum |b_i|/a_i <= 1, else the unique mu > 0 with sum max(|b_i| - mu, 0)/a_i = 1,
found here by sorting the breakpoints |b_i| (a different algorithm from the GPU's).
"""
from __future__ import annotations

import numpy as np

__all__ = ["cost", "prox_cost", "conj_cost", "dcost", "l1_ball_quadratic", "l1_quadratic_value",
           "box"]


def cost(u, a, b, d):
    """c(u) = a|u| + b|u|^d, elementwise."""
    au = np.abs(u)
    return a * au + b * au ** d


def dcost(u, a, b, d):
    """Derivative of c at u != 0: sign(u) (a + b d |u|^(d-1))."""
    au = np.abs(u)
    return np.sign(u) * (a + b * d * au ** (d - 1.0))


def _rho_bisect(r, tb, d, iters=200):
    """Root of rho + tb d rho^(d-1) = r on [0, r] by bisection (monotone in rho)."""
    lo = np.zeros_like(r)
    hi = r.copy()
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        f = mid + tb * d * mid ** (d - 1.0) - r
        pos = f > 0
        hi = np.where(pos, mid, hi)
        lo = np.where(pos, lo, mid)
    return 0.5 * (lo + hi)


def prox_cost(v, t, a, b, d):
    """argmin_x 1/2 (x - v)^2 + t (a|x| + b|x|^d), elementwise; t > 0, a, b >= 0."""
    v = np.asarray(v, dtype=np.float64)
    t = np.broadcast_to(np.asarray(t, dtype=np.float64), v.shape)
    a = np.broadcast_to(np.asarray(a, dtype=np.float64), v.shape)
    b = np.broadcast_to(np.asarray(b, dtype=np.float64), v.shape)
    r = np.maximum(np.abs(v) - t * a, 0.0)
    tb = t * b
    if d == 2.0:
        rho = r / (1.0 + 2.0 * tb)
    elif d == 1.5:
        # rho = u^2 with u^2 + c u - r = 0, c = 1.5 tb; take the nonnegative root,
        # written without cancellation.
        c = 1.5 * tb
        den = c + np.sqrt(c * c + 4.0 * r)
        u = np.where(r > 0, 2.0 * r / np.where(r > 0, den, 1.0), 0.0)
        rho = u * u
    else:
        rho = _rho_bisect(r, tb, d)
    return np.sign(v) * rho


def conj_cost(e, a, b, d):
    """c*(e) = sup_u e u - a|u| - b|u|^d, elementwise (may be +inf when b = 0)."""
    e = np.asarray(e, dtype=np.float64)
    a = np.broadcast_to(np.asarray(a, dtype=np.float64), e.shape)
    b = np.broadcast_to(np.asarray(b, dtype=np.float64), e.shape)
    r = np.maximum(np.abs(e) - a, 0.0)
    out = np.zeros_like(e)
    pos = r > 0
    bz = pos & (b <= 0)
    out[bz] = np.inf
    ok = pos & (b > 0)
    if np.any(ok):
        rr = r[ok]
        u = (rr / (b[ok] * d)) ** (1.0 / (d - 1.0))
        out[ok] = (d - 1.0) / d * rr * u
    return out


def _l1_root_sorted(ab, av):
    """Root mu > 0 of sum max(|b| - mu, 0)/a = 1 over entries with a > 0 (sum |b|/a > 1)."""
    order = np.argsort(-ab, kind="stable")
    bs = ab[order]
    inv = 1.0 / av[order]
    num = np.cumsum(bs * inv) - 1.0
    den = np.cumsum(inv)
    mus = num / den
    nxt = np.append(bs[1:], 0.0)
    # first j where mu_j >= next breakpoint (and mu_j < current breakpoint holds by construction)
    ok = np.nonzero(mus >= nxt)[0]
    return float(mus[int(ok[0])])


def l1_ball_quadratic(bv, av):
    """Minimise sum(a/2 w^2 - b w) over ||w||_1 <= 1 (a >= 0); returns (w, mu).

    Sort-based: with the breakpoints |b| in decreasing order, the active set for the
    root mu is a prefix; mu_j = (sum_{top j} |b|/a - 1) / (sum_{top j} 1/a) is valid for
    the first j at which it is no smaller than the (j+1)-th breakpoint.

    Entries with a_i = 0 are linear: they force mu >= beta = max_{a_i=0} |b_i|.  If the
    quadratic entries alone use less than the whole budget at mu = beta, then mu = beta
    and the rest of the budget goes to one linear entry of largest |b| (the minimiser is
    then not unique; the value is).
    """
    bv = np.asarray(bv, dtype=np.float64)
    av = np.asarray(av, dtype=np.float64)
    ab = np.abs(bv)
    quad = av > 0
    if np.all(quad):
        if np.sum(ab / av) <= 1.0:
            return bv / av, 0.0
        mu = _l1_root_sorted(ab, av)
        w = np.sign(bv) * np.maximum(ab - mu, 0.0) / av
        return w, mu
    lin = ~quad
    beta = float(np.max(ab[lin]))
    w = np.zeros_like(bv)
    aq = av[quad]
    bq = ab[quad]
    used = float(np.sum(np.maximum(bq - beta, 0.0) / aq)) if aq.size else 0.0
    if used >= 1.0 and aq.size:
        mu = _l1_root_sorted(bq, aq)
        w[quad] = np.sign(bv[quad]) * np.maximum(bq - mu, 0.0) / aq
        return w, mu
    mu = beta
    if aq.size:
        w[quad] = np.sign(bv[quad]) * np.maximum(bq - mu, 0.0) / aq
    if beta > 0:
        idx = np.nonzero(lin)[0]
        j = int(idx[np.argmax(ab[lin])])
        w[j] = np.sign(bv[j]) * (1.0 - used)
    return w, mu


def l1_quadratic_value(bv, av):
    """Minimum value of sum(a/2 w^2 - b w) over ||w||_1 <= 1 and its minimiser."""
    w, mu = l1_ball_quadratic(bv, av)
    return float(np.sum(0.5 * av * w * w - bv * w)), w, mu


def box(v, lo, hi):
    """Projection onto [lo, hi] (infinite bounds allowed)."""
    return np.minimum(np.maximum(v, lo), hi)
