"""Synthetic stand-ins for the paper's own benchmark instances (paper Section 3 and 4.1).

The paper builds its instances from licensed data (CRSP prices and volumes,
OptionMetrics implied volatilities, Fama-French factor returns) that is not available
here.  These generators keep the shapes and the construction rules the paper states and
draw the market data from seeded distributions instead:

* risk model (Section 3.2): p = 6 factors (market + five Fama-French style factors) with a
  full factor covariance Sigma_f, loadings beta (market beta around 1, the others around
  0) and diagonal specific variances D; here drawn directly (the regression that builds
  them from a returns panel is ``returns_panel`` plus the risk-model step);
* alpha (Section 3.1): the mean of the next five daily returns plus 0.5 x a Gaussian with
  the stock's daily volatility, the returns simulated from the factor model;
* costs (Section 3.3): s the half bid-ask spread (relative), q = sigma (GMV/ADV)^(d-1)
  with ADV the average daily dollar volume;
* multi-period (Section 3.4): alpha_t = alpha, the same risk model every period, and
  s_t = eta_t / sum_k eta_k s, q_t likewise, with the U-shaped eta_t = 0.5 + 2 (t/T - 0.5)^2
  of eq. 7 for the trades t = 1..T, normalised over all T trades (so the costs of the
  whole path equal the single-period costs; the paper's sum stops at T-1);
* experiment grid (Section 4.1): lambda1 in {1e-8, ..., 1e-4}, lambda2 = lambda3 in
  {1, 10, 100, 1000, 10000}, 21 dates, T = 10.

The paper states no universe size, exposure rows, bounds, start portfolio or GMV; the
exposure rows here are one-hot sectors plus the six factor loadings, with bounds A w0
-/+ 0.05, w0 a random portfolio of gross exposure 0.8, and GMV = 1e9.  Nothing here
computes any part of the solver's method.
"""
from __future__ import annotations

import numpy as np

__all__ = ["LAMBDA1_GRID", "LAMBDA23_GRID", "N_DATES", "paper_instance", "eta_profile", "returns_panel"]

LAMBDA1_GRID = (1e-8, 1e-7, 1e-6, 1e-5, 1e-4)
LAMBDA23_GRID = (1.0, 10.0, 100.0, 1000.0, 10000.0)
N_DATES = 21
P_FACTORS = 6


def eta_profile(T: int) -> np.ndarray:
    """Per-trade scale eta_t / sum_k eta_k for t = 1..T, eta_t = 0.5 + 2 (t/T - 0.5)^2."""
    t = np.arange(1, T + 1, dtype=np.float64)
    eta = 0.5 + 2.0 * (t / T - 0.5) ** 2
    return eta / eta.sum()


def _factor_covariance(rng: np.random.Generator) -> np.ndarray:
    """A full 6 x 6 daily factor covariance: market vol ~1%, style factors ~0.3-0.8%,
    correlations from a random one-factor-plus-noise structure."""
    vol = np.concatenate([[rng.uniform(0.008, 0.012)], rng.uniform(0.003, 0.008, size=P_FACTORS - 1)])
    z = rng.normal(size=(P_FACTORS, 3))
    c = z @ z.T + np.diag(rng.uniform(0.5, 1.5, size=P_FACTORS))
    d = 1.0 / np.sqrt(np.diag(c))
    corr = c * d[:, None] * d[None, :]
    S = corr * vol[:, None] * vol[None, :]
    return 0.5 * (S + S.T)   # exactly symmetric


def paper_instance(date: int, n: int = 1000, lambda1: float = 1e-6, lambda23: float = 1.0, T: int = 0,
                   n_sectors: int = 10, seed: int = 2604) -> dict:
    """One instance of the paper's benchmark shape for a date index (0..20) of the grid.

    The market (risk model, alpha, costs, start portfolio) depends only on (seed, date, n);
    lambda1 and lambda2 = lambda3 select the grid point.  T = 0: single-period; T >= 2:
    multi-period over T trades (the paper uses T = 10)."""
    rng = np.random.default_rng([seed, date, n])
    # risk model: beta (market column around 1), full Sigma_f, specific variances
    beta = rng.normal(0.0, 0.5, size=(n, P_FACTORS))
    beta[:, 0] = rng.normal(1.0, 0.3, size=n)
    Sf = _factor_covariance(rng)
    spec = rng.uniform(0.01, 0.03, size=n)                  # specific daily vol, D = spec^2
    total_vol = np.sqrt(np.einsum("ij,jk,ik->i", beta, Sf, beta) + spec ** 2)
    # alpha: mean of the next five simulated daily returns + 0.5 x N(0, vol^2)
    Lf = np.linalg.cholesky(Sf)
    f = rng.normal(size=(5, P_FACTORS)) @ Lf.T
    r = f @ beta.T + rng.normal(size=(5, n)) * spec[None, :]
    alpha = r.mean(axis=0) + 0.5 * rng.normal(size=n) * total_vol
    # costs: half spread (relative), impact q = vol (GMV/ADV)^(d-1)
    GMV, d = 1e9, 1.5
    s = np.exp(rng.uniform(np.log(1e-4), np.log(1e-3), size=n))
    adv = np.exp(rng.uniform(np.log(2e7), np.log(2e10), size=n))
    q = total_vol * (GMV / adv) ** (d - 1.0)
    # exposure rows: one-hot sectors and the factor loadings; bounds around A w0
    sector = rng.integers(0, n_sectors, size=n)
    A = np.zeros((n_sectors + P_FACTORS, n))
    A[sector, np.arange(n)] = 1.0
    A[n_sectors:, :] = beta.T
    g = rng.normal(size=n)
    w0 = 0.8 * g / np.abs(g).sum()
    c = A @ w0
    L, U = c - 0.05, c + 0.05
    out = dict(T=T, n=n, k=P_FACTORS, m=A.shape[0], F=beta, Omega=Sf, delta=spec, A=A, L=L, U=U, w0=w0,
               d=d, GMV=GMV, lambda1=float(lambda1), lambda2=float(lambda23), lambda3=float(lambda23),
               sector=sector, seed=seed, date=date)
    if T == 0:
        out.update(alpha=alpha[None, :], s=s[None, :], q=q[None, :], w_target=None)
    else:
        scale = eta_profile(T)
        # terminal target: the start portfolio tilted toward alpha (gross 0.9)
        tgt = w0 + 0.5 * np.sign(alpha) * np.abs(w0).mean()
        out.update(alpha=np.repeat(alpha[None, :], T - 1, axis=0), s=scale[:, None] * s[None, :],
                   q=scale[:, None] * q[None, :], w_target=0.9 * tgt / np.abs(tgt).sum())
    for key, v in list(out.items()):
        if isinstance(v, np.ndarray):
            out[key] = np.ascontiguousarray(v)
    return out


def returns_panel(n: int, days: int = 504, seed: int = 7) -> dict:
    """A synthetic daily returns panel for the risk-model construction of Section 3.2:
    factor returns Fr [days][6] with a full covariance, true loadings beta [n][6],
    specific vols spec [n], asset returns R [days][n] = Fr beta^T + eps (eps ~ N(0, spec^2))
    plus a small factor mean.  The estimators recover beta, Sigma_f and D from (R, Fr)."""
    rng = np.random.default_rng([seed, n, days])
    Sf = _factor_covariance(rng)
    mean = rng.normal(0.0, 2e-4, size=P_FACTORS)
    Fr = rng.normal(size=(days, P_FACTORS)) @ np.linalg.cholesky(Sf).T + mean[None, :]
    beta = rng.normal(0.0, 0.5, size=(n, P_FACTORS))
    beta[:, 0] = rng.normal(1.0, 0.3, size=n)
    spec = rng.uniform(0.01, 0.03, size=n)
    R = Fr @ beta.T + rng.normal(size=(days, n)) * spec[None, :]
    return dict(R=np.ascontiguousarray(R), Fr=np.ascontiguousarray(Fr), beta=beta, Sigma_f=Sf, spec=spec,
                days=days, n=n, seed=seed)

