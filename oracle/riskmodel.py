"""Risk-model construction of paper Section 3.2 (plain FP64; test infrastructure only).

From a window of daily factor returns Fr (days x p) and asset returns R (days x n):

* loadings: for every asset i with at least ``min_obs`` observed days, beta_i is the
  least-squares solution of r_i ~ Fr beta_i over its observed days (the paper regresses
  the returns on the factor returns without an intercept); assets with fewer
  observations get no loadings (valid = False, beta_i = 0);
* factor covariance: Sigma_f = (Fr - 1 mean^T)^T (Fr - 1 mean^T) / (days - 1) over the
  whole window;
* specific variances: theta_k = r_ki - beta_i^T f_k on the observed days and
  D_ii = sum_k (theta_k - mean theta)^2 / (count - 1) (for an asset without loadings the
  residual is its return).

The model is then Sigma = beta Sigma_f beta^T + D, i.e. the solver's F = beta,
Omega = Sigma_f and delta = sqrt(D).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = ["RiskModel", "risk_model"]


@dataclass
class RiskModel:
    beta: np.ndarray      # (n, p)
    Sigma_f: np.ndarray   # (p, p)
    D: np.ndarray         # (n,)
    valid: np.ndarray     # (n,) bool
    count: np.ndarray     # (n,) observed days


def risk_model(R, Fr, mask=None, min_obs: int = 42) -> RiskModel:
    R = np.asarray(R, dtype=np.float64)
    Fr = np.asarray(Fr, dtype=np.float64)
    days, n = R.shape
    p = Fr.shape[1]
    M = np.ones((days, n), dtype=bool) if mask is None else np.asarray(mask).astype(bool)
    Fc = Fr - Fr.mean(axis=0, keepdims=True)
    Sigma_f = Fc.T @ Fc / (days - 1)
    beta = np.zeros((n, p))
    D = np.zeros(n)
    valid = np.zeros(n, dtype=bool)
    count = M.sum(axis=0)
    for i in range(n):
        rows = M[:, i]
        r = R[rows, i]
        X = Fr[rows]
        if count[i] >= max(min_obs, p + 1):
            # normal equations of the least-squares fit over the observed days
            b = np.linalg.solve(X.T @ X, X.T @ r)
            beta[i] = b
            valid[i] = True
            theta = r - X @ b
        else:
            theta = r
        if count[i] >= 2:
            D[i] = np.sum((theta - theta.mean()) ** 2) / (count[i] - 1)
        else:
            D[i] = 0.0
    return RiskModel(beta=beta, Sigma_f=Sigma_f, D=D, valid=valid, count=count)
