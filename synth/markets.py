"""Seeded synthetic markets for the single-period and multi-period portfolio models.

Every function here draws from ``numpy.random.default_rng(seed)`` in a fixed order,
so an instance is a pure function of its arguments.  The arrays are float64 and
C-contiguous, in the layouts the solver's C interface uses:

* ``alpha``  [P][n]   P = 1 (single-period) or T-1 (decision periods 1..T-1)
* ``F``      [n][k]   factor loadings (the paper's beta)
* ``Omega``  [k][k]   factor covariance (the paper's Sigma_f)
* ``delta``  [n]      specific volatility, so D = diag(delta^2)
* ``s``, ``q`` [T'][n] spread and impact coefficients, T' = 1 or T (trades 1..T)
* ``A``      [m][n]   exposure rows: sector indicators, then factor-loading rows
* ``L``, ``U`` [m]    exposure bounds
* ``w0``     [n]      initial portfolio; ``w_target`` [n] terminal portfolio (multi-period)

Value distributions (all configs): F ~ N(0,1) with column 0 ~ N(1, 0.3) as a market
beta; Omega = diag(U(0.01,0.05)^2); delta ~ U(0.01,0.04); alpha ~ N(0, 1e-3^2);
s ~ U(5e-4, 2e-3); q ~ U(1e-4, 1e-3); w0 = 0.8 g/||g||_1 with g ~ N(0, I);
L, U = A w0 -/+ 0.05; d = 1.5, GMV = 1e9, lambda1 = 1e-9, lambda2 = lambda3 = 1.
The exposure matrix has m_sec = max(5, m-k) one-hot sector rows followed by the
first m - m_sec columns of F as factor-exposure rows.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["CONFIGS", "make_config", "make_single", "make_multi", "make_batch", "batch_instance",
           "ushape_profile_inputs", "make_tiny"]

# Sizes of the five standard workloads (see make_config).
CONFIGS = {
    0: dict(kind="single", n=500, k=20, m=10, seeds=(0,)),
    1: dict(kind="single", n=5000, k=60, m=80, seeds=tuple(range(1, 11))),
    2: dict(kind="multi", T=20, n=3000, k=50, m=50, seeds=(20,)),
    3: dict(kind="batch", B=256, n_lo=500, n_hi=8000, k=40, m=30, seeds=(30,)),
    4: dict(kind="multi", T=10, n=2000, k=40, m=40, seeds=(40,)),
}

_SCALARS = dict(d=1.5, GMV=1e9, lambda1=1e-9, lambda2=1.0, lambda3=1.0)


def _split_m(m: int, k: int) -> tuple[int, int]:
    m_sec = max(5, m - k)
    if m_sec > m:
        m_sec = m
    return m_sec, m - m_sec


def _universe(rng: np.random.Generator, n: int, k: int, m: int):
    """Draws 1-3 and 7 of the fixed order: loadings, factor covariance, specific vol."""
    F = rng.normal(0.0, 1.0, size=(n, k))
    if k > 0:
        F[:, 0] = rng.normal(1.0, 0.3, size=n)
    om = rng.uniform(0.01, 0.05, size=k) ** 2
    Omega = np.diag(om)
    delta = rng.uniform(0.01, 0.04, size=n)
    return F, Omega, delta


def _exposure(rng: np.random.Generator, F: np.ndarray, m: int):
    n, k = F.shape
    m_sec, m_fac = _split_m(m, k)
    sector = rng.integers(0, m_sec, size=n) if m_sec > 0 else np.zeros(n, dtype=np.int64)
    A = np.zeros((m, n))
    if m_sec > 0:
        A[sector, np.arange(n)] = 1.0
    if m_fac > 0:
        A[m_sec:, :] = F[:, :m_fac].T
    return A, sector


def _portfolio(rng: np.random.Generator, n: int, gross: float) -> np.ndarray:
    g = rng.normal(0.0, 1.0, size=n)
    return gross * g / np.abs(g).sum()


def make_single(n: int, k: int, m: int, seed: int, **overrides) -> dict:
    """One single-period instance (paper eq. 1-3) with the standard draw order."""
    rng = np.random.default_rng(seed)
    F, Omega, delta = _universe(rng, n, k, m)
    alpha = rng.normal(0.0, 1e-3, size=n)
    s = rng.uniform(5e-4, 2e-3, size=n)
    q = rng.uniform(1e-4, 1e-3, size=n)
    A, sector = _exposure(rng, F, m)
    w0 = _portfolio(rng, n, 0.8)
    c = A @ w0
    L, U = c - 0.05, c + 0.05
    out = dict(T=0, n=n, k=k, m=m, alpha=alpha[None, :].copy(), F=F, Omega=Omega, delta=delta,
               s=s[None, :].copy(), q=q[None, :].copy(), A=A, L=L, U=U, w0=w0, w_target=None,
               sector=sector, seed=seed, **_SCALARS)
    out.update(overrides)
    return _contig(out)


def make_multi(T: int, n: int, k: int, m: int, seed: int, **overrides) -> dict:
    """One multi-period instance (paper eq. 4-6).

    Per-period alpha_t = 0.9^t a_t with a_t ~ N(0, 1e-3^2 I) for t = 1..T-1; per-(t,i)
    multipliers U(0.8, 1.2) on s and q for every trade t = 1..T; terminal target
    w_target = 0.9 g'/||g'||_1.  For the differentiation workload a loss direction
    r ~ N(0, 1e-2^2) is drawn last (key ``r``).
    """
    rng = np.random.default_rng(seed)
    F, Omega, delta = _universe(rng, n, k, m)
    _alpha0 = rng.normal(0.0, 1e-3, size=n)  # drawn to keep the base order; unused
    s = rng.uniform(5e-4, 2e-3, size=n)
    q = rng.uniform(1e-4, 1e-3, size=n)
    A, sector = _exposure(rng, F, m)
    w0 = _portfolio(rng, n, 0.8)
    c = A @ w0
    L, U = c - 0.05, c + 0.05
    a = rng.normal(0.0, 1e-3, size=(T - 1, n))
    decay = 0.9 ** np.arange(1, T)
    alpha = decay[:, None] * a
    ms = rng.uniform(0.8, 1.2, size=(T, n))
    mq = rng.uniform(0.8, 1.2, size=(T, n))
    w_target = _portfolio(rng, n, 0.9)
    r = rng.normal(0.0, 1e-2, size=n)
    out = dict(T=T, n=n, k=k, m=m, alpha=alpha, F=F, Omega=Omega, delta=delta,
               s=s[None, :] * ms, q=q[None, :] * mq, A=A, L=L, U=U, w0=w0,
               w_target=w_target, r=r, sector=sector, seed=seed, **_SCALARS)
    out.update(overrides)
    return _contig(out)


def make_batch(B: int, k: int, m: int, seed: int, n_lo: int = 500, n_hi: int = 8000,
               n_max: int | None = None, **overrides) -> dict:
    """A batch of single-period instances sharing one asset universe.

    Instance b uses assets [0, n_b) of an ``n_max``-asset universe: the loadings,
    factor covariance, specific vols, sectors and exposure rows are shared; alpha,
    s, q, w0, L and U are per instance.  n_b = round(exp(U(ln n_lo, ln n_hi))).
    Per-instance vectors are packed back to back ("ragged") with offsets ``offs``.
    """
    rng = np.random.default_rng(seed)
    n_max = n_hi if n_max is None else n_max
    F, Omega, delta = _universe(rng, n_max, k, m)
    A, sector = _exposure(rng, F, m)
    n_b = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=B))).astype(np.int64)
    n_b = np.minimum(n_b, n_max)
    offs = np.zeros(B + 1, dtype=np.int64)
    offs[1:] = np.cumsum(n_b)
    tot = int(offs[-1])
    alpha = np.empty(tot); s = np.empty(tot); q = np.empty(tot); w0 = np.empty(tot)
    L = np.empty((B, m)); U = np.empty((B, m))
    for b in range(B):
        nb = int(n_b[b]); sl = slice(int(offs[b]), int(offs[b + 1]))
        alpha[sl] = rng.normal(0.0, 1e-3, size=nb)
        s[sl] = rng.uniform(5e-4, 2e-3, size=nb)
        q[sl] = rng.uniform(1e-4, 1e-3, size=nb)
        w0[sl] = _portfolio(rng, nb, 0.8)
        c = A[:, :nb] @ w0[sl]
        L[b], U[b] = c - 0.05, c + 0.05
    out = dict(B=B, n_b=n_b, offs=offs, n_max=n_max, k=k, m=m, F=F, Omega=Omega, delta=delta,
               A=A, sector=sector, alpha=alpha, s=s, q=q, w0=w0, L=L, U=U, seed=seed, **_SCALARS)
    out.update(overrides)
    return _contig(out)


def batch_instance(batch: dict, b: int) -> dict:
    """Instance b of a batch as a single-period instance dict (its prefix of the shared
    universe and its slice of the packed vectors)."""
    nb = int(batch["n_b"][b])
    lo, hi = int(batch["offs"][b]), int(batch["offs"][b + 1])
    out = dict(n=nb, k=batch["k"], m=batch["m"], T=0, F=batch["F"][:nb], Omega=batch["Omega"],
               delta=batch["delta"][:nb], A=batch["A"][:, :nb], alpha=batch["alpha"][lo:hi][None, :],
               s=batch["s"][lo:hi][None, :], q=batch["q"][lo:hi][None, :], w0=batch["w0"][lo:hi],
               L=batch["L"][b], U=batch["U"][b], w_target=None, seed=batch["seed"])
    for key in ("d", "GMV", "lambda1", "lambda2", "lambda3"):
        out[key] = batch[key]
    return _contig(out)


def make_config(i: int, seed: int | None = None, **overrides) -> dict:
    """Standard workload ``i`` (0..4) with its first seed unless ``seed`` is given.

    0: single-period, n=500, k=20, m=5+5, seed 0 (small case).
    1: single-period, n=5000, k=60, m=20+60, seeds 1..10.
    2: multi-period, T=20, n=3000, k=50, m=5+45, seed 20.
    3: batch of 256 single-period instances, n_b log-uniform in [500, 8000], k=40,
       m=5+25, one shared universe of 8000 assets, seed 30.
    4: multi-period, T=10, n=2000, k=40, m=5+35, seed 40 (differentiation workload).
    """
    c = CONFIGS[i]
    sd = c["seeds"][0] if seed is None else seed
    if c["kind"] == "single":
        return make_single(c["n"], c["k"], c["m"], sd, **overrides)
    if c["kind"] == "multi":
        return make_multi(c["T"], c["n"], c["k"], c["m"], sd, **overrides)
    return make_batch(c["B"], c["k"], c["m"], sd, n_lo=c["n_lo"], n_hi=c["n_hi"], **overrides)


def ushape_profile_inputs(inst: dict, norm_periods: int | None = None) -> dict:
    """Multi-period inputs with the paper's intraday cost profile (Section 3.4, eq. 7).

    alpha_t = alpha for every decision period, and s_t = eta_t / sum_k eta_k * s,
    q_t = eta_t / sum_k eta_k * q with eta_t = 0.5 + 2 (t/T - 0.5)^2.  The paper
    normalises over k = 1..T-1 while the model has T trades; ``norm_periods``
    selects the upper limit of that sum (default T-1, as printed).
    ``inst`` must be a multi-period instance; its s/q rows 0 are used as the base.
    """
    T = int(inst["T"])
    t = np.arange(1, T + 1, dtype=np.float64)
    eta = 0.5 + 2.0 * (t / T - 0.5) ** 2
    K = T - 1 if norm_periods is None else int(norm_periods)
    scale = eta / eta[:K].sum()
    base_s = inst["s"][0]
    base_q = inst["q"][0]
    out = dict(inst)
    out["alpha"] = np.repeat(inst["alpha"][:1], T - 1, axis=0)
    out["s"] = scale[:, None] * base_s[None, :]
    out["q"] = scale[:, None] * base_q[None, :]
    return _contig(out)


def _contig(d: dict) -> dict:
    for key, v in list(d.items()):
        if isinstance(v, np.ndarray):
            d[key] = np.ascontiguousarray(v)
    return d


def make_tiny(n: int, seed: int, k: int = 2, m: int = 1, T: int = 0, d: float = 1.5,
              alpha_scale: float = 3e-3, **overrides) -> dict:
    """A tiny instance (a handful of assets) with the standard value distributions,
    for brute-force checks.  The exposure rows are the net exposure (a row of ones)
    followed by factor-loading rows; bounds are A w0 -/+ 0.05."""
    rng = np.random.default_rng(seed)
    F, Omega, delta = _universe(rng, n, k, m)
    P = 1 if T == 0 else T - 1
    Tp = 1 if T == 0 else T
    alpha = rng.normal(0.0, alpha_scale, size=(P, n))
    s = rng.uniform(5e-4, 2e-3, size=(Tp, n))
    q = rng.uniform(1e-4, 1e-3, size=(Tp, n))
    A = np.zeros((m, n))
    if m >= 1:
        A[0] = 1.0
    for j in range(1, m):
        A[j] = F[:, (j - 1) % max(k, 1)] if k else rng.normal(size=n)
    w0 = _portfolio(rng, n, 0.8)
    c = A @ w0
    L, U = c - 0.05, c + 0.05
    w_target = _portfolio(rng, n, 0.9) if T else None
    out = dict(T=T, n=n, k=k, m=m, alpha=alpha, F=F, Omega=Omega, delta=delta, s=s, q=q, A=A,
               L=L, U=U, w0=w0, w_target=w_target, seed=seed, **dict(_SCALARS, d=d))
    out.update(overrides)
    return _contig(out)
