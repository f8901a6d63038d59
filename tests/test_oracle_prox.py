"""Pins for the oracle's one-dimensional primitives (cost prox, conjugate, L1 budget).

Each primitive is checked against something other than its own formula: numeric 1-D
minimisation/maximisation with SciPy, the exact optimality condition, the Fenchel-Young
equality, the Moreau decomposition, and two independent L1-ball algorithms (Michelot's
and bisection on the multiplier).
"""
import numpy as np
import pytest
from scipy.optimize import minimize_scalar

from oracle.prox import prox_cost, conj_cost, cost, dcost, l1_ball_quadratic, l1_quadratic_value

RNG = np.random.default_rng(1234)


def _numeric_prox(v, t, a, b, d):
    f = lambda x: 0.5 * (x - v) ** 2 + t * (a * abs(x) + b * abs(x) ** d)
    lo, hi = -abs(v) - 1.0, abs(v) + 1.0
    r = minimize_scalar(f, bounds=(lo, hi), method="bounded", options={"xatol": 1e-14, "maxiter": 2000})
    # compare also with 0, which the bounded search may miss by xatol
    return r.x if f(r.x) < f(0.0) else 0.0


@pytest.mark.parametrize("d", [2.0, 1.5, 1.3, 1.75])
def test_prox_matches_numeric_minimisation(d):
    for _ in range(200):
        v = RNG.normal() * 10 ** RNG.uniform(-4, 0)
        t = 10 ** RNG.uniform(-2, 2)
        a = RNG.uniform(0, 2e-3)
        b = RNG.uniform(0, 1e-3) * 10 ** RNG.uniform(0, 3)
        x = float(prox_cost(np.array([v]), t, a, b, d)[0])
        xn = _numeric_prox(v, t, a, b, d)
        f = lambda z: 0.5 * (z - v) ** 2 + t * (a * abs(z) + b * abs(z) ** d)
        assert f(x) <= f(xn) + 1e-15 * max(1.0, abs(f(xn))) + 1e-24
        assert abs(x - xn) <= 1e-6 * max(1e-3, abs(v))


@pytest.mark.parametrize("d", [2.0, 1.5, 1.3])
def test_prox_optimality_condition(d):
    """x = 0 iff |v| <= t a; otherwise (v - x)/t = sign(x)(a + b d |x|^(d-1)) exactly."""
    v = RNG.normal(size=5000) * 10 ** RNG.uniform(-4, 0, size=5000)
    t = 10 ** RNG.uniform(-2, 2, size=5000)
    a = RNG.uniform(0, 2e-3, size=5000)
    b = RNG.uniform(0, 1e-3, size=5000) * 10 ** RNG.uniform(0, 3, size=5000)
    x = prox_cost(v, t, a, b, d)
    dead = np.abs(v) <= t * a
    assert np.all(x[dead] == 0.0)
    nz = ~dead & (np.abs(x) > 0)
    lhs = (v[nz] - x[nz]) / t[nz]
    rhs = np.sign(x[nz]) * (a[nz] + b[nz] * d * np.abs(x[nz]) ** (d - 1))
    tol = 1e-12 if d in (2.0, 1.5) else 1e-9
    assert np.all(np.abs(lhs - rhs) <= tol * (np.abs(v[nz]) / t[nz] + a[nz]))
    assert np.all(np.sign(x[nz]) == np.sign(v[nz]))


def test_prox_nonexpansive():
    v1 = RNG.normal(size=2000) * 1e-2
    v2 = v1 + RNG.normal(size=2000) * 1e-3
    for d in (1.5, 2.0):
        x1 = prox_cost(v1, 0.7, 1e-3, 5e-4, d)
        x2 = prox_cost(v2, 0.7, 1e-3, 5e-4, d)
        assert np.all(np.abs(x1 - x2) <= np.abs(v1 - v2) * (1 + 1e-14))


@pytest.mark.parametrize("d", [2.0, 1.5, 1.2])
def test_conjugate_matches_numeric_sup(d):
    for _ in range(200):
        a = RNG.uniform(0, 2e-3)
        b = 10 ** RNG.uniform(-5, -2)
        e = RNG.normal() * 4e-3
        val = float(conj_cost(np.array([e]), a, b, d)[0])
        # beyond |u| = (|e|/b)^(1/(d-1)) the objective e u - b|u|^d is negative
        B = 2.0 * (abs(e) / b) ** (1.0 / (d - 1.0)) + 1e-12
        r = minimize_scalar(lambda u: -(e * u - a * abs(u) - b * abs(u) ** d), bounds=(-B, B),
                            method="bounded", options={"xatol": 1e-13 * B, "maxiter": 5000})
        num = max(-r.fun, 0.0)
        assert abs(val - num) <= 1e-9 * max(abs(num), 1e-12)


def test_conjugate_infinite_without_impact():
    assert np.isinf(conj_cost(np.array([2e-3]), 1e-3, 0.0, 1.5)[0])
    assert conj_cost(np.array([5e-4]), 1e-3, 0.0, 1.5)[0] == 0.0


@pytest.mark.parametrize("d", [2.0, 1.5])
def test_fenchel_young_equality(d):
    x = RNG.normal(size=1000) * 1e-2
    a = RNG.uniform(0, 2e-3, size=1000)
    b = RNG.uniform(1e-4, 1e-3, size=1000)
    y = dcost(x, a, b, d)
    lhs = cost(x, a, b, d) + conj_cost(y, a, b, d)
    assert np.allclose(lhs, x * y, rtol=1e-11, atol=1e-20)


@pytest.mark.parametrize("d", [2.0, 1.5])
def test_moreau_decomposition(d):
    """prox_{t c}(v) + t prox_{c*/t}(v/t) = v, with the conjugate prox found numerically."""
    for _ in range(50):
        v = RNG.normal() * 1e-2
        t = 10 ** RNG.uniform(-1, 1)
        a, b = RNG.uniform(0, 2e-3), RNG.uniform(1e-4, 1e-3)
        p = float(prox_cost(np.array([v]), t, a, b, d)[0])
        g = lambda z: float(conj_cost(np.array([z]), a, b, d)[0]) / t + 0.5 * (z - v / t) ** 2
        r = minimize_scalar(g, bounds=(-abs(v / t) - 1, abs(v / t) + 1), method="bounded",
                            options={"xatol": 1e-14, "maxiter": 5000})
        assert abs(p + t * r.x - v) <= 1e-8 * max(abs(v), 1e-6)


def _michelot(b, a):
    """Michelot (1986) style: iterate mu on the current support until it stops changing."""
    ab = np.abs(b)
    if np.sum(ab / a) <= 1:
        return b / a
    sup = np.ones_like(ab, dtype=bool)
    for _ in range(1000):
        mu = (np.sum(ab[sup] / a[sup]) - 1.0) / np.sum(1.0 / a[sup])
        new = ab > mu
        if np.array_equal(new, sup):
            break
        sup = new
    return np.sign(b) * np.maximum(ab - mu, 0.0) / a


def _bisect(b, a):
    ab = np.abs(b)
    if np.sum(ab / a) <= 1:
        return b / a
    lo, hi = 0.0, ab.max()
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if np.sum(np.maximum(ab - mid, 0) / a) > 1:
            lo = mid
        else:
            hi = mid
    mu = 0.5 * (lo + hi)
    return np.sign(b) * np.maximum(ab - mu, 0.0) / a


@pytest.mark.parametrize("n", [1, 2, 7, 100, 5000])
def test_l1_ball_three_algorithms(n):
    for _ in range(5):
        b = RNG.normal(size=n) * 10 ** RNG.uniform(-3, 1)
        a = 10 ** RNG.uniform(-2, 2, size=n)
        w, mu = l1_ball_quadratic(b, a)
        assert np.allclose(w, _michelot(b, a), rtol=1e-10, atol=1e-13)
        assert np.allclose(w, _bisect(b, a), rtol=1e-9, atol=1e-12)
        if mu > 0:
            assert abs(np.abs(w).sum() - 1.0) <= 1e-12
        else:
            assert np.abs(w).sum() <= 1.0 + 1e-12


def test_l1_ball_optimal_against_random_feasible_points():
    n = 30
    b = RNG.normal(size=n)
    a = RNG.uniform(0.5, 2.0, size=n)
    val, w, _ = l1_quadratic_value(b, a)
    for _ in range(2000):
        z = RNG.normal(size=n)
        z /= max(1.0, np.abs(z).sum()) * RNG.uniform(1.0, 3.0)
        assert np.sum(0.5 * a * z * z - b * z) >= val - 1e-14


def _duchi_projection(v):
    """Euclidean projection onto the unit L1 ball (Duchi et al. 2008, sort-based)."""
    if np.abs(v).sum() <= 1:
        return v.copy()
    u = np.sort(np.abs(v))[::-1]
    cs = np.cumsum(u)
    j = np.arange(1, len(u) + 1)
    rho = np.nonzero(u * j > (cs - 1.0))[0][-1]
    theta = (cs[rho] - 1.0) / (rho + 1.0)
    return np.sign(v) * np.maximum(np.abs(v) - theta, 0.0)


def test_l1_uniform_weights_is_euclidean_projection():
    for _ in range(20):
        v = RNG.normal(size=50) * 0.3
        w, _ = l1_ball_quadratic(v, np.ones(50))
        assert np.allclose(w, _duchi_projection(v), atol=1e-14)


def test_l1_linear_entries_value_is_minus_max():
    b = RNG.normal(size=20)
    val, w, mu = l1_quadratic_value(b, np.zeros(20))
    assert abs(val + np.abs(b).max()) <= 1e-15
    assert abs(np.abs(w).sum() - 1.0) <= 1e-15 and mu == np.abs(b).max()
