"""Pins of the oracle's risk-model construction (paper Section 3.2): closed forms, exact
recovery, the textbook covariance, invariances and the minimum-history rule."""
import numpy as np
import pytest

from oracle.riskmodel import risk_model
from synth import returns_panel


def _panel(days=120, n=30, p=6, seed=0):
    rng = np.random.default_rng(seed)
    Fr = rng.normal(0.0, 0.01, size=(days, p))
    beta = rng.normal(size=(n, p))
    return rng, Fr, beta


def test_noise_free_returns_are_recovered_exactly():
    rng, Fr, beta = _panel()
    R = Fr @ beta.T
    rm = risk_model(R, Fr)
    np.testing.assert_allclose(rm.beta, beta, rtol=0, atol=1e-10)
    assert np.all(rm.D <= 1e-24) and np.all(rm.valid)


def test_single_factor_closed_form():
    # p = 1, no intercept: beta = sum f r / sum f^2; D = variance of r - beta f
    rng = np.random.default_rng(1)
    f = rng.normal(0.0, 0.01, size=(200, 1))
    R = rng.normal(0.0, 0.02, size=(200, 5))
    rm = risk_model(R, f, min_obs=10)
    for i in range(5):
        b = float(np.sum(f[:, 0] * R[:, i]) / np.sum(f[:, 0] ** 2))
        assert rm.beta[i, 0] == pytest.approx(b, rel=1e-12)
        th = R[:, i] - b * f[:, 0]
        assert rm.D[i] == pytest.approx(np.sum((th - th.mean()) ** 2) / 199, rel=1e-12)


def test_factor_covariance_is_the_sample_covariance():
    rng, Fr, beta = _panel(days=300)
    rm = risk_model(Fr @ beta.T, Fr)
    np.testing.assert_allclose(rm.Sigma_f, np.cov(Fr, rowvar=False), rtol=1e-12, atol=0)


def test_scaling_and_factor_shift_invariances():
    rng, Fr, beta = _panel(days=150, n=12)
    R = Fr @ beta.T + rng.normal(0.0, 0.02, size=(150, 12))
    a = risk_model(R, Fr)
    b = risk_model(3.0 * R, Fr)
    np.testing.assert_allclose(b.beta, 3.0 * a.beta, rtol=1e-11)
    np.testing.assert_allclose(b.D, 9.0 * a.D, rtol=1e-11)
    # adding 0.7 f_2 to every asset's returns moves only the third loading
    c = risk_model(R + 0.7 * Fr[:, [2]], Fr)
    np.testing.assert_allclose(c.beta[:, 2], a.beta[:, 2] + 0.7, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(np.delete(c.beta, 2, axis=1), np.delete(a.beta, 2, axis=1), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(c.D, a.D, rtol=1e-10)


def test_residuals_are_orthogonal_to_the_factors():
    rng, Fr, beta = _panel(days=100, n=8)
    R = Fr @ beta.T + rng.normal(0.0, 0.02, size=(100, 8))
    M = rng.random((100, 8)) > 0.2
    rm = risk_model(R, Fr, mask=M, min_obs=20)
    for i in range(8):
        rows = M[:, i]
        th = R[rows, i] - Fr[rows] @ rm.beta[i]
        assert np.abs(Fr[rows].T @ th).max() <= 1e-14


def test_minimum_history_rule():
    rng, Fr, beta = _panel(days=100, n=4)
    R = Fr @ beta.T + rng.normal(0.0, 0.02, size=(100, 4))
    M = np.ones((100, 4), dtype=bool)
    M[:70, 1] = False            # 30 observed days < 42
    rm = risk_model(R, Fr, mask=M, min_obs=42)
    assert list(rm.valid) == [True, False, True, True]
    assert np.all(rm.beta[1] == 0.0)
    r = R[70:, 1]
    assert rm.D[1] == pytest.approx(np.sum((r - r.mean()) ** 2) / 29, rel=1e-12)
    assert rm.count[1] == 30


def test_recovers_the_true_model_statistically():
    """On a panel simulated from a known model the loadings' errors, scaled by their
    least-squares standard errors sqrt(D_i [(X^T X)^-1]_jj), are standard normal; the
    specific volatilities are recovered to a few percent."""
    P = returns_panel(n=300, days=504, seed=3)
    rm = risk_model(P["R"], P["Fr"])
    XtXi = np.linalg.inv(P["Fr"].T @ P["Fr"])
    se = np.sqrt(rm.D[:, None] * np.diag(XtXi)[None, :])
    z = ((rm.beta - P["beta"]) / se).ravel()
    assert abs(z.mean()) < 0.1 and 0.9 < z.std() < 1.1, (z.mean(), z.std())
    assert np.median(np.abs(np.sqrt(rm.D) / P["spec"] - 1.0)) < 0.05
