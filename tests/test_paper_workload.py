"""CPU checks of the paper-shaped workload generator (paper Section 3 and 4.1) and of the
Table 1 reporting (SGM1), against facts the paper fixes."""
import numpy as np
import pytest

import oracle
from oracle.problem import normalize
from synth import LAMBDA1_GRID, LAMBDA23_GRID, N_DATES, eta_profile, paper_instance


def test_grid_is_the_papers():
    assert LAMBDA1_GRID == (1e-8, 1e-7, 1e-6, 1e-5, 1e-4)
    assert LAMBDA23_GRID == (1.0, 10.0, 100.0, 1000.0, 10000.0)
    assert N_DATES == 21


def test_u_shaped_profile():
    # eq. 7: eta_t = 0.5 + 2 (t/T - 0.5)^2, here normalised over the T trades
    T = 10
    e = eta_profile(T)
    raw = np.array([0.5 + 2.0 * (t / T - 0.5) ** 2 for t in range(1, T + 1)])
    np.testing.assert_allclose(e, raw / raw.sum(), rtol=1e-15)
    assert abs(e.sum() - 1.0) < 1e-15
    # U shape: decreasing to the middle, then increasing; minimum 0.5 at t = T/2
    assert np.all(np.diff(e[:5]) < 0) and np.all(np.diff(e[4:]) > 0)
    assert raw[4] == 0.5


@pytest.mark.parametrize("T", [0, 10])
def test_instance_shape_and_model(T):
    inst = paper_instance(3, n=120, lambda1=1e-6, lambda23=10.0, T=T)
    n, k = 120, 6
    assert inst["F"].shape == (n, k) and inst["Omega"].shape == (k, k)
    # the factor covariance is full (not diagonal), symmetric and positive definite
    Om = inst["Omega"]
    assert np.abs(Om - np.diag(np.diag(Om))).max() > 0
    np.testing.assert_array_equal(Om, Om.T)
    assert np.linalg.eigvalsh(Om).min() > 0
    P = 1 if T == 0 else T - 1
    Tp = 1 if T == 0 else T
    assert inst["alpha"].shape == (P, n) and inst["s"].shape == (Tp, n)
    if T:
        # constant alpha across periods; costs scaled by the U-shaped profile, whose sum
        # over the T trades is the single-period cost
        np.testing.assert_array_equal(inst["alpha"], np.repeat(inst["alpha"][:1], P, axis=0))
        sp = paper_instance(3, n=120, lambda1=1e-6, lambda23=10.0, T=0)
        np.testing.assert_allclose(inst["s"].sum(axis=0), sp["s"][0], rtol=1e-14)
        np.testing.assert_allclose(inst["q"].sum(axis=0), sp["q"][0], rtol=1e-14)
        np.testing.assert_array_equal(inst["alpha"][0], sp["alpha"][0])
    # the market is the same at every grid point of a date
    other = paper_instance(3, n=120, lambda1=1e-4, lambda23=1e4, T=T)
    np.testing.assert_array_equal(other["F"], inst["F"])
    assert other["lambda1"] == 1e-4 and other["lambda2"] == other["lambda3"] == 1e4
    # impact q = vol (GMV / ADV)^(d - 1) > 0, spreads in [1, 10] bp
    assert np.all(inst["q"] > 0) and np.all((inst["s"] > 0))
    # the start portfolio is feasible: the box is centred on A w0
    np.testing.assert_allclose(inst["A"] @ inst["w0"], 0.5 * (inst["L"] + inst["U"]), atol=1e-15)


def test_no_trade_at_huge_cost_weight():
    # lambda2 = lambda3 = 1e4 with lambda1 = 1e-8: the cost-free gain of moving is far
    # smaller than the spread, so the optimum stays (within rounding) at w0
    inst = paper_instance(0, n=150, lambda1=1e-8, lambda23=1e4, T=0)
    r = oracle.solve(inst, tol=1e-10)
    assert r.polished
    assert np.abs(r.W[0] - inst["w0"]).max() <= 1e-12


def test_sgm1_definition():
    import bench
    assert bench.sgm1([2.0, 2.0, 2.0]) == pytest.approx(2.0, rel=1e-15)
    # (prod (t_i + 1))^(1/n) - 1
    t = [0.1, 0.5, 3.0]
    assert bench.sgm1(t) == pytest.approx((1.1 * 1.5 * 4.0) ** (1 / 3) - 1.0, rel=1e-14)
    assert bench.sgm1([0.0]) == 0.0
