"""The oracle against exact active-set enumeration (oracle/enumerate.py), the brute-force
pin of the optimum at up to eight assets (paper eq. 1-3 and 4-6).

The enumeration forms Sigma = F Omega F^T + diag(delta^2) explicitly and solves every
piece's equality-constrained optimality system (linear at d = 2, Newton otherwise), so
it shares nothing with the oracle's splitting, dual, prox maps or polish. At d = 2 both
sides are exact up to rounding, so the bar is 1e-12; at d != 2 the enumeration's Newton
solves bound it at 1e-9. Each case also checks that the instance exercises what the
pin is for: zero trades, active exposure rows, a tight budget with a zero weight."""
import numpy as np
import pytest

import oracle
from oracle.enumerate import active_set_enumeration
from synth.markets import make_tiny


def _compare(inst, w_tol, require_polish=True):
    r = active_set_enumeration(inst)
    o = oracle.solve(inst, tol=1e-10, require_polish=require_polish)
    assert r.consistent >= 1 and r.spread <= 1e-13
    assert np.max(np.abs(o.W - r.W)) <= w_tol, np.max(np.abs(o.W - r.W))
    assert abs(o.phi - r.phi) <= 1e-12 * abs(r.phi)
    return r


def _features(inst, W):
    W = np.atleast_2d(W)
    u = W[0] - inst["w0"]
    aw = np.atleast_2d(W) @ inst["A"].T if inst["A"].size else np.zeros((W.shape[0], 0))
    active = np.sum((np.abs(aw - inst["L"]) <= 1e-12) | (np.abs(aw - inst["U"]) <= 1e-12))
    return int(np.sum(np.abs(u) <= 1e-13)), int(active), int(np.sum(np.abs(W) <= 1e-13))


@pytest.mark.parametrize("seed,lambda1", [(1, 2e-8), (3, 5e-8)])
def test_eight_assets_two_rows(seed, lambda1):
    # 3^8 trade states x 3^2 row states, budget slack: 59,049 pieces, exactly one consistent
    inst = make_tiny(8, seed=seed, k=2, m=2, d=2.0, lambda1=lambda1)
    r = _compare(inst, 1e-12)
    assert r.pieces == 59049 and r.consistent == 1 and r.budget_tight == (False,)
    zero_trades, active_rows, _ = _features(inst, r.W)
    assert zero_trades >= 1 and active_rows >= 1


@pytest.mark.parametrize("seed", [1, 2])
def test_tight_budget_five_assets(seed):
    inst = make_tiny(5, seed=seed, k=2, m=2, d=2.0)
    r = _compare(inst, 1e-12)
    assert r.consistent == 1 and r.budget_tight == (True,)
    assert abs(np.abs(r.W).sum() - 1.0) <= 1e-13
    assert _features(inst, r.W)[2] >= 1          # a weight at zero under the tight budget


def test_three_halves_impact_six_assets():
    inst = make_tiny(6, seed=0, k=2, m=2, d=1.5, lambda1=3e-8)
    r = _compare(inst, 1e-9)
    assert r.consistent == 1


def test_three_halves_impact_tight_budget():
    inst = make_tiny(4, seed=0, k=2, m=1, d=1.5)
    r = _compare(inst, 1e-9)
    assert r.consistent == 1 and r.budget_tight == (True,)


def test_general_exponent():
    # d = 1.3: the oracle's prox takes its safeguarded Newton path
    inst = make_tiny(5, seed=1, k=2, m=1, d=1.3, lambda1=3e-8)
    r = _compare(inst, 1e-9)
    assert r.consistent == 1


@pytest.mark.parametrize("seed", [40, 41])
def test_multi_period_tight_budgets(seed):
    # T = 3 (two decisions, three trades), both budgets tight, a weight at zero
    inst = make_tiny(2, seed=seed, k=1, m=0, T=3, d=2.0, alpha_scale=2e-2)
    r = _compare(inst, 1e-12)
    assert r.consistent == 1 and r.budget_tight == (True, True)
    assert np.sum(np.abs(r.W) <= 1e-13) >= 1


def test_multi_period_with_a_row_three_halves():
    inst = make_tiny(2, seed=20, k=1, m=1, T=3, d=1.5)
    r = _compare(inst, 1e-9)
    assert r.consistent == 1


def test_degenerate_case_has_one_solution_on_two_pieces():
    """A multiplier exactly at its limit: two pieces are consistent and give the same W*.
    The oracle's polish cannot certify this case (its sign chain is ambiguous), so the
    comparison takes the oracle's PDHG iterate at relative KKT 1e-10."""
    inst = make_tiny(2, seed=21, k=1, m=1, T=3, d=2.0)
    r = active_set_enumeration(inst)
    assert r.consistent == 2 and r.spread <= 1e-14
    o = oracle.solve(inst, tol=1e-10, require_polish=False)
    assert np.max(np.abs(o.W - r.W)) <= 1e-10
