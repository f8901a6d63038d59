"""Pins of oracle.feasibility: the minimal budget of the exposure box (a linear program)
and the infeasibility certificate value (paper Section 2.1 eq. 2-3: the box L <= A w <= U
and the budget ||w||_1 <= 1)."""
import numpy as np
import pytest
from scipy.optimize import linprog

from oracle.feasibility import certificate_value, is_feasible, min_budget
from synth import make_config, make_single


def _sector_row_target(inst, value):
    """Set the first sector row (one-hot) to L = U = value."""
    out = dict(inst)
    out["L"] = inst["L"].copy()
    out["U"] = inst["U"].copy()
    out["L"][0] = out["U"][0] = value
    return out


def test_min_budget_of_one_sector_row_is_its_target():
    # a one-hot row j with L_j = U_j = 1.5: the cheapest w puts 1.5 on one member of the
    # sector, and no w with A_j w = 1.5 has ||w||_1 < 1.5; every other row of this small
    # instance stays satisfiable alongside
    inst = make_single(40, 0, 1, seed=3)
    inst = _sector_row_target(inst, 1.5)
    assert min_budget(inst) == pytest.approx(1.5, rel=1e-9)
    assert not is_feasible(inst)


def test_hand_certificate_for_the_sector_row():
    inst = _sector_row_target(make_single(40, 0, 1, seed=3), 1.5)
    y = np.array([-1.0])
    # sum_j max(U y, L y) = -1.5; ||A^T y||_inf = 1 (one-hot row)
    assert certificate_value(inst, y) == pytest.approx(-0.5, abs=1e-15)


def test_two_conflicting_sector_rows():
    inst = make_single(60, 0, 2, seed=4)            # two one-hot sector rows
    inst = dict(inst)
    inst["L"] = np.array([0.6, 0.6])
    inst["U"] = np.array([0.7, 0.7])
    # disjoint sectors each need >= 0.6 of gross exposure: min budget exactly 1.2
    assert min_budget(inst) == pytest.approx(1.2, rel=1e-9)
    assert certificate_value(inst, [-1.0, -1.0]) == pytest.approx(-0.2, abs=1e-15)


def test_feasible_markets_have_the_start_portfolio_inside():
    # L, U = A w0 -/+ 0.05 and ||w0||_1 = 0.8, so the minimal budget is at most 0.8
    inst = make_config(0)
    assert min_budget(inst) <= 0.8 + 1e-9
    assert is_feasible(inst)


def test_no_certificate_exists_for_a_feasible_set():
    inst = make_config(0)
    rng = np.random.default_rng(0)
    for _ in range(300):
        y = rng.normal(size=inst["A"].shape[0]) * 10.0 ** rng.uniform(-3, 3)
        assert certificate_value(inst, y) >= -1e-12 * (1.0 + np.abs(y).sum())


def test_lp_dual_gives_a_certificate_when_infeasible():
    # LP duality: min ||w||_1 s.t. A w = b equals max b^T z s.t. ||A^T z||_inf <= 1, so a
    # minimal budget above 1 yields y = -z with sum max(U y, L y) + ||A^T y||_inf < 0
    inst = make_single(30, 3, 6, seed=8)
    inst = dict(inst)
    inst["L"] = inst["U"] = np.asarray(inst["A"]) @ (1.3 * inst["w0"] / np.abs(inst["w0"]).sum())
    A = np.asarray(inst["A"])
    res = linprog(-inst["L"], A_ub=np.vstack([A.T, -A.T]), b_ub=np.ones(2 * A.shape[1]),
                  bounds=[(None, None)] * A.shape[0], method="highs")
    assert res.status == 0
    bstar = -res.fun
    assert bstar == pytest.approx(min_budget(inst), rel=1e-7)
    if bstar > 1.0:
        assert certificate_value(inst, -res.x) < 0.0
