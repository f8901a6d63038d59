"""Pins of the oracle's relative KKT evaluation (oracle.problem.kkt, project_dual_domain).

Each case builds a primal-dual pair with one violation of a known size and compares the
reported rel_pri / rel_dual with the value worked out by hand from the definitions:

  rel_pri  = ||[A W - clip(A W, L, U); (||w_t||_1 - 1)_+]|| / (1 + ||clip(A W, L, U)||)
  rel_dual = ||Y - proj_dom(h*)(Y)|| / (1 + ||Y||)

The domain of h* (the conjugate of the dual part of the splitting, paper Section 2.1 eq. 2
and 3 for the exposure box and the cost terms) is: y_A,j >= 0 where L_j = -inf (the support
function max(U y, L y) is finite only there), y_A,j <= 0 where U_j = +inf, y_F = 0 when
g1 = 0, and |y_C,i| <= g2 s_i where the impact weight g3 q_i vanishes (the conjugate of a
purely linear cost is the indicator of that interval).  A dropped term, a swapped sign or
a transposed operand in kkt() changes one of these numbers.
"""
import math

import numpy as np
import pytest

from oracle.problem import kkt, normalize, project_dual_domain


def _inst(n=3, m=2, k=1, T=0, L=None, U=None, q=None, lambda1=1e-9):
    """A hand-sized instance with simple numbers (F, A chosen so A W is easy to read)."""
    P = 1 if T == 0 else T - 1
    Tp = 1 if T == 0 else T
    A = np.zeros((m, n))
    A[0, :] = 1.0                         # row 0: net exposure sum_i w_i
    if m > 1:
        A[1, 0] = 2.0                     # row 1: 2 w_0
    inst = dict(
        alpha=np.full((P, n), 1e-3), F=np.ones((n, k)), Omega=np.eye(k) * 1e-4,
        delta=np.full(n, 0.02), s=np.full((Tp, n), 1e-3),
        q=np.full((Tp, n), 5e-4) if q is None else np.asarray(q, dtype=float).reshape(Tp, n),
        d=1.5, A=A, L=np.full(m, -0.5) if L is None else np.asarray(L, float),
        U=np.full(m, 0.5) if U is None else np.asarray(U, float), w0=np.zeros(n), GMV=1e9,
        lambda1=lambda1, lambda2=1.0, lambda3=1.0, T=T)
    if T:
        inst["w_target"] = np.zeros(n)
    return inst


def _zero_duals(pb):
    return np.zeros((pb.P, pb.m)), np.zeros((pb.P, pb.k)), np.zeros((pb.Tp, pb.n))


def test_exposure_row_above_its_upper_bound():
    pb = normalize(_inst())
    # A W = (sum w, 2 w_0) = (0.8, 0.2): row 0 exceeds U = 0.5 by 0.3, row 1 inside
    W = np.array([[0.1, 0.3, 0.4]])
    K = kkt(pb, W, *_zero_duals(pb))
    clip_norm = math.hypot(0.5, 0.2)
    assert K.rel_pri == pytest.approx(0.3 / (1.0 + clip_norm), rel=1e-14)
    assert K.budget_excess == 0.0
    assert K.rel_dual == 0.0


def test_exposure_row_below_its_lower_bound_in_one_of_several_periods():
    pb = normalize(_inst(T=4))            # P = 3 decision periods
    W = np.array([[0.1, 0.1, 0.1], [-0.2, -0.2, -0.3], [0.0, 0.1, 0.0]])
    # period 1: row 0 = -0.7 < L = -0.5 (violation 0.2), row 1 = -0.4 (inside)
    K = kkt(pb, W, *_zero_duals(pb))
    clipped = np.array([[0.3, 0.2], [-0.5, -0.4], [0.1, 0.0]])
    assert K.rel_pri == pytest.approx(0.2 / (1.0 + np.linalg.norm(clipped)), rel=1e-14)


def test_budget_excess_counts_in_the_primal_residual():
    pb = normalize(_inst(L=[-2.0, -2.0], U=[2.0, 2.0]))
    eps = 0.25
    W = np.array([[0.5, -0.5, 0.25]])     # ||w||_1 = 1.25, every exposure row inside
    K = kkt(pb, W, *_zero_duals(pb))
    AW = np.array([0.25, 1.0])
    assert K.budget_excess == pytest.approx(eps, rel=1e-15)
    assert K.rel_pri == pytest.approx(eps / (1.0 + np.linalg.norm(AW)), rel=1e-14)


def test_both_primal_violations_add_in_quadrature():
    pb = normalize(_inst())
    W = np.array([[0.6, 0.3, 0.3]])       # ||w||_1 = 1.2; A W = (1.2, 1.2) vs U = 0.5
    K = kkt(pb, W, *_zero_duals(pb))
    num = math.sqrt(0.7 ** 2 + 0.7 ** 2 + 0.2 ** 2)
    assert K.rel_pri == pytest.approx(num / (1.0 + math.hypot(0.5, 0.5)), rel=1e-14)


def test_wrong_sign_on_an_infinite_lower_bound():
    # L_0 = -inf: the support term max(U y, L y) is +inf for y < 0, so y_A,0 must be >= 0
    pb = normalize(_inst(L=[-np.inf, -0.5], U=[0.5, 0.5]))
    W = np.zeros((1, 3))
    yA = np.array([[-0.4, 0.3]])          # row 0 has the wrong sign, row 1 is free
    yF = np.zeros((1, 1))
    yC = np.zeros((1, 3))
    K = kkt(pb, W, yA, yF, yC)
    assert K.rel_dual == pytest.approx(0.4 / (1.0 + 0.5), rel=1e-14)
    pA, _, _ = project_dual_domain(pb, yA, yF, yC)
    np.testing.assert_array_equal(pA, [[0.0, 0.3]])


def test_wrong_sign_on_an_infinite_upper_bound():
    pb = normalize(_inst(L=[-0.5, -0.5], U=[0.5, np.inf]))
    yA = np.array([[-0.2, 0.6]])          # row 1 (U = +inf) needs y <= 0
    K = kkt(pb, np.zeros((1, 3)), yA, np.zeros((1, 1)), np.zeros((1, 3)))
    assert K.rel_dual == pytest.approx(0.6 / (1.0 + math.hypot(0.2, 0.6)), rel=1e-14)


def test_finite_bounds_leave_any_sign_in_the_domain():
    pb = normalize(_inst())
    yA = np.array([[-3.0, 7.0]])
    K = kkt(pb, np.zeros((1, 3)), yA, np.zeros((1, 1)), np.zeros((1, 3)))
    assert K.rel_dual == 0.0


def test_trade_dual_beyond_the_spread_where_impact_vanishes():
    # q_1 = 0: the cost of asset 1 is linear (g2 s |u|), its conjugate is the indicator of
    # |y| <= g2 s = 1e-3; asset 0 has impact, so any y_C,0 is allowed
    pb = normalize(_inst(q=[5e-4, 0.0, 5e-4]))
    yC = np.array([[0.5, 1e-3 + 0.7, -2e-3]])
    K = kkt(pb, np.zeros((1, 3)), np.zeros((1, 2)), np.zeros((1, 1)), yC)
    assert K.rel_dual == pytest.approx(0.7 / (1.0 + np.linalg.norm(yC)), rel=1e-13)
    _, _, pC = project_dual_domain(pb, np.zeros((1, 2)), np.zeros((1, 1)), yC)
    np.testing.assert_allclose(pC, [[0.5, 1e-3, -2e-3]], rtol=0, atol=0)


def test_trade_dual_below_minus_the_spread_where_impact_vanishes():
    pb = normalize(_inst(q=[0.0, 0.0, 0.0]))
    yC = np.array([[-1e-3 - 0.25, 0.0, 1e-4]])
    K = kkt(pb, np.zeros((1, 3)), np.zeros((1, 2)), np.zeros((1, 1)), yC)
    assert K.rel_dual == pytest.approx(0.25 / (1.0 + np.linalg.norm(yC)), rel=1e-13)


def test_factor_dual_must_vanish_without_risk_aversion():
    pb = normalize(_inst(lambda1=0.0))
    yF = np.array([[0.3]])
    K = kkt(pb, np.zeros((1, 3)), np.zeros((1, 2)), yF, np.zeros((1, 3)))
    assert K.rel_dual == pytest.approx(0.3 / 1.3, rel=1e-14)


def test_several_dual_violations_add_in_quadrature_over_periods():
    pb = normalize(_inst(T=3, L=[-np.inf, -0.5], U=[0.5, np.inf], q=np.zeros(9)))
    yA = np.array([[-0.1, 0.0], [0.0, 0.2]])          # one wrong sign in each period
    yF = np.zeros((2, 1))
    yC = np.zeros((3, 3))
    yC[2, 1] = 1e-3 + 0.3                             # beyond the spread, no impact
    K = kkt(pb, np.zeros((2, 3)), yA, yF, yC)
    num = math.sqrt(0.1 ** 2 + 0.2 ** 2 + 0.3 ** 2)
    den = 1.0 + math.sqrt(0.1 ** 2 + 0.2 ** 2 + (1e-3 + 0.3) ** 2)
    assert K.rel_dual == pytest.approx(num / den, rel=1e-13)


def test_gap_term_is_the_relative_difference_of_the_two_objectives():
    pb = normalize(_inst())
    W = np.array([[0.1, -0.05, 0.02]])
    yA, yF, yC = np.array([[1e-4, -2e-4]]), np.array([[3e-5]]), np.array([[2e-4, -1e-4, 5e-5]])
    K = kkt(pb, W, yA, yF, yC)
    assert K.rel_gap == pytest.approx(abs(K.primal_obj - K.dual_obj) / (abs(K.primal_obj) + abs(K.dual_obj)),
                                      rel=1e-14)
    # weak duality at a feasible W
    assert K.dual_obj <= K.primal_obj
    assert K.rel_kkt == max(K.rel_pri, K.rel_dual, K.rel_gap)
