"""Pins for the oracle's full solves (paper Section 2, eq. 1-6).

The oracle's argmin is checked against: closed forms (unconstrained mean-variance,
Woodbury-free dense solve), a separable case solved asset by asset with a 1-D
minimiser and a bisection on the budget multiplier, brute-force enumeration of sign
pieces on tiny instances, the LP special case against HiGHS, weak duality, metamorphic
invariances, and the multi-period T=2 reduction to the single-period model.
"""
import numpy as np
import pytest
from scipy.optimize import linprog, minimize_scalar

import oracle
from oracle.brute import brute_force
from oracle.problem import normalize, objective, dual_objective, project_dual_domain, kkt, trades
from synth import make_single, make_multi, make_tiny, make_config


def _dense_sigma(inst):
    return inst["F"] @ inst["Omega"] @ inst["F"].T + np.diag(inst["delta"] ** 2)


def _no_costs_no_rows(inst, scale_alpha=True):
    inst = dict(inst)
    inst["lambda2"] = 0.0
    inst["lambda3"] = 0.0
    inst["L"] = np.full_like(inst["L"], -np.inf)
    inst["U"] = np.full_like(inst["U"], np.inf)
    return inst


def test_closed_form_unconstrained_single_period():
    """Costs off and rows inactive: w* = Sigma^-1 alpha / (2 lambda1 GMV) (budget slack)."""
    inst = _no_costs_no_rows(make_single(200, 5, 4, seed=3))
    S = _dense_sigma(inst)
    g1 = inst["lambda1"] * inst["GMV"]
    w = np.linalg.solve(S, inst["alpha"][0]) / (2 * g1)
    inst["alpha"] = inst["alpha"] * (0.5 / np.abs(w).sum())   # make ||w*||_1 = 0.5
    w = np.linalg.solve(S, inst["alpha"][0]) / (2 * g1)
    r = oracle.solve(inst, tol=1e-10)
    assert r.polished
    assert np.max(np.abs(r.W[0] - w)) <= 1e-9 * np.abs(w).max()


def test_closed_form_unconstrained_multi_period():
    """Costs off: every period separates, w_t* = w_T + Sigma^-1 alpha_t / (2 g1)."""
    inst = _no_costs_no_rows(make_multi(4, 60, 3, 4, seed=5))
    S = _dense_sigma(inst)
    g1 = inst["lambda1"] * inst["GMV"]
    sol = np.linalg.solve(S, inst["alpha"].T).T / (2 * g1)
    worst = np.max(np.abs(inst["w_target"][None, :] + sol).sum(axis=1))
    inst["alpha"] = inst["alpha"] * (0.05 / worst)
    want = inst["w_target"][None, :] + np.linalg.solve(S, inst["alpha"].T).T / (2 * g1)
    assert np.all(np.abs(want).sum(axis=1) < 1.0)
    r = oracle.solve(inst, tol=1e-10)
    assert np.max(np.abs(r.W - want)) <= 1e-9 * np.abs(want).max()


def _separable_reference(inst):
    """Omega = 0, no rows: per-asset 1-D problems coupled only by the budget multiplier."""
    g1 = inst["lambda1"] * inst["GMV"]
    d2 = inst["delta"] ** 2
    a = inst["lambda2"] * inst["s"][0]
    b = inst["lambda3"] * inst["q"][0]
    al = inst["alpha"][0]
    w0 = inst["w0"]
    d = inst["d"]

    def one(i, mu):
        f = lambda w: -al[i] * w + g1 * d2[i] * w * w + a[i] * abs(w - w0[i]) + b[i] * abs(w - w0[i]) ** d + mu * abs(w)
        cands = [0.0, w0[i]]
        lo, hi = -2.0, 2.0
        r = minimize_scalar(f, bounds=(lo, hi), method="bounded", options={"xatol": 1e-15, "maxiter": 3000})
        cands.append(r.x)
        # refine on both sides of each kink
        for kk in (0.0, w0[i]):
            for side in ((kk - 1.0, kk), (kk, kk + 1.0)):
                rr = minimize_scalar(f, bounds=side, method="bounded", options={"xatol": 1e-15, "maxiter": 3000})
                cands.append(rr.x)
        vals = [f(c) for c in cands]
        return cands[int(np.argmin(vals))]

    def all_w(mu):
        return np.array([one(i, mu) for i in range(len(al))])

    w = all_w(0.0)
    if np.abs(w).sum() <= 1.0:
        return w
    lo, hi = 0.0, 1.0
    while np.abs(all_w(hi)).sum() > 1.0:
        hi *= 2
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if np.abs(all_w(mid)).sum() > 1.0:
            lo = mid
        else:
            hi = mid
    return all_w(hi)


@pytest.mark.slow
def test_separable_case_matches_one_dimensional_solves():
    inst = make_single(12, 3, 2, seed=11)
    inst["Omega"] = np.zeros_like(inst["Omega"])
    inst["L"] = np.full_like(inst["L"], -np.inf)
    inst["U"] = np.full_like(inst["U"], np.inf)
    inst["alpha"] = inst["alpha"] * 3.0
    want = _separable_reference(inst)
    assert abs(np.abs(want).sum() - 1.0) < 1e-6          # budget active: the interesting case
    r = oracle.solve(inst, tol=1e-10)
    assert np.max(np.abs(r.W[0] - want)) <= 1e-7


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("d", [1.5, 2.0])
def test_brute_force_single_period(seed, d):
    inst = make_tiny(3, seed=seed, k=2, m=1, d=d)
    Wb, fb = brute_force(inst)
    r = oracle.solve(inst, tol=1e-10)
    assert r.polished
    assert r.phi <= fb + 1e-12 * abs(fb) + 1e-16
    assert abs(r.phi - fb) <= 1e-8 * abs(fb)
    assert np.max(np.abs(r.W - Wb)) <= 2e-5


@pytest.mark.parametrize("seed", [0, 1])
def test_brute_force_single_period_four_assets_two_rows(seed):
    inst = make_tiny(4, seed=seed + 10, k=2, m=2, d=1.5)
    Wb, fb = brute_force(inst)
    r = oracle.solve(inst, tol=1e-10)
    assert r.phi <= fb + 1e-12 * abs(fb) + 1e-16
    assert abs(r.phi - fb) <= 1e-8 * abs(fb)


@pytest.mark.parametrize("seed,n,T", [(0, 2, 2), (1, 1, 3), (2, 2, 2), (3, 1, 4)])
def test_brute_force_multi_period(seed, n, T):
    inst = make_tiny(n, seed=seed + 20, k=1, m=1, T=T, d=1.5)
    Wb, fb = brute_force(inst)
    r = oracle.solve(inst, tol=1e-10)
    assert r.phi <= fb + 1e-12 * abs(fb) + 1e-16
    assert abs(r.phi - fb) <= 1e-8 * abs(fb)
    assert np.max(np.abs(r.W - Wb)) <= 2e-5


def test_lp_special_case_matches_highs():
    """lambda1 = lambda3 = 0: an LP; the optimal value must equal HiGHS's."""
    inst = make_single(40, 3, 4, seed=7)
    inst["lambda1"] = 0.0
    inst["lambda3"] = 0.0
    n = 40
    al = inst["alpha"][0]
    s = inst["lambda2"] * inst["s"][0]
    w0 = inst["w0"]
    A, L, U = inst["A"], inst["L"], inst["U"]
    # variables: w+ , w- (weights), u+, u- (trades); w = w+ - w-, w - w0 = u+ - u-
    c = np.concatenate([-al, al, s, s])
    Aeq = np.hstack([np.eye(n), -np.eye(n), -np.eye(n), np.eye(n)])
    beq = w0
    Aub = np.vstack([np.hstack([A, -A, np.zeros((4, 2 * n))]), np.hstack([-A, A, np.zeros((4, 2 * n))]),
                     np.concatenate([np.ones(2 * n), np.zeros(2 * n)])[None, :]])
    bub = np.concatenate([U, -L, [1.0]])
    lp = linprog(c, A_ub=Aub, b_ub=bub, A_eq=Aeq, b_eq=beq, bounds=(0, None), method="highs")
    assert lp.status == 0
    r = oracle.solve(inst, tol=1e-9, require_polish=False)
    assert abs(r.phi - lp.fun) <= 1e-6 * abs(lp.fun)
    assert abs(dual_objective(normalize(inst), *project_dual_domain(normalize(inst), r.yA, r.yF, r.yC)) - lp.fun) <= 1e-6 * abs(lp.fun)


@pytest.mark.parametrize("maker", ["single", "multi"])
def test_weak_duality_random_points(maker):
    rng = np.random.default_rng(99)
    inst = make_single(50, 4, 6, seed=4) if maker == "single" else make_multi(5, 30, 3, 6, seed=4)
    pb = normalize(inst)
    for _ in range(200):
        # feasible W: w0 plus a perturbation whose exposure change stays inside the +-0.05 band
        W = np.tile(pb.w0, (pb.P, 1))
        dW = rng.normal(size=W.shape) * 1e-3
        dW *= min(1.0, 0.04 / max(1e-12, np.abs(dW @ pb.A.T).max()))
        W = W + dW
        W /= np.maximum(1.0, np.abs(W).sum(axis=1))[:, None]
        if np.any(W @ pb.A.T < pb.L - 1e-15) or np.any(W @ pb.A.T > pb.U + 1e-15):
            continue
        yA = rng.normal(size=(pb.P, pb.m)) * 10 ** rng.uniform(-5, -2)
        yF = rng.normal(size=(pb.P, pb.k)) * 10 ** rng.uniform(-5, -2)
        yC = rng.normal(size=(pb.Tp, pb.n)) * 10 ** rng.uniform(-5, -2)
        assert dual_objective(pb, yA, yF, yC) <= objective(pb, W) + 1e-15


def test_invariances():
    inst = make_single(30, 3, 4, seed=8)
    base = oracle.solve(inst, tol=1e-10)
    # asset permutation
    perm = np.random.default_rng(0).permutation(30)
    p = dict(inst)
    for key in ("alpha", "s", "q"):
        p[key] = inst[key][:, perm]
    p["F"], p["delta"], p["w0"], p["A"] = inst["F"][perm], inst["delta"][perm], inst["w0"][perm], inst["A"][:, perm]
    rp = oracle.solve(p, tol=1e-10)
    assert np.max(np.abs(rp.W[0] - base.W[0][perm])) <= 1e-12
    # sign flip: alpha, w0 -> -alpha, -w0 and [L, U] -> [-U, -L] maps W* to -W*
    f = dict(inst)
    f["alpha"], f["w0"], f["L"], f["U"] = -inst["alpha"], -inst["w0"], -inst["U"], -inst["L"]
    rf = oracle.solve(f, tol=1e-10)
    assert np.max(np.abs(rf.W + base.W)) <= 1e-12
    # joint scaling of alpha and the three penalties leaves W* fixed
    c = dict(inst)
    c["alpha"] = 3.0 * inst["alpha"]
    c["lambda1"], c["lambda2"], c["lambda3"] = 3 * inst["lambda1"], 3 * inst["lambda2"], 3 * inst["lambda3"]
    rc = oracle.solve(c, tol=1e-10)
    assert np.max(np.abs(rc.W - base.W)) <= 1e-11
    # GMV change with lambda1 GMV fixed leaves W* fixed; the paper objective scales with GMV
    g = dict(inst)
    g["GMV"], g["lambda1"] = 2 * inst["GMV"], inst["lambda1"] / 2
    rg = oracle.solve(g, tol=1e-10)
    assert np.max(np.abs(rg.W - base.W)) <= 1e-12
    assert abs(rg.paper_obj - 2 * base.paper_obj) <= 1e-9 * abs(base.paper_obj)


def test_no_trade_when_w0_is_the_cost_free_optimum():
    inst = make_single(40, 3, 4, seed=9)
    pb = normalize(inst)
    S = _dense_sigma(inst)
    inst["alpha"] = (2 * pb.g1 * S @ inst["w0"])[None, :]   # makes w0 stationary without costs
    for l23 in (0.1, 1.0, 100.0):
        x = dict(inst, lambda2=l23, lambda3=l23)
        r = oracle.solve(x, tol=1e-10)
        assert np.max(np.abs(r.W[0] - inst["w0"])) <= 1e-12


def test_multi_period_T2_reduces_to_single_period():
    sp = make_single(25, 3, 3, seed=12)
    mp = dict(sp)
    mp["T"] = 2
    mp["w_target"] = np.zeros(25)
    mp["s"] = np.vstack([sp["s"], np.zeros((1, 25))])
    mp["q"] = np.vstack([sp["q"], np.zeros((1, 25))])
    r1 = oracle.solve(sp, tol=1e-10)
    r2 = oracle.solve(mp, tol=1e-10)
    assert np.max(np.abs(r1.W - r2.W)) <= 1e-12
    assert abs(r1.phi - r2.phi) <= 1e-14


def test_certificate_small_config():
    r = oracle.solve(make_config(0), tol=1e-9)
    assert r.polished
    assert abs(r.gap) <= 1e-15 * max(1.0, abs(r.phi)) * 1e3
    assert r.rel_kkt <= 1e-12
    assert r.err_bound <= 1e-6
