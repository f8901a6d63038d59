"""Pins of the oracle's reference gradient (oracle/grad.py): a closed form, and central
finite differences of the oracle's own certified solve along random directions."""
import numpy as np
import pytest

import oracle
from oracle.grad import reference_gradient, piece_of
from oracle.problem import normalize
from synth import make_single, make_multi


def _solve(inst):
    r = oracle.solve(inst, tol=1e-11)
    assert r.polished
    return r


def _fd(inst, key, direction, h, grad_W):
    """Central difference of l(W*) = <grad_W, W*> along inst[key] += h * direction;
    None when the active piece changes between the two sides."""
    vals, pieces = [], []
    for sgn in (1.0, -1.0):
        d = dict(inst)
        d[key] = np.asarray(inst[key], dtype=np.float64) + sgn * h * direction
        r = _solve(d)
        pb = normalize(d)
        pc = piece_of(pb, r.W)
        pieces.append((pc.zero_trade.tobytes(), pc.zero_w.tobytes(), pc.tight.tobytes(),
                       tuple(tuple(x[0]) for x in pc.rows)))
        vals.append(float(np.sum(grad_W * r.W)))
    if pieces[0] != pieces[1]:
        return None
    return (vals[0] - vals[1]) / (2.0 * h)


def test_unconstrained_closed_form():
    """No costs, no exposure rows, small alpha: W* = Sigma^-1 alpha / (2 g1), so
    dl/dalpha = Sigma^-1 grad_W / (2 g1) exactly."""
    inst = make_single(12, 3, 0, seed=4, lambda2=0.0, lambda3=0.0)
    inst["alpha"] = inst["alpha"] * 1e-3
    rng = np.random.default_rng(1)
    gW = rng.normal(size=(1, 12))
    g = reference_gradient(inst, gW)
    pb = normalize(inst)
    Sigma = inst["F"] @ inst["Omega"] @ inst["F"].T + np.diag(inst["delta"] ** 2)
    assert np.abs(g.W).sum() < 0.9
    expect = np.linalg.solve(Sigma, gW[0]) / (2.0 * pb.g1)
    np.testing.assert_allclose(g.alpha[0], expect, rtol=1e-9, atol=1e-12 * np.abs(expect).max())


@pytest.mark.parametrize("seed", [3, 8])
def test_single_period_against_finite_differences(seed):
    inst = make_single(30, 3, 2, seed=seed)
    rng = np.random.default_rng(seed)
    gW = rng.normal(size=(1, 30))
    g = reference_gradient(inst, gW)
    checked = 0
    for key, h, grad, shape in (("alpha", 1e-8, g.alpha, (1, 30)), ("s", 1e-8, g.s, (1, 30)),
                                ("F", 1e-6, g.F, (30, 3))):
        for trial in range(3):
            dvec = rng.normal(size=shape)
            fd = _fd(inst, key, dvec, h, gW)
            if fd is None:
                continue
            an = float(np.sum(grad * dvec))
            assert abs(an - fd) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(grad).max() * np.abs(dvec).sum()), (key, an, fd)
            checked += 1
    assert checked >= 5


def test_multi_period_against_finite_differences():
    inst = make_multi(3, 16, 2, 2, seed=12)
    rng = np.random.default_rng(5)
    gW = np.zeros((2, 16))
    gW[-1] = rng.normal(size=16)      # loss on the last decision
    g = reference_gradient(inst, gW)
    checked = 0
    for key, h, grad, shape in (("alpha", 1e-8, g.alpha, (2, 16)), ("s", 1e-8, g.s, (3, 16)),
                                ("F", 1e-6, g.F, (16, 2))):
        for trial in range(3):
            dvec = rng.normal(size=shape)
            fd = _fd(inst, key, dvec, h, gW)
            if fd is None:
                continue
            an = float(np.sum(grad * dvec))
            assert abs(an - fd) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(grad).max() * np.abs(dvec).sum()), (key, an, fd)
            checked += 1
    assert checked >= 5
