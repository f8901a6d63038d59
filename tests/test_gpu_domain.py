"""GPU parity over the rest of the API domain the paper states (Section 2.1 and 3.2): a
full (non-diagonal) factor covariance, a singular positive semidefinite one, exposure
rows with one-sided and infinite bounds, and the rejected inputs (lambda1 = 0, a zero
specific volatility), each against the oracle."""
import numpy as np
import pytest

import oracle
from oracle.problem import normalize, kkt, objective
from synth import make_multi, make_single

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_22625_amd as ff
    return ff


def _with_omega(inst, Om):
    out = dict(inst)
    out["Omega"] = np.ascontiguousarray(Om)
    return out


def _full_omega(k, seed, rank=None):
    """A full symmetric PSD k x k matrix with factor variances ~(0.01..0.05)^2; rank < k
    makes it singular."""
    rng = np.random.default_rng(seed)
    r = k if rank is None else rank
    Z = rng.normal(size=(k, r)) * rng.uniform(0.01, 0.05, size=r)[None, :]
    Om = Z @ Z.T
    return 0.5 * (Om + Om.T)


def _solve_and_compare(inst, tol, w_tol, kkt_basis):
    ff = _gpu()
    print(f"[case] n={inst['alpha'].shape[-1]} T={inst.get('T', 0)} tol={tol}", flush=True)
    W, info, Y = ff.solve_instance(inst, tol=tol, return_dual=True, time_limit_s=60, max_iter=400000)
    W = W.cpu().numpy()
    ref = oracle.solve(inst, tol=1e-10)
    pb = normalize(inst)
    assert info.status == 0, info
    assert np.max(np.abs(W - ref.W)) <= w_tol, np.max(np.abs(W - ref.W))
    assert abs(objective(pb, W) - ref.phi) <= 2.0 * tol * abs(ref.phi)
    if kkt_basis:
        # y_F is reported in the Cholesky basis of Omega
        pbc = normalize(inst, factor=np.linalg.cholesky(inst["Omega"]))
        K = kkt(pbc, W, *(y.cpu().numpy() for y in Y))
        assert K.rel_kkt <= 2.0 * tol, K
    return W, info


@pytest.mark.parametrize("T", [0, 5])
def test_full_factor_covariance(T):
    base = make_single(400, 8, 10, seed=71) if T == 0 else make_multi(T, 150, 8, 10, seed=72)
    inst = _with_omega(base, _full_omega(8, 3))
    assert np.abs(inst["Omega"] - np.diag(np.diag(inst["Omega"]))).max() > 0
    _solve_and_compare(inst, 1e-9, 1e-6, kkt_basis=True)


@pytest.mark.parametrize("T", [0, 5])
def test_singular_factor_covariance(T):
    # rank 5 of 8: Cholesky fails on the host and the factor comes from the Jacobi
    # eigendecomposition; W and Phi do not depend on the factor's basis
    base = make_single(400, 8, 10, seed=73) if T == 0 else make_multi(T, 150, 8, 10, seed=74)
    Om = _full_omega(8, 4, rank=5)
    assert np.linalg.matrix_rank(Om, tol=1e-12) == 5
    inst = _with_omega(base, Om)
    _solve_and_compare(inst, 1e-9, 1e-6, kkt_basis=False)


def test_zero_factor_covariance_is_allowed():
    # Omega = 0: no factor risk at all (the factor rows carry zeros)
    base = make_single(200, 4, 6, seed=75)
    inst = _with_omega(base, np.zeros((4, 4)))
    _solve_and_compare(inst, 1e-9, 1e-6, kkt_basis=False)


@pytest.mark.parametrize("T", [0, 4])
def test_one_sided_and_infinite_bounds(T):
    inst = make_single(300, 6, 8, seed=76) if T == 0 else make_multi(T, 120, 6, 8, seed=77)
    inst = dict(inst)
    L, U = inst["L"].copy(), inst["U"].copy()
    L[0] = -np.inf                 # upper bound only
    U[1] = np.inf                  # lower bound only
    L[2], U[2] = -np.inf, np.inf   # unbounded row
    L[3] = U[3] = 0.5 * (L[3] + U[3])   # equality row
    inst["L"], inst["U"] = L, U
    W, info = _solve_and_compare(inst, 1e-9, 1e-6, kkt_basis=True)
    AW = np.atleast_2d(W) @ inst["A"].T
    assert np.all(AW[:, 0] <= U[0] + 1e-7) and np.all(AW[:, 1] >= L[1] - 1e-7)
    assert np.all(np.abs(AW[:, 3] - L[3]) <= 1e-7)


def test_no_exposure_rows_multi_period():
    inst = make_multi(4, 100, 3, 0, seed=78)
    _solve_and_compare(inst, 1e-9, 1e-6, kkt_basis=True)


def test_rejected_inputs():
    """lambda1 = 0 and a zero specific volatility are rejected (the solver relies on the
    strictly convex risk term: it makes W* unique and keeps every asset's curvature and
    the dual's inner problem finite); a tiny positive lambda1 is the supported limit."""
    ff = _gpu()
    inst = make_single(100, 3, 4, seed=79)
    with pytest.raises(ff.FolioError) as e:
        ff.solve_instance(dict(inst, lambda1=0.0))
    assert e.value.status == 1 and "lambda1" in str(e.value)
    bad = dict(inst)
    bad["delta"] = inst["delta"].copy()
    bad["delta"][5] = 0.0
    with pytest.raises(ff.FolioError) as e:
        ff.solve_instance(bad)
    assert e.value.status == 1 and "delta" in str(e.value)
    # a non-symmetric or indefinite Omega is rejected as well
    with pytest.raises(ff.FolioError):
        ff.solve_instance(_with_omega(inst, np.diag([1e-4, -1e-4, 1e-4])))
