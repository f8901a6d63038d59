"""GPU parity of the risk-model construction (paper Section 3.2, ffo_risk_model) against
the oracle's plain least-squares definition, on synthetic return panels with missing
history; then the model it builds feeds the solver."""
import numpy as np
import pytest

import oracle
from oracle.riskmodel import risk_model as oracle_risk_model
from synth import make_single, returns_panel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_22625_amd as ff
    return ff


def _mask(days, n, seed, frac_late=0.15):
    """Listing dates: a fraction of the assets start late (some with under two months),
    plus a few scattered missing days."""
    rng = np.random.default_rng(seed)
    M = np.ones((days, n), dtype=np.uint8)
    late = rng.random(n) < frac_late
    start = rng.integers(0, days - 5, size=n)
    for i in np.nonzero(late)[0]:
        M[:start[i], i] = 0
    M[rng.random((days, n)) < 0.01] = 0
    return M


def _compare(P, mask, min_obs, p=None):
    ff = _gpu()
    R, Fr = P["R"], P["Fr"]
    if p is not None:
        Fr = np.ascontiguousarray(Fr[:, :p])
    Rm = R.copy()
    if mask is not None:
        Rm[mask == 0] = np.nan            # unobserved entries are never read
    print(f"[case] riskmodel days={R.shape[0]} n={R.shape[1]} p={Fr.shape[1]} mask={mask is not None}", flush=True)
    beta, Sf, D, valid = ff.risk_model(Rm, Fr, mask=mask, min_obs=min_obs)
    torch.cuda.synchronize()
    ref = oracle_risk_model(R, Fr, mask=mask, min_obs=min_obs)
    np.testing.assert_array_equal(valid.cpu().numpy().astype(bool), ref.valid)
    b = beta.cpu().numpy()
    assert np.abs(b - ref.beta).max() <= 1e-9 * max(1.0, np.abs(ref.beta).max()), np.abs(b - ref.beta).max()
    d = D.cpu().numpy()
    np.testing.assert_allclose(d, ref.D, rtol=1e-9, atol=1e-20)
    np.testing.assert_allclose(Sf.cpu().numpy(), ref.Sigma_f, rtol=1e-12, atol=1e-20)
    return beta, Sf, D, valid


@pytest.mark.parametrize("n,days", [(1000, 504), (77, 504), (64, 63), (65, 65), (300, 2)])
def test_matches_oracle_without_mask(n, days):
    P = returns_panel(n=n, days=days, seed=11)
    _compare(P, None, min_obs=2 if days < 10 else 42)


@pytest.mark.parametrize("n", [1000, 129])
def test_matches_oracle_with_missing_history(n):
    P = returns_panel(n=n, days=504, seed=12)
    M = _mask(504, n, seed=13)
    _, _, _, valid = _compare(P, M, min_obs=42)
    assert 0 < int((valid.cpu().numpy() == 0).sum()) < n   # some assets lack two months


@pytest.mark.parametrize("p", [1, 3, 6])
def test_factor_counts(p):
    P = returns_panel(n=200, days=300, seed=14)
    _compare(P, _mask(300, 200, seed=15), min_obs=42, p=p)


def test_built_model_feeds_the_solver():
    """The device-built model and the oracle-built model of the same panel give the same
    optimal portfolio (paper eq. 1-3 with S = beta Sigma_f beta^T + D)."""
    ff = _gpu()
    P = returns_panel(n=400, days=504, seed=16)
    beta, Sf, D, valid = ff.risk_model(P["R"], P["Fr"], min_obs=42)
    ref = oracle_risk_model(P["R"], P["Fr"], min_obs=42)
    base = make_single(400, 6, 10, seed=17)
    inst_gpu = dict(base, F=beta.cpu().numpy(), Omega=Sf.cpu().numpy(), delta=np.sqrt(D.cpu().numpy()))
    inst_ref = dict(base, F=ref.beta, Omega=ref.Sigma_f, delta=np.sqrt(ref.D))
    W, info = ff.solve_instance(inst_gpu, tol=1e-9)
    r = oracle.solve(inst_ref, tol=1e-10)
    assert info.status == 0
    assert np.max(np.abs(W.cpu().numpy() - r.W)) <= 1e-6


def test_rejects_bad_arguments():
    ff = _gpu()
    P = returns_panel(n=10, days=50, seed=18)
    with pytest.raises(ff.FolioError):
        ff.risk_model(P["R"][:1], P["Fr"][:1])                  # days < 2
    with pytest.raises(ff.FolioError):
        ff.risk_model(P["R"], np.zeros((50, 9)))                # p > 8
    with pytest.raises(ff.FolioError):
        ff.risk_model(P["R"], P["Fr"], min_obs=51)              # min_obs > days
