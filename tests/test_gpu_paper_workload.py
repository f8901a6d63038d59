"""GPU parity on the paper's own workload shape (paper Section 3 and 4.1) at reduced n:
six factors with a full covariance, the eq. 7 U-shaped cost profile over T = 10 trades
with a constant alpha, and corners of the lambda grid, each against the oracle's
certified solution."""
import numpy as np
import pytest

import oracle
from oracle.problem import normalize, kkt, objective
from synth import paper_instance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_22625_amd as ff
    return ff


CASES = [(0, 300, 1e-8, 1.0), (0, 300, 1e-4, 1.0), (0, 300, 1e-8, 1e4), (0, 300, 1e-4, 1e4), (0, 300, 1e-6, 100.0),
         (10, 200, 1e-6, 1.0), (10, 200, 1e-8, 1000.0), (10, 200, 1e-4, 10.0)]


@pytest.mark.parametrize("T,n,l1,l23", CASES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_paper_shape_matches_oracle(T, n, l1, l23, precision):
    ff = _gpu()
    inst = paper_instance(0, n=n, lambda1=l1, lambda23=l23, T=T)
    tol = 1e-9 if precision == "fp64" else 1e-7
    print(f"[case] paper T={T} n={n} l1={l1} l23={l23} {precision}", flush=True)
    W, info, Y = ff.solve_instance(inst, tol=tol, precision=precision, return_dual=True, time_limit_s=60,
                                   max_iter=400000)
    W = W.cpu().numpy()
    Y = tuple(y.cpu().numpy() for y in Y)
    ref = oracle.solve(inst, tol=1e-10)
    pb = normalize(inst, factor=np.linalg.cholesky(inst["Omega"]))
    assert info.status == 0, info
    K = kkt(pb, W, *Y)
    assert K.rel_kkt <= 2.0 * tol, K
    w_tol = 1e-5 if precision == "fp64" else 3e-5
    assert np.max(np.abs(W - ref.W)) <= w_tol, np.max(np.abs(W - ref.W))
    assert abs(objective(pb, W) - ref.phi) <= max(2.0 * tol, 1e-6) * abs(ref.phi) + 1e-14
