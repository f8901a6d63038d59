"""GPU parity: the HIP solver (through the C ABI) against the FP64 CPU oracle.

Every check: the solver's own relative KKT <= tol and the oracle's independent
re-evaluation of the returned primal-dual pair agreeing with it (a property that holds
at any size).  The relative gap divides |Phi - Psi| by |Phi| + |Psi| ~ 2|Phi|, so a
solve to relative KKT tol has a relative objective error up to ~2 tol; the weights
follow only through strong convexity (error ~ sqrt of the gap).  The stated parity bars
|W - W*|_inf <= 1e-5 and relative objective <= 1e-6 are therefore asserted for solves run
to relative KKT 2e-7; at the default 1e-6 the bars are 2e-5 and 2e-6 (1.1e-5 and 1.5e-6
were observed on the n = 500 case).
"""
import functools
import os

import numpy as np
import pytest

import oracle
from oracle.problem import normalize, kkt, objective
from synth import make_config, make_single, make_multi, make_tiny

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_22625_amd as ff
    return ff


def _run(inst, **kw):
    ff = _gpu()
    print(f"[case] n={inst['alpha'].shape[-1]} T={inst.get('T', 0)} kw={kw}", flush=True)
    kw.setdefault("time_limit_s", 30.0)
    kw.setdefault("max_iter", 200000)
    W, info, (yA, yF, yC) = ff.solve_instance(inst, return_dual=True, **kw)
    torch.cuda.synchronize()
    return W.cpu().numpy(), info, (yA.cpu().numpy(), yF.cpu().numpy(), yC.cpu().numpy())


def _dual_problem(inst):
    """Oracle problem in the factor basis the solver reports y_F in (Cholesky of Omega)."""
    k = inst["F"].shape[1] if inst["F"].ndim == 2 else 0
    return normalize(inst, factor=np.linalg.cholesky(inst["Omega"]) if k else None)


def _check(inst, W, info, Y, ref, tol_kkt, w_tol=1e-5, obj_tol=None):
    obj_tol = 2.0 * tol_kkt if obj_tol is None else obj_tol
    pb = _dual_problem(inst)
    assert info.status == 0, info
    assert info.rel_kkt <= tol_kkt
    K = kkt(pb, W, *Y)
    # the oracle's independent evaluation of the returned pair agrees with the device's
    assert K.rel_kkt <= 2.0 * tol_kkt, (K, info)
    assert abs(K.rel_gap - info.rel_gap) <= 1e-3 * max(K.rel_gap, 1e-12) + 1e-11
    assert abs(K.primal_obj - info.primal_obj) <= 1e-12 * abs(K.primal_obj) + 1e-18
    assert np.max(np.abs(W - ref.W)) <= w_tol
    assert abs(objective(pb, W) - ref.phi) <= obj_tol * abs(ref.phi)


def test_small_config_matches_oracle():
    inst = make_config(0)
    ref = oracle.solve(inst, tol=1e-9)
    W, info, Y = _run(inst, tol=1e-6)
    _check(inst, W, info, Y, ref, 1e-6, w_tol=2e-5, obj_tol=2e-6)


def test_small_config_contract_bars():
    """|W - W*|_inf <= 1e-5 and relative objective <= 1e-6 at relative KKT 2e-7."""
    inst = make_config(0)
    ref = oracle.solve(inst, tol=1e-9)
    W, info, Y = _run(inst, tol=2e-7)
    _check(inst, W, info, Y, ref, 2e-7, w_tol=1e-5, obj_tol=1e-6)


def test_small_config_tight_tolerance():
    inst = make_config(0)
    ref = oracle.solve(inst, tol=1e-9)
    W, info, Y = _run(inst, tol=1e-9)
    _check(inst, W, info, Y, ref, 1e-9, w_tol=3e-7)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_tiny_instances(seed):
    inst = make_tiny(3 + seed, seed=seed, k=2, m=1)
    ref = oracle.solve(inst, tol=1e-10)
    W, info, Y = _run(inst, tol=1e-9)
    _check(inst, W, info, Y, ref, 1e-9, w_tol=1e-6)


@pytest.mark.parametrize("n,wg", [(1, 0), (2, 1), (63, 2), (65, 3), (130, 7), (257, 0), (777, 5)])
def test_ragged_sizes_and_workgroup_counts(n, wg):
    inst = make_single(n, 3, 4, seed=100 + n)
    ref = oracle.solve(inst, tol=1e-10)
    W, info, Y = _run(inst, tol=1e-8, workgroups=wg)
    _check(inst, W, info, Y, ref, 1e-8, w_tol=1e-6)


def test_no_exposure_rows_and_no_factors():
    inst = make_single(200, 0, 0, seed=9)
    ref = oracle.solve(inst, tol=1e-10)
    W, info, Y = _run(inst, tol=1e-8)
    _check(inst, W, info, Y, ref, 1e-8, w_tol=1e-6)


@pytest.mark.parametrize("d", [2.0, 1.3])
def test_other_impact_exponents(d):
    # d = 1.3 has trades near zero where the impact slope is steep: W converges more
    # slowly than the objective, hence the tighter solve
    inst = make_single(150, 4, 4, seed=17, d=d)
    ref = oracle.solve(inst, tol=1e-10)
    W, info, Y = _run(inst, tol=1e-9)
    _check(inst, W, info, Y, ref, 1e-9, w_tol=1e-6)


@pytest.mark.parametrize("T,n", [(2, 50), (4, 60), (6, 120)])
def test_multi_period_small(T, n):
    inst = make_multi(T, n, 4, 6, seed=30 + T)
    ref = oracle.solve(inst, tol=1e-10)
    W, info, Y = _run(inst, tol=1e-8)
    _check(inst, W, info, Y, ref, 1e-8, w_tol=1e-6)


def test_iteration_limit_returns_last_iterate():
    ff = _gpu()
    inst = make_config(0)
    W, info = ff.solve_instance(inst, max_iter=64, raise_on_failure=False)
    assert info.status == 4 and info.iters == 64
    assert np.all(np.isfinite(W.cpu().numpy()))
    assert np.abs(W.cpu().numpy()).sum() <= 1.0 + 1e-12


def test_deterministic_mode_is_bitwise_repeatable():
    ff = _gpu()
    inst = make_config(0)
    W1, i1 = ff.solve_instance(inst, tol=1e-7, deterministic=True)
    W2, i2 = ff.solve_instance(inst, tol=1e-7, deterministic=True)
    assert i1.iters == i2.iters
    assert torch.equal(W1, W2)


@pytest.mark.parametrize("T,n,wg,tol", [(0, 500, 0, 1e-8), (0, 500, 6, 1e-8), (6, 120, 0, 1e-8), (6, 120, 5, 1e-8),
                                        (10, 300, 7, 1e-9)])
def test_breakpoint_lists_match_multisection(T, n, wg, tol):
    """The multiplier finished from the published breakpoint lists (default) and by
    multisection exchanges alone (breakpoint_lists=0) give the same solution; both meet the
    oracle's bars.  Several workgroups make the lists cross workgroup boundaries.  (The
    T=10 case needs relative KKT 1e-9 for 1e-6 in the weights: at 1e-8 either path is
    1.9e-6 away, the weak strong convexity noted in the module docstring.)"""
    inst = make_config(0) if T == 0 else make_multi(T, n, 4, 6, seed=50 + T)
    ref = oracle.solve(inst, tol=1e-10)
    out = {}
    for lists in (False, True):
        W, info, Y = _run(inst, tol=tol, workgroups=wg, breakpoint_lists=lists)
        _check(inst, W, info, Y, ref, tol, w_tol=1e-6)
        out[lists] = W
    assert np.max(np.abs(out[False] - out[True])) <= 1e-6


def test_deterministic_mode_multi_period_bitwise_repeatable():
    """Lists are gathered in arrival order and then sorted: repeated solves in the
    deterministic mode (fixed-order sums) stay bitwise identical."""
    ff = _gpu()
    inst = make_multi(6, 120, 4, 6, seed=56)
    W1, i1 = ff.solve_instance(inst, tol=1e-8, workgroups=5, deterministic=True)
    W2, i2 = ff.solve_instance(inst, tol=1e-8, workgroups=5, deterministic=True)
    assert i1.iters == i2.iters
    assert torch.equal(W1, W2)


def test_invalid_values_rejected():
    ff = _gpu()
    inst = make_config(0)
    bad = dict(inst)
    bad["delta"] = inst["delta"].copy()
    bad["delta"][3] = 0.0
    with pytest.raises(ff.FolioError) as e:
        ff.solve_instance(bad)
    assert e.value.status == 1
    bad = dict(inst)
    bad["L"] = inst["U"] + 1.0
    with pytest.raises(ff.FolioError):
        ff.solve_instance(bad)


# ---------------------------------------------------------------- FP32 form
# Iterates and LDS copies in float32; every reduction, the multiplier search and the
# checks in float64 against the FP64 problem data, so the same bars apply.

def test_fp32_small_config_matches_oracle():
    inst = make_config(0)
    ref = oracle.solve(inst, tol=1e-9)
    W, info, Y = _run(inst, tol=1e-6, precision="fp32")
    _check(inst, W, info, Y, ref, 1e-6, w_tol=2e-5, obj_tol=2e-6)


def test_fp32_small_config_contract_bars():
    """|W - W*|_inf <= 1e-5 and relative objective <= 1e-6 at relative KKT 2e-7."""
    inst = make_config(0)
    ref = oracle.solve(inst, tol=1e-9)
    W, info, Y = _run(inst, tol=2e-7, precision="fp32")
    _check(inst, W, info, Y, ref, 2e-7, w_tol=1e-5, obj_tol=1e-6)


@pytest.mark.parametrize("n,wg", [(65, 3), (257, 0), (777, 5)])
def test_fp32_ragged_sizes(n, wg):
    # n = 257 holds one dominant position (0.278) whose weight is still 3.4e-5 off at
    # relative KKT 2.9e-7 (the weights follow the gap only through strong convexity)
    inst = make_single(n, 3, 4, seed=100 + n)
    ref = oracle.solve(inst, tol=1e-10)
    W, info, Y = _run(inst, tol=1e-7, workgroups=wg, precision="fp32")
    _check(inst, W, info, Y, ref, 1e-7, w_tol=1e-5)


@functools.lru_cache(maxsize=None)
def _long_slice_case(T, n):
    inst = make_single(n, 40, 30, seed=70 + n) if T == 0 else make_multi(T, n, 40, 30, seed=70 + n)
    return inst, oracle.solve(inst, tol=1e-10)


@pytest.mark.parametrize("precision,tol,w_tol", [("fp64", 1e-9, 1e-6), ("fp32", 1e-7, 3e-5)])
@pytest.mark.parametrize("T,n,wg", [(0, 1200, 2), (3, 1100, 2)])
def test_long_slices_read_rows_from_device_memory(precision, tol, w_tol, T, n, wg):
    """Two workgroups over 1100-1200 assets with 70 rows: the constraint slice (>= 168 KB
    even as floats) does not fit in LDS, so the rows come from device memory (float copies
    in the FP32 form) through the long-slice products (more than 512 assets per
    workgroup).  The weight bars follow the gap through strong convexity (module
    docstring): 1e-6 needs relative KKT 1e-9 here, and the FP32 form is held to 3e-5."""
    inst, ref = _long_slice_case(T, n)
    W, info, Y = _run(inst, tol=tol, workgroups=wg, precision=precision, verbose=1)
    _check(inst, W, info, Y, ref, tol, w_tol=w_tol)


def test_fp32_multi_period_small():
    inst = make_multi(4, 60, 4, 6, seed=34)
    ref = oracle.solve(inst, tol=1e-10)
    W, info, Y = _run(inst, tol=1e-6, precision="fp32")
    _check(inst, W, info, Y, ref, 1e-6, w_tol=2e-5)


# ---------------------------------------------------------------- full sizes
# The n = 5000 single-period market against the oracle's certified solution (written by
# tests/golden/make_golden.py, which calls only the oracle); the multi-period markets
# (T = 20, n = 3000 and T = 10, n = 2000) through the oracle's independent KKT
# evaluation of the returned primal-dual pair, a property that holds at any size.

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name, seed):
    g = np.load(os.path.join(GOLDEN, f"{name}_seed{seed}_oracle.npz"))
    assert bool(g["polished"]) and abs(float(g["gap"])) <= 1e-10 * abs(float(g["phi"]))
    return g


C1_GOLDEN_SEEDS = sorted(int(f.split("seed")[1].split("_")[0]) for f in os.listdir(GOLDEN)
                         if f.startswith("c1_seed") and f.endswith("_oracle.npz"))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("seed", C1_GOLDEN_SEEDS)
def test_full_size_single_period_against_golden(precision, seed):
    """n = 5000 markets at the benchmark's relative KKT 1e-6 (measured over seeds 1-7, 9,
    10: |W - W*|_inf up to 2.9e-5, relative objective up to 1.2e-6; bars 5e-5 and 3e-6),
    then the stated parity bars (|W - W*|_inf <= 1e-5, relative objective <= 1e-6) at
    relative KKT 2e-7 (measured 8.6e-6 and 3.3e-7 at most)."""
    inst = make_config(1, seed=seed)
    g = _golden("c1", seed)
    pb = _dual_problem(inst)
    for tol, w_tol, obj_tol in ((1e-6, 5e-5, 3e-6), (2e-7, 1e-5, 1e-6)):
        W, info, Y = _run(inst, tol=tol, precision=precision)
        assert info.status == 0 and info.rel_kkt <= tol
        K = kkt(pb, W, *Y)
        assert K.rel_kkt <= 2.0 * tol, (K, info)
        assert np.max(np.abs(W - g["W"])) <= w_tol, (tol, np.max(np.abs(W - g["W"])))
        assert abs(objective(pb, W) - float(g["phi"])) <= obj_tol * abs(float(g["phi"]))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_full_size_T20_against_golden(precision):
    """T = 20, n = 3000 (19 decision periods) element-wise against the oracle's certified
    W* (paper Section 2.2, eq. 4-6).  At relative KKT 1e-6 the weights are 2.3e-5 away
    (bar 3e-5) with the objective within 2.3e-7 (bar 2e-6); at 1e-8 the stated parity bars
    hold (measured 7.7e-6 in W, 1.5e-8 in the objective)."""
    inst = make_config(2, seed=20)
    g = _golden("c2", 20)
    pb = _dual_problem(inst)
    for tol, w_tol, obj_tol in ((1e-6, 3e-5, 2e-6), (1e-8, 1e-5, 1e-6)):
        W, info, Y = _run(inst, tol=tol, precision=precision, max_iter=400000)
        assert info.status == 0 and info.rel_kkt <= tol
        K = kkt(pb, W, *Y)
        assert K.rel_kkt <= 2.0 * tol, (K, info)
        err = np.max(np.abs(W - g["W"]))
        assert err <= w_tol, (tol, err)
        assert abs(objective(pb, W) - float(g["phi"])) <= obj_tol * abs(float(g["phi"]))
        # feasibility: budgets and exposure bounds of every period
        assert np.all(np.abs(W).sum(axis=1) <= 1.0 + 1e-9)
        AW = W @ pb.A.T
        assert np.all(AW >= pb.L - 1e-5) and np.all(AW <= pb.U + 1e-5)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_full_size_T10_against_golden(precision):
    """The differentiation workload (T = 10, n = 2000, k = 40, m = 5 + 35) element-wise
    against the oracle's certified W*: KKT-implied bars at relative KKT 1e-6, the stated
    parity bars at 1e-8."""
    inst = make_config(4, seed=40)
    g = _golden("c4", 40)
    pb = _dual_problem(inst)
    for tol, w_tol, obj_tol in ((1e-6, 3e-5, 2e-6), (1e-8, 1e-5, 1e-6)):
        W, info, Y = _run(inst, tol=tol, precision=precision, max_iter=400000)
        assert info.status == 0 and info.rel_kkt <= tol
        err = np.max(np.abs(W - g["W"]))
        print(f"  tol {tol:g}: |W - W*| {err:.2e}", flush=True)
        assert err <= w_tol, (tol, err)
        assert abs(objective(pb, W) - float(g["phi"])) <= obj_tol * abs(float(g["phi"]))


@pytest.mark.parametrize("cfg,seed", [(2, 20), (4, 40)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_full_size_multi_period_kkt(cfg, seed, precision):
    inst = make_config(cfg, seed=seed)
    W, info, Y = _run(inst, tol=1e-6, precision=precision)
    pb = _dual_problem(inst)
    assert info.status == 0 and info.rel_kkt <= 1e-6
    K = kkt(pb, W, *Y)
    assert K.rel_kkt <= 2e-6, (K, info)
    assert abs(K.primal_obj - info.primal_obj) <= 1e-10 * abs(K.primal_obj)
    # feasibility of the returned weights: budgets and exposure bounds
    assert np.all(np.abs(W).sum(axis=1) <= 1.0 + 1e-5)
    AW = W @ pb.A.T
    assert np.all(AW >= pb.L - 1e-4) and np.all(AW <= pb.U + 1e-4)


def test_large_single_period_kkt():
    """n = 200000 (k = 60, m = 80): 782 assets per workgroup, so every workgroup reads its
    rows from device memory (the wide row products).  Checked through the oracle's
    independent KKT evaluation of the returned pair and the feasibility of W."""
    inst = make_single(200000, 60, 80, seed=5)
    W, info, Y = _run(inst, tol=1e-6)
    pb = _dual_problem(inst)
    assert info.status == 0 and info.rel_kkt <= 1e-6
    K = kkt(pb, W, *Y)
    assert K.rel_kkt <= 2e-6, (K, info)
    assert abs(K.primal_obj - info.primal_obj) <= 1e-10 * abs(K.primal_obj)
    # feasibility of the returned weights: budget and exposure bounds
    assert np.all(np.abs(W).sum(axis=1) <= 1.0 + 1e-5)
    AW = W @ pb.A.T
    assert np.all(AW >= pb.L - 1e-4) and np.all(AW <= pb.U + 1e-4)
