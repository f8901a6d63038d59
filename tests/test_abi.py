"""C-ABI checks that need no GPU: the library loads, exports every declared entry point,
and rejects invalid sizes, pointers and scalars with FFO_EINVAL before any device work."""
import ctypes
import os
import re

import pytest

import paper_2604_22625_amd as ff

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "ffolio.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ffo_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = ff.lib()
    names = _declared()
    assert "ffo_solve" in names and "ffo_default_options" in names
    for name in names:
        assert hasattr(lib, name), name


def test_default_options():
    o = ff.default_options()
    assert o.tol_rel_kkt == 1e-6 and o.check_every == 64 and o.time_limit_s == 360.0
    assert (o.restart_suff, o.restart_nec, o.restart_art) == (0.2, 0.8, 0.36)
    assert o.reflection == 1.0 and o.precision == 0
    assert (o.deterministic, o.speculative, o.breakpoint_lists, o.infeasibility_check) == (0, -1, 1, 1)


def _call(**over):
    """ffo_solve with fake (never dereferenced) pointers; invalid arguments must be
    rejected by the host-side checks before any pointer is touched."""
    fake = ctypes.c_void_p(0x1000)
    args = dict(n=10, k=2, m=1, T=0, alpha=fake, F=fake, Omega=fake, delta=fake, s=fake, q=fake, d=1.5,
                A=fake, L=fake, U=fake, w0=fake, GMV=1e9, l1=1e-9, l2=1.0, l3=1.0, wT=None, w_out=fake)
    args.update(over)
    info = ff._Info()
    lib = ff.lib()
    rc = lib.ffo_solve(args["n"], args["k"], args["m"], args["T"], args["alpha"], args["F"], args["Omega"],
                       args["delta"], args["s"], args["q"], args["d"], args["A"], args["L"], args["U"],
                       args["w0"], args["GMV"], args["l1"], args["l2"], args["l3"], args["wT"], None, None,
                       args["w_out"], None, ctypes.byref(info))
    return rc, lib.ffo_last_error().decode()


@pytest.mark.parametrize("over,needle", [
    (dict(n=0), "n must"),
    (dict(k=-1), "k must"),
    (dict(k=129), "k must"),
    (dict(m=-2), "m must"),
    (dict(T=1), "T must"),
    (dict(T=3), "w_target"),
    (dict(wT=ctypes.c_void_p(0x2000)), "w_target"),
    (dict(alpha=None), "null"),
    (dict(w_out=None), "null"),
    (dict(F=None), "F and Omega"),
    (dict(A=None), "A, L and U"),
    (dict(d=1.0), "d must"),
    (dict(d=2.5), "d must"),
    (dict(d=float("nan")), "d must"),
    (dict(GMV=0.0), "GMV"),
    (dict(GMV=float("inf")), "GMV"),
    (dict(l1=0.0), "lambda1"),
    (dict(l2=-1.0), "lambda2"),
    (dict(l3=float("nan")), "lambda2 and lambda3"),
    (dict(l1=1e200, GMV=1e200), "lambda1 * GMV"),
])
def test_invalid_arguments_rejected_on_host(over, needle):
    rc, msg = _call(**over)
    assert rc == 1, (rc, msg)
    assert needle in msg


def test_invalid_options_rejected_on_host():
    lib = ff.lib()
    fake = ctypes.c_void_p(0x1000)
    for field, val in (("tol_rel_kkt", 0.0), ("max_iter", 0), ("check_every", 0), ("reflection", 1.5),
                       ("precision", 7), ("precision", 2), ("time_limit_s", -1.0),   # bf16 rows: batched only
                       ("deterministic", 2), ("speculative", -2), ("speculative", 2), ("breakpoint_lists", -1),
                       ("infeasibility_check", 2), ("workgroups", -1)):
        o = ff.default_options()
        setattr(o, field, val)
        info = ff._Info()
        rc = lib.ffo_solve(10, 2, 1, 0, fake, fake, fake, fake, fake, fake, 1.5, fake, fake, fake, fake, 1e9,
                           1e-9, 1.0, 1.0, None, ctypes.byref(o), None, fake, None, ctypes.byref(info))
        assert rc == 1, field


def test_version_string():
    assert b"gfx950" in ff.lib().ffo_version()


def _call_batched(B=3, n_b=(5, 7, 9), n_max=10, k=2, m=1, offs=None, d=1.5, precision=0, null=()):
    """ffo_solve_batched with fake device pointers and real host arrays; invalid
    arguments must be rejected before any device pointer is touched."""
    import numpy as np
    fake = ctypes.c_void_p(0x1000)
    nb = np.ascontiguousarray(np.asarray(n_b, dtype=np.int64))
    of = np.concatenate([[0], np.cumsum(nb)]).astype(np.int64) if offs is None else np.asarray(offs, np.int64)
    of = np.ascontiguousarray(of)
    ptr = {name: (None if name in null else fake) for name in
           ("F", "Omega", "delta", "A", "alpha", "s", "q", "w0", "L", "U", "w_out")}
    infos = (ff._Info * max(B, 1))()
    o = ff.default_options()
    o.precision = precision
    lib = ff.lib()
    rc = lib.ffo_solve_batched(B, nb.ctypes.data_as(ctypes.c_void_p), n_max, k, m, ptr["F"], ptr["Omega"],
                               ptr["delta"], ptr["A"], of.ctypes.data_as(ctypes.c_void_p), ptr["alpha"], ptr["s"],
                               ptr["q"], ptr["w0"], ptr["L"], ptr["U"], d, 1e9, 1e-9, 1.0, 1.0, ctypes.byref(o),
                               None, ptr["w_out"], infos)
    return rc, lib.ffo_last_error().decode()


@pytest.mark.parametrize("kw,needle", [
    (dict(B=0, n_b=()), "B must"),
    (dict(n_b=(5, 11, 9)), "n_b"),
    (dict(n_b=(0, 7, 9)), "n_b"),
    (dict(offs=(0, 5, 13, 21)), "offs"),
    (dict(offs=(1, 6, 13, 22)), "offs[0]"),
    (dict(k=129), "k must"),
    (dict(m=-1), "m must"),
    (dict(d=1.0), "d must"),
    (dict(precision=7), "FFO_FP64, FFO_FP32 or FFO_FP32_BF16K"),
    (dict(null=("alpha",)), "null"),
    (dict(null=("w_out",)), "null"),
    (dict(null=("F",)), "F and Omega"),
    (dict(null=("L",)), "A, L and U"),
])
def test_batched_rejects_invalid_arguments(kw, needle):
    rc, msg = _call_batched(**kw)
    assert rc == 1, (rc, msg)
    assert needle in msg, msg


def _call_many(B=3, n=(5, 7, 9), k=2, m=1, T=0, d=1.5, precision=0, null=(), null_at=None, with_target=None):
    """ffo_solve_many with fake device pointers in real host pointer arrays; invalid
    arguments must be rejected before any device pointer is touched.  null: arrays passed
    as NULL; null_at: (name, b) sets one instance's pointer to NULL."""
    import numpy as np
    fake = 0x1000
    nn = np.ascontiguousarray(np.asarray(n, dtype=np.int64))
    arrays = {}
    for name in ("alpha", "F", "Omega", "delta", "s", "q", "A", "L", "U", "w0", "w_target", "w_out"):
        a = (ctypes.c_void_p * max(B, 1))(*([fake] * max(B, 1)))
        if null_at and null_at[0] == name:
            a[null_at[1]] = None
        skip = name in null or (name == "w_target" and not (T > 0 if with_target is None else with_target))
        arrays[name] = None if skip else ctypes.cast(a, ctypes.c_void_p)
        arrays[name + "_keep"] = a
    infos = (ff._Info * max(B, 1))()
    o = ff.default_options()
    o.precision = precision
    lib = ff.lib()
    g = arrays
    rc = lib.ffo_solve_many(B, nn.ctypes.data_as(ctypes.c_void_p), k, m, T, g["alpha"], g["F"], g["Omega"],
                            g["delta"], g["s"], g["q"], g["A"], g["L"], g["U"], g["w0"], g["w_target"], d, 1e9,
                            1e-9, 1.0, 1.0, ctypes.byref(o), None, g["w_out"], infos)
    return rc, lib.ffo_last_error().decode()


@pytest.mark.parametrize("kw,needle", [
    (dict(B=0, n=()), "B must"),
    (dict(n=(5, 0, 9)), "n must"),
    (dict(k=129), "k must"),
    (dict(m=-1), "m must"),
    (dict(d=1.0), "d must"),
    (dict(precision=2), "FFO_FP64 or FFO_FP32"),
    (dict(null=("alpha",)), "null host array"),
    (dict(null=("w_out",)), "null host array"),
    (dict(null=("F",)), "F and Omega"),
    (dict(null=("L",)), "A, L and U"),
    (dict(null_at=("s", 1)), "instance 1"),
    (dict(null_at=("w_out", 2)), "instance 2"),
    (dict(T=1), "T must"),
    (dict(T=0, with_target=True), "w_target"),
    (dict(T=3, with_target=False), "w_target"),
    (dict(T=3, null_at=("w_target", 0)), "instance 0"),
])
def test_many_rejects_invalid_arguments(kw, needle):
    rc, msg = _call_many(**kw)
    assert rc == 1, (rc, msg)
    assert needle in msg, msg


@pytest.mark.parametrize("omega", [-1.0, float("nan"), float("inf")])
def test_warm_start_rejects_bad_primal_weight(omega):
    lib = ff.lib()
    fake = ctypes.c_void_p(0x1000)
    info = ff._Info()
    rc = lib.ffo_solve_warm(10, 2, 1, 0, fake, fake, fake, fake, fake, fake, 1.5, fake, fake, fake, fake, 1e9,
                            1e-9, 1.0, 1.0, None, fake, fake, omega, None, None, fake, None, ctypes.byref(info))
    assert rc == 1
    assert "omega_init" in lib.ffo_last_error().decode()


def test_warm_start_checks_problem_arguments_first():
    lib = ff.lib()
    fake = ctypes.c_void_p(0x1000)
    info = ff._Info()
    rc = lib.ffo_solve_warm(0, 2, 1, 0, fake, fake, fake, fake, fake, fake, 1.5, fake, fake, fake, fake, 1e9,
                            1e-9, 1.0, 1.0, None, fake, fake, 1.0, None, None, fake, None, ctypes.byref(info))
    assert rc == 1 and "n must" in lib.ffo_last_error().decode()
