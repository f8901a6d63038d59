"""MI355X (gfx950) first-order solver for the FlashFolio portfolio models (arXiv 2604.22625).

Thin Python binding over the C library ``libffolio.so`` (include/ffolio.h).  This module
only marshals arguments: every step of the solve runs in the library's HIP kernels.
PyTorch provides device memory and the current HIP stream.  There is no CPU fallback:
if the library or a GPU is missing, the calls raise.
"""
from __future__ import annotations

import atexit
import ctypes
import os
from dataclasses import dataclass, asdict

import numpy as np

__all__ = ["solve", "solve_instance", "solve_batched", "adjoint", "risk_model", "FolioFn", "Info", "FolioError",
           "lib", "LIB_PATH", "STATUS"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libffolio.so")

STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "NOT_CONVERGED", 5: "NUMERIC",
          6: "INFEASIBLE", 7: "TIMEOUT"}


class FolioError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ffolio status {status} ({STATUS.get(status, '?')}): {msg}")
        self.status = status


class _Options(ctypes.Structure):
    _fields_ = [("tol_rel_kkt", ctypes.c_double), ("max_iter", ctypes.c_int64),
                ("time_limit_s", ctypes.c_double), ("check_every", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("restart_suff", ctypes.c_double),
                ("restart_nec", ctypes.c_double), ("restart_art", ctypes.c_double),
                ("reflection", ctypes.c_double), ("workgroups", ctypes.c_int32),
                ("verbose", ctypes.c_int32), ("deterministic", ctypes.c_int32),
                ("speculative", ctypes.c_int32), ("breakpoint_lists", ctypes.c_int32),
                ("infeasibility_check", ctypes.c_int32), ("batched_form", ctypes.c_int32),
                ("autotune", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int64), ("restarts", ctypes.c_int64),
                ("rel_kkt", ctypes.c_double), ("rel_pri", ctypes.c_double), ("rel_dual", ctypes.c_double),
                ("rel_gap", ctypes.c_double), ("fixed_point_res", ctypes.c_double),
                ("primal_obj", ctypes.c_double), ("dual_obj", ctypes.c_double), ("omega", ctypes.c_double),
                ("ms_setup", ctypes.c_double), ("ms_iter", ctypes.c_double)]


@dataclass
class Info:
    status: int
    iters: int
    restarts: int
    rel_kkt: float
    rel_pri: float
    rel_dual: float
    rel_gap: float
    fixed_point_res: float
    primal_obj: float
    dual_obj: float
    omega: float
    ms_setup: float
    ms_iter: float

    def as_dict(self) -> dict:
        return asdict(self)


_lib = None
_P = ctypes.c_void_p
_D = ctypes.c_double
_I64 = ctypes.c_int64


def lib() -> ctypes.CDLL:
    """Load libffolio.so (built in-tree by paper_2604_22625_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2604_22625_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.ffo_default_options.argtypes = [ctypes.POINTER(_Options)]
        L.ffo_default_options.restype = None
        L.ffo_solve.argtypes = [_I64, _I64, _I64, _I64, _P, _P, _P, _P, _P, _P, _D, _P, _P, _P, _P,
                                _D, _D, _D, _D, _P, ctypes.POINTER(_Options), _P, _P, _P,
                                ctypes.POINTER(_Info)]
        L.ffo_solve.restype = ctypes.c_int
        L.ffo_solve_warm.argtypes = [_I64, _I64, _I64, _I64, _P, _P, _P, _P, _P, _P, _D, _P, _P, _P, _P,
                                     _D, _D, _D, _D, _P, _P, _P, _D, ctypes.POINTER(_Options), _P, _P, _P,
                                     ctypes.POINTER(_Info)]
        L.ffo_solve_warm.restype = ctypes.c_int
        L.ffo_solve_noalloc.argtypes = L.ffo_solve.argtypes
        L.ffo_solve_noalloc.restype = ctypes.c_int
        L.ffo_risk_model.argtypes = [_I64, _I64, _I64, _P, _P, _P, _I64, _P, _P, _P, _P, _P]
        L.ffo_risk_model.restype = ctypes.c_int
        L.ffo_solve_batched.argtypes = [_I64, _P, _I64, _I64, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                        _D, _D, _D, _D, _D, ctypes.POINTER(_Options), _P, _P, _P]
        L.ffo_solve_batched.restype = ctypes.c_int
        L.ffo_solve_many.argtypes = [_I64, _P, _I64, _I64, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                     _D, _D, _D, _D, _D, ctypes.POINTER(_Options), _P, _P, _P]
        L.ffo_solve_many.restype = ctypes.c_int
        L.ffo_adjoint.argtypes = [_I64, _I64, _I64, _I64, _P, _P, _P, _P, _P, _P, _D, _P, _P, _P, _P,
                                  _D, _D, _D, _D, _P, _P, _P, _P, _D, ctypes.POINTER(_Options), _P, _P, _P, _P,
                                  ctypes.POINTER(_Info)]
        L.ffo_adjoint.restype = ctypes.c_int
        L.ffo_last_error.argtypes = []
        L.ffo_last_error.restype = ctypes.c_char_p
        L.ffo_release.argtypes = []
        L.ffo_release.restype = None
        L.ffo_version.argtypes = []
        L.ffo_version.restype = ctypes.c_char_p
        _lib = L
        # release the library's cached workspaces (device memory, pinned host buffers,
        # events) while the HIP runtime is still alive, not in its teardown
        atexit.register(_release_at_exit)
    return _lib


def _release_at_exit():
    if _lib is None:
        return
    try:
        torch = _torch()
        if torch.cuda.is_available() and torch.cuda.is_initialized():
            torch.cuda.synchronize()
    except Exception:  # pragma: no cover - interpreter shutdown
        pass
    _lib.ffo_release()


def default_options() -> _Options:
    o = _Options()
    lib().ffo_default_options(ctypes.byref(o))
    return o


def _torch():
    import torch
    return torch


def _dev_f64(x, device):
    """Contiguous float64 tensor on `device` (None passes through)."""
    if x is None:
        return None
    torch = _torch()
    if not isinstance(x, torch.Tensor):
        x = torch.as_tensor(np.asarray(x, dtype=np.float64))
    return x.to(device=device, dtype=torch.float64).contiguous()


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


PRECISION = {"fp64": 0, "fp32": 1, "fp32_bf16k": 2}


def solve(alpha, F, Omega, delta, s, q, d, A, L, U, w0, GMV, lambda1, lambda2, lambda3,
          w_target=None, *, tol: float = 1e-6, max_iter: int = 1_000_000, time_limit_s: float = 360.0,
          check_every: int = 64, restart=(0.2, 0.8, 0.36), reflection: float = 1.0,
          workgroups: int = 0, verbose: int = 0, return_dual: bool = False, precision="fp64",
          deterministic: bool = False, speculative: int = -1, breakpoint_lists: bool = True,
          infeasibility_check: bool = True, w_init=None, y_init=None, omega_init: float = 0.0,
          noalloc: bool = False, raise_on_failure: bool = True, device=None, stream=None, out=None):
    """Solve one single-period (w_target is None) or multi-period instance on the GPU.

    Arrays follow include/ffolio.h: alpha [P][n] (P = 1 or T-1), F [n][k], Omega [k][k],
    delta [n], s and q [T'][n] (T' = 1 or T), A [m][n], L and U [m], w0 and w_target [n].
    Returns (W [P][n] float64 CUDA tensor, Info) or (W, Info, (yA, yF, yC)) with
    ``return_dual``.  Non-OK statuses raise FolioError unless ``raise_on_failure`` is
    False (NOT_CONVERGED/TIMEOUT/NUMERIC/INFEASIBLE still fill W).  ``precision`` is
    "fp64" or "fp32" (float32 iterates and matrix copies, float64 reductions and checks).
    ``w_init`` [P][n], ``y_init`` (tuple yA, yF, yC or the packed vector) and
    ``omega_init`` start the iteration from a previous solution (ffo_solve_warm).
    ``noalloc`` calls the allocation-free entry point (ffo_solve_noalloc; no warm start).
    """
    torch = _torch()
    if not torch.cuda.is_available():
        raise FolioError(3, "no GPU visible to PyTorch: the solver has no CPU path")
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    a = _dev_f64(alpha, dev)
    if a.dim() == 1:
        a = a[None, :]
    n = a.shape[1]
    T = 0 if w_target is None else a.shape[0] + 1
    Fd = _dev_f64(F, dev).reshape(n, -1)
    k = Fd.shape[1]
    Od = _dev_f64(Omega, dev).reshape(k, k) if k else _dev_f64(np.zeros((0, 0)), dev)
    Ad = _dev_f64(A, dev)
    Ad = Ad.reshape(-1, n) if Ad is not None and Ad.numel() else _dev_f64(np.zeros((0, n)), dev)
    m = Ad.shape[0]
    sd = _dev_f64(s, dev).reshape(-1, n)
    qd = _dev_f64(q, dev).reshape(-1, n)
    Ld = _dev_f64(L, dev).reshape(m) if m else _dev_f64(np.zeros(0), dev)
    Ud = _dev_f64(U, dev).reshape(m) if m else _dev_f64(np.zeros(0), dev)
    dd = _dev_f64(delta, dev).reshape(n)
    w0d = _dev_f64(w0, dev).reshape(n)
    wTd = _dev_f64(w_target, dev).reshape(n) if w_target is not None else None
    P = 1 if T == 0 else T - 1
    Tp = 1 if T == 0 else T
    W = out if out is not None else torch.empty((P, n), dtype=torch.float64, device=dev)
    Y = torch.empty(P * m + P * k + Tp * n, dtype=torch.float64, device=dev) if return_dual else None
    o = default_options()
    o.tol_rel_kkt = float(tol)
    o.max_iter = int(max_iter)
    o.time_limit_s = float(time_limit_s)
    o.check_every = int(check_every)
    o.restart_suff, o.restart_nec, o.restart_art = (float(v) for v in restart)
    o.reflection = float(reflection)
    o.workgroups = int(workgroups)
    o.verbose = int(verbose)
    o.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    o.deterministic = int(bool(deterministic))
    o.speculative = int(speculative)
    o.breakpoint_lists = int(bool(breakpoint_lists))
    o.infeasibility_check = int(bool(infeasibility_check))
    info = _Info()
    st = torch.cuda.current_stream(dev) if stream is None else stream
    args = (n, k, m, T, _ptr(a), _ptr(Fd if k else None), _ptr(Od if k else None), _ptr(dd),
            _ptr(sd), _ptr(qd), float(d), _ptr(Ad if m else None), _ptr(Ld if m else None),
            _ptr(Ud if m else None), _ptr(w0d), float(GMV), float(lambda1), float(lambda2),
            float(lambda3), _ptr(wTd))
    tail = (ctypes.byref(o), ctypes.c_void_p(st.cuda_stream), _ptr(W), _ptr(Y), ctypes.byref(info))
    with torch.cuda.device(dev):
        if noalloc:
            if w_init is not None or y_init is not None or omega_init:
                raise ValueError("the allocation-free entry point takes no warm start")
            rc = lib().ffo_solve_noalloc(*args, *tail)
        elif w_init is None and y_init is None and not omega_init:
            rc = lib().ffo_solve(*args, *tail)
        else:
            wi = _dev_f64(w_init, dev).reshape(P, n) if w_init is not None else None
            if isinstance(y_init, (tuple, list)):
                yi = torch.cat([_dev_f64(y, dev).reshape(-1) for y in y_init])
            else:
                yi = _dev_f64(y_init, dev).reshape(-1) if y_init is not None else None
            if yi is not None and yi.numel() != P * m + P * k + Tp * n:
                raise ValueError("y_init must hold P*m + P*k + T'*n values")
            rc = lib().ffo_solve_warm(*args, _ptr(wi), _ptr(yi), float(omega_init), *tail)
    inf = Info(**{f[0]: getattr(info, f[0]) for f in _Info._fields_})
    if rc == 1 or (rc in (2, 3)) or (rc != 0 and raise_on_failure):
        raise FolioError(rc, lib().ffo_last_error().decode())
    if return_dual:
        yA = Y[:P * m].reshape(P, m)
        yF = Y[P * m:P * m + P * k].reshape(P, k)
        yC = Y[P * m + P * k:].reshape(Tp, n)
        return W, inf, (yA, yF, yC)
    return W, inf


def solve_instance(inst: dict, **kw):
    """Solve an instance dict in the layout of ``synth`` (keys alpha, F, Omega, ...)."""
    T = int(inst.get("T", 0) or 0)
    return solve(inst["alpha"], inst["F"], inst["Omega"], inst["delta"], inst["s"], inst["q"], inst["d"],
                 inst["A"], inst["L"], inst["U"], inst["w0"], inst["GMV"], inst["lambda1"], inst["lambda2"],
                 inst["lambda3"], inst.get("w_target") if T else None, **kw)


def solve_batched(batch: dict, *, tol: float = 1e-6, max_iter: int = 1_000_000, time_limit_s: float = 360.0,
                  check_every: int = 64, restart=(0.2, 0.8, 0.36), reflection: float = 1.0, verbose: int = 0,
                  precision="fp64", form="auto", deterministic: bool = False, autotune: int = 1,
                  raise_on_failure: bool = True, device=None, stream=None, out=None):
    """Solve a batch of single-period instances on one shared universe (layout of
    ``synth.make_batch``: n_b, offs, n_max, F, Omega, delta, A shared; alpha, s, q, w0
    packed; L, U [B][m]).  ``form``: "lockstep" (every unconverged instance advances one
    iteration per step, the shared-row products on the matrix cores; FP64), "teams" (one
    team of workgroups per instance) or "auto" (lockstep when it applies).  Returns
    (w packed [N] float64 CUDA tensor, list of Info)."""
    torch = _torch()
    if not torch.cuda.is_available():
        raise FolioError(3, "no GPU visible to PyTorch: the solver has no CPU path")
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    n_b = np.ascontiguousarray(np.asarray(batch["n_b"], dtype=np.int64))
    offs = np.ascontiguousarray(np.asarray(batch["offs"], dtype=np.int64))
    B = int(n_b.shape[0])
    n_max = int(batch["n_max"])
    k = int(batch["k"])
    m = int(batch["m"])
    Fd = _dev_f64(batch["F"], dev).reshape(n_max, k) if k else None
    Od = _dev_f64(batch["Omega"], dev).reshape(k, k) if k else None
    dd = _dev_f64(batch["delta"], dev).reshape(n_max)
    Ad = _dev_f64(batch["A"], dev).reshape(m, n_max) if m else None
    a = _dev_f64(batch["alpha"], dev).reshape(-1)
    sd = _dev_f64(batch["s"], dev).reshape(-1)
    qd = _dev_f64(batch["q"], dev).reshape(-1)
    w0d = _dev_f64(batch["w0"], dev).reshape(-1)
    Ld = _dev_f64(batch["L"], dev).reshape(B, m) if m else None
    Ud = _dev_f64(batch["U"], dev).reshape(B, m) if m else None
    N = int(offs[-1])
    W = out if out is not None else torch.empty(N, dtype=torch.float64, device=dev)
    o = default_options()
    o.tol_rel_kkt = float(tol)
    o.max_iter = int(max_iter)
    o.time_limit_s = float(time_limit_s)
    o.check_every = int(check_every)
    o.restart_suff, o.restart_nec, o.restart_art = (float(v) for v in restart)
    o.reflection = float(reflection)
    o.verbose = int(verbose)
    o.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    o.batched_form = {"auto": 0, "teams": 1, "lockstep": 2}[form]
    o.autotune = int(autotune)
    o.deterministic = int(bool(deterministic))
    infos = (_Info * B)()
    st = torch.cuda.current_stream(dev) if stream is None else stream
    with torch.cuda.device(dev):
        rc = lib().ffo_solve_batched(B, n_b.ctypes.data_as(ctypes.c_void_p), n_max, k, m, _ptr(Fd), _ptr(Od),
                                     _ptr(dd), _ptr(Ad), offs.ctypes.data_as(ctypes.c_void_p), _ptr(a), _ptr(sd),
                                     _ptr(qd), _ptr(w0d), _ptr(Ld), _ptr(Ud), float(batch["d"]), float(batch["GMV"]),
                                     float(batch["lambda1"]), float(batch["lambda2"]), float(batch["lambda3"]),
                                     ctypes.byref(o), ctypes.c_void_p(st.cuda_stream), _ptr(W), infos)
    out_infos = [Info(**{f[0]: getattr(i, f[0]) for f in _Info._fields_}) for i in infos]
    if rc == 1 or (rc in (2, 3)) or (rc != 0 and raise_on_failure):
        raise FolioError(rc, lib().ffo_last_error().decode())
    return W, out_infos


def solve_many(insts, *, tol: float = 1e-6, max_iter: int = 1_000_000, time_limit_s: float = 360.0,
               check_every: int = 64, restart=(0.2, 0.8, 0.36), reflection: float = 1.0, verbose: int = 0,
               precision="fp64", speculative: int = -1, raise_on_failure: bool = True, device=None,
               stream=None):
    """Solve unrelated instances (dicts in the layout of ``synth.make_single`` or
    ``synth.make_multi``, each with its own n, F, Omega, delta, A, L, U, vectors and target;
    k, m, T, d, GMV and the lambdas shared) in one launch of the team form
    (ffo_solve_many).  Returns (list of W [P][n_b] float64 CUDA tensors, P = T - 1 or 1,
    list of Info)."""
    torch = _torch()
    if not torch.cuda.is_available():
        raise FolioError(3, "no GPU visible to PyTorch: the solver has no CPU path")
    insts = list(insts)
    if not insts:
        raise ValueError("solve_many needs at least one instance")
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    first = insts[0]
    k, m, T = int(first["k"]), int(first["m"]), int(first.get("T", 0) or 0)
    P, Tp = (T - 1, T) if T else (1, 1)
    shared = ("d", "GMV", "lambda1", "lambda2", "lambda3")
    for inst in insts:
        if (int(inst["k"]) != k or int(inst["m"]) != m or int(inst.get("T", 0) or 0) != T
                or any(float(inst[x]) != float(first[x]) for x in shared)):
            raise ValueError("solve_many needs the same k, m, T, d, GMV and lambdas in every instance")
    B = len(insts)
    keep = []   # device tensors that must outlive the call

    def arr(key, shape_of):
        ptrs = (ctypes.c_void_p * B)()
        for b, inst in enumerate(insts):
            t = _dev_f64(inst[key], dev)
            if t is not None:
                t = t.reshape(shape_of(inst))
                keep.append(t)
            ptrs[b] = _ptr(t).value
        return ptrs

    n = np.ascontiguousarray(np.array([int(inst["n"]) for inst in insts], dtype=np.int64))
    a = arr("alpha", lambda i: (P, int(i["n"])))
    Fp = arr("F", lambda i: (int(i["n"]), k)) if k else None
    Op = arr("Omega", lambda i: (k, k)) if k else None
    dp = arr("delta", lambda i: (int(i["n"]),))
    sp = arr("s", lambda i: (Tp, int(i["n"])))
    qp = arr("q", lambda i: (Tp, int(i["n"])))
    Ap = arr("A", lambda i: (m, int(i["n"]))) if m else None
    Lp = arr("L", lambda i: (m,)) if m else None
    Up = arr("U", lambda i: (m,)) if m else None
    wp = arr("w0", lambda i: (int(i["n"]),))
    tp = arr("w_target", lambda i: (int(i["n"]),)) if T else None
    Ws = [torch.empty((P, int(inst["n"])), dtype=torch.float64, device=dev) for inst in insts]
    wo = (ctypes.c_void_p * B)(*[w.data_ptr() for w in Ws])
    o = default_options()
    o.tol_rel_kkt = float(tol)
    o.max_iter = int(max_iter)
    o.time_limit_s = float(time_limit_s)
    o.check_every = int(check_every)
    o.restart_suff, o.restart_nec, o.restart_art = (float(v) for v in restart)
    o.reflection = float(reflection)
    o.verbose = int(verbose)
    o.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    o.speculative = int(speculative)
    infos = (_Info * B)()
    st = torch.cuda.current_stream(dev) if stream is None else stream
    vp = lambda x: ctypes.cast(x, ctypes.c_void_p) if x is not None else ctypes.c_void_p(0)
    with torch.cuda.device(dev):
        rc = lib().ffo_solve_many(B, n.ctypes.data_as(ctypes.c_void_p), k, m, T, vp(a), vp(Fp), vp(Op), vp(dp),
                                  vp(sp), vp(qp), vp(Ap), vp(Lp), vp(Up), vp(wp), vp(tp), float(first["d"]),
                                  float(first["GMV"]),
                                  float(first["lambda1"]), float(first["lambda2"]), float(first["lambda3"]),
                                  ctypes.byref(o), ctypes.c_void_p(st.cuda_stream), vp(wo), infos)
    out_infos = [Info(**{f[0]: getattr(i, f[0]) for f in _Info._fields_}) for i in infos]
    if rc == 1 or (rc in (2, 3)) or (rc != 0 and raise_on_failure):
        raise FolioError(rc, lib().ffo_last_error().decode())
    return Ws, out_infos


def adjoint(inst: dict, W, Y, grad_w, *, omega: float = 0.0, tol: float = 1e-9, max_iter: int = 1_000_000,
            time_limit_s: float = 360.0, check_every: int = 64, verbose: int = 0, raise_on_failure: bool = True,
            device=None, stream=None):
    """Gradients of l(W*) with respect to alpha, s and F (ffo_adjoint).

    ``inst``: the instance dict the solve ran on; ``W``: its solution [P][n]; ``Y``: its
    duals as returned by ``solve(..., return_dual=True)`` (tuple yA, yF, yC) or the packed
    vector; ``grad_w``: dl/dW [P][n].  Returns (grad_alpha [P][n], grad_s [T'][n],
    grad_F [n][k], Info), float64 CUDA tensors."""
    torch = _torch()
    if not torch.cuda.is_available():
        raise FolioError(3, "no GPU visible to PyTorch: the solver has no CPU path")
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    T = int(inst.get("T", 0) or 0)
    a = _dev_f64(inst["alpha"], dev)
    if a.dim() == 1:
        a = a[None, :]
    n = a.shape[1]
    P = 1 if T == 0 else T - 1
    Tp = 1 if T == 0 else T
    Fd = _dev_f64(inst["F"], dev).reshape(n, -1)
    k = Fd.shape[1]
    Od = _dev_f64(inst["Omega"], dev).reshape(k, k) if k else None
    Ad = _dev_f64(inst["A"], dev)
    Ad = Ad.reshape(-1, n) if Ad is not None and Ad.numel() else None
    m = 0 if Ad is None else Ad.shape[0]
    sd = _dev_f64(inst["s"], dev).reshape(-1, n)
    qd = _dev_f64(inst["q"], dev).reshape(-1, n)
    Ld = _dev_f64(inst["L"], dev).reshape(m) if m else None
    Ud = _dev_f64(inst["U"], dev).reshape(m) if m else None
    dd = _dev_f64(inst["delta"], dev).reshape(n)
    w0d = _dev_f64(inst["w0"], dev).reshape(n)
    wTd = _dev_f64(inst["w_target"], dev).reshape(n) if T else None
    Wd = _dev_f64(W, dev).reshape(P, n)
    if isinstance(Y, (tuple, list)):
        Yd = torch.cat([_dev_f64(y, dev).reshape(-1) for y in Y])
    else:
        Yd = _dev_f64(Y, dev).reshape(-1)
    gw = _dev_f64(grad_w, dev).reshape(P, n)
    g_a = torch.empty((P, n), dtype=torch.float64, device=dev)
    g_s = torch.empty((Tp, n), dtype=torch.float64, device=dev)
    g_F = torch.empty((n, k), dtype=torch.float64, device=dev)
    o = default_options()
    o.tol_rel_kkt = float(tol)
    o.max_iter = int(max_iter)
    o.time_limit_s = float(time_limit_s)
    o.check_every = int(check_every)
    o.verbose = int(verbose)
    info = _Info()
    st = torch.cuda.current_stream(dev) if stream is None else stream
    with torch.cuda.device(dev):
        rc = lib().ffo_adjoint(n, k, m, T, _ptr(a), _ptr(Fd if k else None), _ptr(Od), _ptr(dd), _ptr(sd),
                               _ptr(qd), float(inst["d"]), _ptr(Ad), _ptr(Ld), _ptr(Ud), _ptr(w0d),
                               float(inst["GMV"]), float(inst["lambda1"]), float(inst["lambda2"]),
                               float(inst["lambda3"]), _ptr(wTd), _ptr(Wd), _ptr(Yd), _ptr(gw), float(omega),
                               ctypes.byref(o), ctypes.c_void_p(st.cuda_stream), _ptr(g_a), _ptr(g_s),
                               _ptr(g_F if k else None), ctypes.byref(info))
    inf = Info(**{f[0]: getattr(info, f[0]) for f in _Info._fields_})
    if rc == 1 or (rc in (2, 3)) or (rc != 0 and raise_on_failure):
        raise FolioError(rc, lib().ffo_last_error().decode())
    return g_a, g_s, g_F, inf


def risk_model(R, Fr, mask=None, min_obs: int = 42, device=None, stream=None):
    """Risk model of paper Section 3.2 on the GPU (ffo_risk_model): R [days][n] asset
    returns, Fr [days][p] factor returns, optional mask [days][n] (nonzero = observed).
    Returns (beta [n][p], Sigma_f [p][p], D [n], valid [n] int32) as CUDA tensors; the
    solver takes F = beta, Omega = Sigma_f, delta = sqrt(D)."""
    torch = _torch()
    if not torch.cuda.is_available():
        raise FolioError(3, "no GPU visible to PyTorch: the library has no CPU path")
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    Rd = _dev_f64(R, dev)
    days, n = Rd.shape
    Fd = _dev_f64(Fr, dev).reshape(days, -1)
    p = Fd.shape[1]
    Md = None
    if mask is not None:
        Md = torch.as_tensor(np.asarray(mask) if not isinstance(mask, torch.Tensor) else mask)
        Md = Md.to(device=dev, dtype=torch.uint8).reshape(days, n).contiguous()
    beta = torch.empty((n, p), dtype=torch.float64, device=dev)
    Sf = torch.empty((p, p), dtype=torch.float64, device=dev)
    D = torch.empty(n, dtype=torch.float64, device=dev)
    valid = torch.empty(n, dtype=torch.int32, device=dev)
    st = torch.cuda.current_stream(dev) if stream is None else stream
    with torch.cuda.device(dev):
        rc = lib().ffo_risk_model(days, n, p, _ptr(Rd), _ptr(Fd), _ptr(Md), int(min_obs),
                                  ctypes.c_void_p(st.cuda_stream), _ptr(beta), _ptr(Sf), _ptr(D), _ptr(valid))
    if rc != 0:
        raise FolioError(rc, lib().ffo_last_error().decode())
    return beta, Sf, D, valid


def _folio_fn():
    torch = _torch()

    class _FolioFn(torch.autograd.Function):
        """W* = solve(alpha, s, F; rest) with gradients from the device adjoint.

        forward(alpha [P][n], s [T'][n], F [n][k], rest: dict of the other instance
        fields, opts: dict of solve keywords) -> W [P][n] (float64 CUDA)."""

        @staticmethod
        def forward(ctx, alpha, s, F, rest, opts):
            inst = dict(rest)
            inst["alpha"], inst["s"], inst["F"] = alpha.detach(), s.detach(), F.detach()
            W, info, Y = solve_instance(inst, return_dual=True, **(opts or {}))
            ctx.inst = inst
            ctx.omega = info.omega
            ctx.save_for_backward(W, torch.cat([y.reshape(-1) for y in Y]))
            return W

        @staticmethod
        def backward(ctx, grad_W):
            W, Y = ctx.saved_tensors
            g_a, g_s, g_F, _ = adjoint(ctx.inst, W, Y, grad_W.contiguous(), omega=ctx.omega)
            return g_a, g_s, g_F, None, None

    return _FolioFn


class _LazyFn:
    _fn = None

    def apply(self, *args):
        if _LazyFn._fn is None:
            _LazyFn._fn = _folio_fn()
        return _LazyFn._fn.apply(*args)


FolioFn = _LazyFn()
