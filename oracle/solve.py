"""Top-level oracle driver: PDHG, then active-set polish, then the certificate."""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from .pdhg import pdhg
from .polish import polish, certify_dual
from .problem import Problem, normalize, objective, kkt

__all__ = ["solve", "OracleResult"]


@dataclass
class OracleResult:
    W: np.ndarray          # (P, n) optimal decisions
    yA: np.ndarray
    yF: np.ndarray
    yC: np.ndarray
    phi: float             # scaled objective Phi(W)
    paper_obj: float       # -GMV * Phi(W) (paper eq. 1 / eq. 4 without constants)
    gap: float             # Phi(W) - Psi(Y)
    err_bound: float       # bound on ||W - W*||_F from the gap
    rel_kkt: float
    polished: bool
    pdhg_iters: int
    seconds: float
    reason: str = ""


def solve(inst, tol: float = 1e-9, max_iter: int = 400000, require_polish: bool = True,
          verbose: bool = False, start=None) -> OracleResult:
    """Optimal W for a single- or multi-period instance (dict of arrays or Problem).

    Runs the averaged PDHG to relative KKT ``tol``, polishes on the identified active
    set and certifies by a duality gap at rounding level.  If the polish fails, the
    PDHG is tightened by 100x (twice) and the polish retried; ``require_polish``
    raises if it never succeeds.  ``start``: an optional (W, yA, yF, yC) to start the
    PDHG from (e.g. the solution of a nearby instance).
    """
    t0 = time.perf_counter()
    pb = inst if isinstance(inst, Problem) else normalize(inst)
    if start is None:
        r = pdhg(pb, tol=tol, max_iter=max_iter, verbose=verbose)
    else:
        W0, yA0, yF0, yC0 = start
        r = pdhg(pb, tol=tol, max_iter=max_iter, verbose=verbose, W0=W0, Y0=(yA0, yF0, yC0))
    iters = r.iters
    pol = polish(pb, r.W, r.yA, r.yF, r.yC)
    cur_tol = tol
    tries = 0
    while not pol.ok and tries < 2 and pb.g1 > 0:
        cur_tol *= 1e-2
        r = pdhg(pb, tol=cur_tol, max_iter=max_iter, W0=r.W, Y0=(r.yA, r.yF, r.yC), verbose=verbose)
        iters += r.iters
        pol = polish(pb, r.W, r.yA, r.yF, r.yC)
        tries += 1
    if pol.ok:
        W, yA, yF, yC = pol.W, pol.yA, pol.yF, pol.yC
    else:
        if require_polish and pb.g1 > 0:
            raise RuntimeError(f"oracle polish failed: {pol.reason}")
        W, yA, yF, yC = r.W, r.yA, r.yF, r.yC
    po, do, gap, bound = certify_dual(pb, W, yA, yF, yC)
    K = kkt(pb, W, yA, yF, yC)
    return OracleResult(W=W, yA=yA, yF=yF, yC=yC, phi=po, paper_obj=-pb.GMV * po, gap=gap,
                        err_bound=float(bound), rel_kkt=K.rel_kkt, polished=pol.ok,
                        pdhg_iters=iters, seconds=time.perf_counter() - t0, reason=pol.reason)
