"""Plain FP64 CPU oracle for the portfolio problems of FlashFolio (arXiv 2604.22625).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's CPU
baseline may import this package.  It shares no code with the GPU solver in
``paper_2604_22625_amd`` and imports nothing from it; the two meet only through the
seeded inputs of ``synth``.

What it computes is the plain definition of the two models:

* single-period (paper Section 2.1, eq. 1-3): maximise
  GMV a^T w - l1 GMV^2 w^T S w - l2 GMV s^T|w-w0| - l3 GMV q^T|w-w0|^d
  subject to L <= A w <= U and ||w||_1 <= 1;
* multi-period (paper Section 2.2, eq. 4-6): the sum over t = 1..T of the same
  terms with per-period a_t, s_t, q_t, risk measured against the terminal target
  w_T and costs on the trades w_t - w_{t-1}; w_0 and w_T are given and the
  constraints hold for t = 1..T-1;

with the factor risk matrix S = F Omega F^T + diag(delta^2) (paper Section 3.2).
Everything is carried in the scaled minimisation form

    Phi(W) = sum_t [ -a_t^T w_t + g1 (w_t - c)^T S (w_t - c) ]
           + sum_trades [ g2 s_t^T |u_t| + g3 q_t^T |u_t|^d ],

g1 = l1 GMV, g2 = l2, g3 = l3 (the paper's objective equals -GMV Phi, plus the
constant GMV a_T^T w_T in the multi-period model).

Modules
-------
prox     one-dimensional proximal maps, conjugates, the weighted L1-ball solve
problem  normalisation, Phi, the closed-form dual Psi, feasibility and relative KKT
pdhg     a restarted, averaged, diagonally preconditioned PDHG
polish   active-set identification, Newton on the reduced KKT system, and an exact
         optimality certificate (primal feasibility + a dual point with zero gap)
brute    enumeration of active sets for tiny instances
solve    the top-level driver: pdhg -> polish -> certificate
grad     implicit differentiation of the polished solution
feasibility  minimal budget of the exposure box (LP) and infeasibility certificates
"""
from .problem import Problem, normalize  # noqa: F401
from .solve import solve, OracleResult  # noqa: F401
