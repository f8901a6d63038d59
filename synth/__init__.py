"""Seeded synthetic portfolio markets.

This module only draws random inputs; it holds none of the solver's arithmetic.  The
oracle (``oracle/``), the GPU path (``paper_2604_22625_amd``), the tests and the
benchmark all take their inputs from here, so both sides of every parity check see
bit-identical arrays.

The paper builds its instances from licensed market data (alpha from forward
returns plus volatility-scaled noise, a 6-factor risk model fitted by regression,
spreads from bid/ask quotes, impact coefficients from volume; paper Section 3).
That data is not available, so these generators stand in for it with the value
distributions listed in ``make_config``'s docstring.  Shapes follow the paper's
model (Section 2): a factor risk model Sigma = F Omega F^T + diag(delta^2), linear
spread and power-law impact coefficients, and an exposure matrix whose rows are
sector indicators and factor loadings.
"""
from .markets import (  # noqa: F401
    CONFIGS,
    make_config,
    make_single,
    make_multi,
    make_batch,
    batch_instance,
    ushape_profile_inputs,
    make_tiny,
)
from .paper import (  # noqa: F401
    LAMBDA1_GRID,
    LAMBDA23_GRID,
    N_DATES,
    paper_instance,
    eta_profile,
    returns_panel,
)
