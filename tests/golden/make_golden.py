"""Write the oracle's certified solutions of the full-size workloads to tests/golden/.

Calls only the oracle (and the seeded input generator).  Usage:
    python tests/golden/make_golden.py c1      # single-period n=5000, seed 1
    python tests/golden/make_golden.py c1:4    # the same market with seed 4
    python tests/golden/make_golden.py c2      # multi-period T=20, n=3000, seed 20
    python tests/golden/make_golden.py c4      # multi-period T=10, n=2000, seed 40
Each file holds W* (float64), Phi*, the certified duality gap and the error bound.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import make_config  # noqa: E402

WHICH = {"c1": (1, 1), "c2": (2, 20), "c4": (4, 40)}


def main(name):
    name, _, sd = name.partition(":")
    cfg, seed = WHICH[name]
    seed = int(sd) if sd else seed
    t0 = time.time()
    r = oracle.solve(make_config(cfg, seed=seed), tol=1e-9)
    out = os.path.join(HERE, f"{name}_seed{seed}_oracle.npz")
    np.savez_compressed(out, W=r.W, phi=r.phi, gap=r.gap, err_bound=r.err_bound, polished=r.polished)
    print(f"{out}: polished {r.polished} phi {r.phi:.15e} gap {r.gap:.2e} bound {r.err_bound:.2e} "
          f"({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["c1"]:
        main(nm)
