"""Write the oracle's certified solutions of the full-size workloads to tests/golden/.

Calls only the oracle (and the seeded input generator).  Usage:
    python tests/golden/make_golden.py c1      # single-period n=5000, seed 1
    python tests/golden/make_golden.py c1:4    # the same market with seed 4
    python tests/golden/make_golden.py c2      # multi-period T=20, n=3000, seed 20
    python tests/golden/make_golden.py c4      # multi-period T=10, n=2000, seed 40
    python tests/golden/make_golden.py c4fd    # central differences of the c4 loss (see below)
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


def c4_differences():
    """Central differences of the loss l = r^T w_{T-1} (the c4 workload's loss on the last
    decision) along seeded random directions of alpha, s and F, from the oracle's
    certified solves of the perturbed instances (warm-started at the base solution).
    Stored: directions' seed, steps, derivative estimates and whether the active pieces
    of the two perturbed solutions agree (a difference across a kink is no derivative)."""
    from oracle.grad import piece_of
    from oracle.problem import normalize
    t0 = time.time()
    inst = make_config(4, seed=40)
    base = oracle.solve(inst, tol=1e-11)
    P, n = np.atleast_2d(inst["alpha"]).shape
    gW = np.zeros((P, n))
    gW[-1] = inst["r"]
    rng = np.random.default_rng(7)
    out = {"W": base.W, "seed": 7}
    for key, h in (("alpha", 1e-7), ("s", 1e-7), ("F", 1e-6)):
        d = rng.normal(size=np.asarray(inst[key]).shape)
        vals, pieces = [], []
        for sgn in (1.0, -1.0):
            q = dict(inst)
            q[key] = inst[key] + sgn * h * d
            r = oracle.solve(q, tol=1e-11, start=(base.W, base.yA, base.yF, base.yC))
            vals.append(float(np.sum(gW * r.W)))
            pc = piece_of(normalize(q), r.W)
            pieces.append((pc.zero_trade, pc.zero_w, pc.tight))
        same = all(np.array_equal(a, b) for a, b in zip(pieces[0], pieces[1]))
        out[f"fd_{key}"] = (vals[0] - vals[1]) / (2.0 * h)
        out[f"h_{key}"] = h
        out[f"same_piece_{key}"] = same
        print(f"{key}: fd {out[f'fd_{key}']:.12e} same piece {same} ({time.time() - t0:.0f} s)", flush=True)
    path = os.path.join(HERE, "c4_seed40_differences.npz")
    np.savez_compressed(path, **out)
    print(path, flush=True)


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["c1"]:
        if nm == "c4fd":
            c4_differences()
        else:
            main(nm)
