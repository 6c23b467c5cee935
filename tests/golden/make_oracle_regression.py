"""Writes oracle_regression.json from the FP64 oracle only (no HIP path):
a few tensor blocks, the demag field, the energy terms and ten RK4 steps of
a small seeded problem.  Re-run only when a change to the oracle's
arithmetic is intended, and name the paper passage that justifies it."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2107_05364_amd import workloads as W  # noqa: E402


def compute():
    c, s = W.grid(4, 3, 2, 5e-9, 4e-9, 3e-9)
    n = c.shape[0]
    P = oracle.Problem(c, s, 8.0e5, 1.3e-11, 0.3, Ku=2.0e4, easy=W.random_unit_vectors(3, n))
    m = W.random_unit_vectors(2, n)
    Ha = [1.5e4, -2.0e4, 3.0e3]
    return {
        "blocks": {"0,0": P.T[0:3, 0:3].tolist(), "0,23": P.T[0:3, 69:72].tolist(),
                   "7,15": P.T[21:24, 45:48].tolist()},
        "demag_first_tiles": P.demag(m)[:4].tolist(),
        "energy": P.energy(m, Ha).tolist(),
        "rk4_10_steps_first_tiles": P.rk4(m, Ha, 5e-14, 10)[:4].tolist(),
    }


if __name__ == "__main__":
    out = compute()
    out["source"] = "tests/golden/make_oracle_regression.py (FP64 oracle only)"
    with open(os.path.join(HERE, "oracle_regression.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("written")
