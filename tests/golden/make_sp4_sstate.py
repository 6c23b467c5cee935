"""Writes sp4_sstate_n5.json: the standard-problem-4 s-state at resolution
[100, 25, 1] (paper Sec. 4.3), computed by the FP64 oracle alone.

Protocol (the workload's reading of the paper's preparation): start
saturated along [1, 1, 1]; for each field of the staircase along [1, 1, 1]
relax by pure damping (LL with c1 = 0, c2 = gamma0) with adaptive
Dormand-Prince steps (atol = rtol = 1e-6, first step 1e-14 s at every level)
until an accepted step leaves max_a |dm/dt|_a below the threshold.  The state
is stored rounded to float32 (base64 of the little-endian bytes, [n][3]), the
precision in which both paths start the reversal dynamics from it, with its
FP64 mean magnetisation and the attempts per level.

Run: python tests/golden/make_sp4_sstate.py   (a few minutes on 8 cores)."""
import base64
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2107_05364_amd import workloads as W  # noqa: E402

N_RES = 5
OUT = os.path.join(HERE, "sp4_sstate_n%d.json" % N_RES)


def relax(n_res):
    wl = W.sp4_film(n_res)
    c1, c2 = wl.extra["relax_ll"]
    P = oracle.Problem(wl.centers, wl.sizes, wl.Ms, wl.A, c2, gamma0=c1, ll_form=1)
    y = wl.m0[0].astype(np.float64).copy()
    stop = wl.extra["relax_stop"]
    levels = []
    for H in wl.extra["levels"]:
        k1 = P.rhs(y, H)
        dt, t, att = 1e-14, 0.0, 0
        while True:
            ok, dt, t, _, dmx = P.dp45_attempt(y, k1, H, dt, t)
            att += 1
            if ok and dmx < stop:
                break
        levels.append({"field_A_per_m": float(np.linalg.norm(H)), "attempts": att, "t": t})
    return wl, P, y, levels


def main():
    t0 = time.time()
    wl, P, y, levels = relax(N_RES)
    w = P.vol * P.Ms
    mean = (w[:, None] * y).sum(axis=0) / w.sum()
    m32 = np.ascontiguousarray(y, dtype="<f4")
    out = {"source": "FP64 oracle (oracle/), tests/golden/make_sp4_sstate.py; protocol of "
                     "paper_2107_05364_amd.workloads.sp4_film (paper Sec. 4.3 s-state)",
           "resolution": [20 * N_RES, 5 * N_RES, 1], "n": int(y.shape[0]),
           "mean_m_fp64": mean.tolist(), "levels": levels,
           "m_float32_le_base64": base64.b64encode(m32.tobytes()).decode(),
           "seconds": round(time.time() - t0, 1), "oracle_threads": oracle.num_threads()}
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print("wrote", OUT, "mean m", mean, "in %.1f s" % (time.time() - t0))


if __name__ == "__main__":
    main()
