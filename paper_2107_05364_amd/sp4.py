"""Standard problem 4 on the device (paper Sec. 4.3, the timing experiment of
its Fig. 5b): the s-state preparation and the reversal dynamics, as
sequences of tm_run calls on one operator (argument marshalling only; every
step runs in the HIP library).

* s-state: the film starts saturated along [1, 1, 1]; a staircase of fields
  along [1, 1, 1] is removed level by level, each level relaxed by pure
  damping (LL with c1 = 0, c2 = gamma0) to max_a |dm/dt|_a below the
  workload's threshold.
* dynamics: from the s-state, field 1 or field 2 switched on at t = 0 with the
  paper's LL parameters (c1 = gamma = 2.21e5, c2 = alpha = 4.42e3), adaptive
  Dormand-Prince to the end time.
"""
from __future__ import annotations

import time

import numpy as np

from . import tilemag as tmg


def prepare_sstate(ctx, geom, tensor, wl, max_steps=200000, dt0=1e-14):
    """Relaxes wl.m0 through the field staircase on the device; returns
    (m [1, n, 3] device tensor, per-level records with the device
    diagnostics' <m> after each level)."""
    import torch

    c1, c2 = wl.extra["relax_ll"]
    p = tmg.Problem(ctx, geom, tensor, wl.Ms, wl.A, alpha=c2, gamma0=c1, ll_form=1)
    m = torch.as_tensor(np.ascontiguousarray(wl.m0, np.float32), device="cuda")
    levels = []
    try:
        for H in wl.extra["levels"]:
            Ha = torch.as_tensor(np.asarray(H, np.float32)[None], device="cuda")
            t0 = time.perf_counter()
            t, dt, steps, st = p.run(m, Ha, tmg.TM_DP45, dt=dt0, max_steps=max_steps,
                                     dmdt_stop=wl.extra["relax_stop"])
            D = p.diagnostics(m, Ha).cpu().numpy()[0]
            levels.append({"field_A_per_m": float(np.linalg.norm(H)), "accepted": int(st.accepted_max),
                           "rejected": int(st.rejected), "attempts": int(st.attempts),
                           "t": float(t.cpu()[0]), "seconds": time.perf_counter() - t0,
                           "mean_m": [float(x) for x in D[4:7]]})
    finally:
        p.close()
    return m, levels


def dynamics(ctx, geom, tensor, wl, m_start, field, t_end=None, dt0=1e-14, max_steps=10_000_000,
             tune_iters=0):
    """Integrates a copy of the s-state under reversal field `field` (1 or 2)
    from t = 0 to t_end (default: the workload's duration); returns
    (m [1, n, 3] device tensor at t_end, run stats, wall seconds, <m> at t_end
    from the device diagnostics).  tune_iters > 0 first runs the autotuner on
    the new problem (not timed)."""
    import torch

    c1, c2 = wl.extra["dyn_ll"]
    p = tmg.Problem(ctx, geom, tensor, wl.Ms, wl.A, alpha=c2, gamma0=c1, ll_form=1)
    try:
        if tune_iters:
            tmg.tm_problem_tune(p.handle, 1, tune_iters)  # launch shape / tile-pass loads, untimed
        m = m_start.clone()
        Ha = torch.as_tensor(np.asarray(wl.extra["fields"][field], np.float32)[None], device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t, dt, steps, st = p.run(m, Ha, tmg.TM_DP45, dt=dt0, max_steps=max_steps,
                                 t_end=wl.extra["dyn_time"] if t_end is None else t_end)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        mean = p.diagnostics(m, Ha).cpu().numpy()[0, 4:7].astype(np.float64)
    finally:
        p.close()
    return m, st, wall, mean
