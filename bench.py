#!/usr/bin/env python3
"""Benchmark: adaptive LLG steps per second on one MI355X.

Workload: the standard-problem-4 thin film, 100 x 25 x 1 cuboid tiles of
5 x 5 x 3 nm (N = 2500, dense operator 7500 x 7500), Ms = 8.0e5 A/m,
A = 1.3e-11 J/m, alpha = 0.02, seeded near-saturated in-plane texture and a
seeded in-plane applied field of 10-50 mT.  One step is one attempted
Dormand-Prince 5(4) step of the whole hot path: six fused demag + effective
field + Landau-Lifshitz + stage kernels, the float64 error estimate, step
control and commit, replayed from a hipGraph with all inputs resident in HBM.
The demag operator is assembled once per geometry (float64 on the GPU) and
timed separately.

Prints one JSON line.  Run with no arguments for the default configuration.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--profile-iters", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=60,
                    help="attempted steps of the oracle in the CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def cpu_baseline(wl, nsteps):
    """The FP64 oracle, as it stands, on a bounded sample of the same
    workload: operator assembly once, then `nsteps` attempted DP45 steps."""
    import oracle

    t0 = time.perf_counter()
    P = oracle.Problem(wl.centers, wl.sizes, wl.Ms, wl.A, wl.alpha)
    t_asm = time.perf_counter() - t0
    y = wl.m0[0].astype(np.float32).astype(np.float64)
    Ha = wl.Ha[0].astype(np.float32).astype(np.float64)
    k1 = P.rhs(y, Ha)
    dt, t = 1e-14, 0.0
    t0 = time.perf_counter()
    for _ in range(nsteps):
        _, dt, t, _, _ = P.dp45_attempt(y, k1, Ha, dt, t)
    el = time.perf_counter() - t0
    return {"value": nsteps / el, "unit": "steps/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "%d attempted DP45 steps of the same film workload after one FP64 operator "
                      "assembly (%.1f s, not included)" % (nsteps, t_asm),
            "assembly_s": round(t_asm, 3)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only; --gpus %d is not supported (the multi-GPU "
              "sharding is design-only)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2107_05364_amd import tilemag as tmg
    from paper_2107_05364_amd import workloads as W

    tmg.load()
    wl = W.thin_film()
    n = wl.n
    ctx = tmg.Context(0)
    geom = tmg.Geometry(ctx, wl.centers, wl.sizes)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T = tmg.Tensor(ctx, geom, tmg.TM_PREC_FP32, tmg.TM_LAYOUT_SYM6)
    torch.cuda.synchronize()
    asm_ms = (time.perf_counter() - t0) * 1e3
    p = tmg.Problem(ctx, geom, T, wl.Ms, wl.A, wl.alpha, wl.gamma0)

    m = torch.as_tensor(wl.m0.astype(np.float32), device="cuda")
    Ha = torch.as_tensor(wl.Ha.astype(np.float32), device="cuda")
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt = torch.full((1,), 1e-14, dtype=torch.float64, device="cuda")
    big = 1 << 40
    # warmup (graph capture happens here)
    p.run(m, Ha, tmg.TM_DP45, dt=dt, t=t, max_steps=big, max_attempts=max(1, args.warmup))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tt, dd, steps, st = p.run(m, Ha, tmg.TM_DP45, dt=dt, t=t, max_steps=big,
                              max_attempts=args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    assert torch.isfinite(m).all().item(), "non-finite state after the timed run"
    accepted = int(steps.cpu()[0])

    # dominant kernel: the fused field/stage kernel, timed with HIP events on
    # the stream it runs on
    avg_ms, bytes_per = tmg.tm_profile_field(p.handle, 1, args.profile_iters)
    achieved = bytes_per / (avg_ms * 1e-3) / 1e9

    rec = {
        "metric": "LLG steps/s",
        "value": round(args.steps / el, 2),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el * 1e3 / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "SP4 thin film 100x25x1 tiles of 5x5x3 nm (N=2500), one state, "
                               "adaptive DP45, fp32 SYM6 operator",
                   "n_tiles": n, "batch": 1, "integrator": "DP45", "operator": "fp32 sym6",
                   "accepted_steps": accepted, "rejected_steps": int(st.rejected),
                   "simulated_ns": round(float(tt.cpu()[0]) * 1e9, 4),
                   "assembly_ms": round(asm_ms, 2)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_field<256,4,STAGE> (fused demag matvec + H_eff + LL + stage)",
                     "avg_launch_us": round(avg_ms * 1e3, 3), "bytes_per_launch": bytes_per},
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(wl, args.cpu_steps)
    p.close()
    T.close()
    geom.close()
    ctx.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
