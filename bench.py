#!/usr/bin/env python3
"""Benchmark: adaptive LLG steps per second on one MI355X.

Workload: the standard-problem-4 thin film, 100 x 25 x 1 cuboid tiles of
5 x 5 x 3 nm (N = 2500, dense operator 7500 x 7500), Ms = 8.0e5 A/m,
A = 1.3e-11 J/m, alpha = 0.02, seeded near-saturated in-plane texture and a
seeded in-plane applied field of 10-50 mT.  One step is one attempted
Dormand-Prince 5(4) step of the whole hot path: six evaluations of the demag
product with the effective field, the Landau-Lifshitz right-hand side and
the stage update, the float64 error estimate, step control and commit,
replayed from a hipGraph with all inputs resident in HBM.  The film's tiles
are identical, so the default operator is the pair-symmetric one (each pair
of blocks stored once; --layout sym6 streams all six planes instead).  The
demag operator is assembled once per geometry (float64 on the GPU) and timed
separately.

Prints one JSON line.  Run with no arguments for the default configuration.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

_T_START = time.perf_counter()

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--profile-iters", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=1000,
                    help="attempted steps of the oracle in the CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--no-cube", action="store_true")
    ap.add_argument("--no-peaks", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-threshold", action="store_true")
    ap.add_argument("--no-sp3", action="store_true")
    ap.add_argument("--no-cache-free", action="store_true")
    ap.add_argument("--no-sp4-dynamics", action="store_true")
    ap.add_argument("--tile-loads", choices=["auto", "cached", "nontemporal"], default="auto",
                    help="pair-symmetric layouts: operator loads of the tile pass (auto: the autotuner's pick)")
    ap.add_argument("--profile-batch", type=int, default=1,
                    help="--profile-only: states integrated together (a batch reads each operator tile "
                         "once per tile pass)")
    ap.add_argument("--profile-film", choices=["100x25", "160x40"], default="100x25",
                    help="film of the counter runs (--profile-only): the headline N = 2500, or N = 6400 "
                         "whose operator exceeds the Infinity Cache")
    ap.add_argument("--profile-only", action="store_true",
                    help="counter runs: one 1 GiB device copy (calibration) and the stage kernel "
                         "of the film workload only")
    ap.add_argument("--serving-count", type=int, default=40,
                    help="requests of the serving stream (the full stream has 200)")
    ap.add_argument("--serving-nmax", type=int, default=20000,
                    help="largest tile count of the serving stream (log-uniform from 500)")
    ap.add_argument("--serving-max-active", type=int, default=3,
                    help="groups the server advances per round, oldest first (0: all)")
    ap.add_argument("--layout", choices=["psym4", "psym6", "sym6"], default="psym4",
                    help="operator layout of the headline run: pair-symmetric with four planes "
                         "(the film is one layer of identical tiles), pair-symmetric with six "
                         "planes, or six planes")
    return ap.parse_args()


# dominant kernel of each headline layout: its sources and committed counter summary
KERNELS = {
    "sym6": (["paper_2107_05364_amd/csrc/fieldstep.hip", "paper_2107_05364_amd/csrc/epilogue.h",
              "paper_2107_05364_amd/csrc/common.h"],
             os.path.join(ROOT, "profiles", "k_field_stage_film_N2500_counters.md")),
    "psym6": (["paper_2107_05364_amd/csrc/psym.hip", "paper_2107_05364_amd/csrc/epilogue.h",
               "paper_2107_05364_amd/csrc/common.h"],
              os.path.join(ROOT, "profiles", "k_psym_tiles_film_N2500_counters.md")),
    "psym4": (["paper_2107_05364_amd/csrc/psym.hip", "paper_2107_05364_amd/csrc/epilogue.h",
               "paper_2107_05364_amd/csrc/common.h"],
              os.path.join(ROOT, "profiles", "k_psym_tiles_4planes_film_N2500_counters.md")),
}
LAYOUT_CODE = {"sym6": 0, "psym6": 3, "psym4": 4}  # tm_layout values


def kernel_source_hash(layout):
    h = hashlib.sha256()
    for f in KERNELS[layout][0]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def progress(section):
    """One line per benchmark section on stderr (stdout carries only the
    result line), so that a long default run shows it is alive."""
    print("bench: %s (%.0f s)" % (section, time.perf_counter() - _T_START), file=sys.stderr, flush=True)


def _same_pass(a, b):
    """The pair-symmetric tile pass reads the same operator bytes with cached
    or with nontemporal operator loads (the autotuner picks either): its two
    load variants count as one kernel here."""
    import re

    def norm(k):
        k = re.sub(r"\s+", "", k.split("(")[0])
        return re.sub(r"^k_psym_tiles<true,true,(true|false),(\d),(true|false)>$", r"k_psym_tiles<true,true,*,\2,\3>", k)

    return norm(a) == norm(b)


def counter_traffic(layout, kname):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE runs, calibrated against a 1 GiB copy),
    or None when the kernel sources or the kernel instance changed since."""
    try:
        text = open(KERNELS[layout][1]).read()
    except OSError:
        return None
    vals = dict(ln.split(":", 1) for ln in text.splitlines() if ln.startswith(("source_hash:", "kernel:", "traffic_bytes_per_launch:")))
    if vals.get("source_hash", "").strip() != kernel_source_hash(layout) or not _same_pass(vals.get("kernel", ""), kname):
        return None
    return int(vals["traffic_bytes_per_launch"].strip())


def cpu_baseline(wl, nsteps, m_final=None, hd_final=None, batched=None):
    """The FP64 oracle, as it stands, on a bounded sample of the same
    workload: operator assembly once, then `nsteps` attempted DP45 steps.
    The same leg states the GPU results' errors against the oracle: H_d of
    the headline run's final state, and H_d of the batched states for each
    storage precision (one FP64 product with the oracle's dense operator)."""
    import oracle

    t0 = time.perf_counter()
    P = oracle.Problem(wl.centers, wl.sizes, wl.Ms, wl.A, wl.alpha)
    t_asm = time.perf_counter() - t0
    y = wl.m0[0].astype(np.float32).astype(np.float64)
    Ha = wl.Ha[0].astype(np.float32).astype(np.float64)
    k1 = P.rhs(y, Ha)
    dt, t = 1e-14, 0.0
    cores = oracle.num_threads()
    t0 = time.perf_counter()
    for _ in range(nsteps):
        _, dt, t, _, _ = P.dp45_attempt(y, k1, Ha, dt, t)
    el = time.perf_counter() - t0
    # single thread, on a tenth of the sample
    oracle.set_num_threads(1)
    n1 = max(1, nsteps // 10)
    t0 = time.perf_counter()
    for _ in range(n1):
        _, dt, t, _, _ = P.dp45_attempt(y, k1, Ha, dt, t)
    el1 = time.perf_counter() - t0
    oracle.set_num_threads(cores)
    base = {"value": nsteps / el, "unit": "steps/s", "cores": cores, "kind": "oracle",
            "sample": "%d attempted DP45 steps of the same film workload after one FP64 operator "
                      "assembly (%.1f s, not included); single-thread rate from %d further steps"
                      % (nsteps, t_asm, n1),
            "single_thread_steps_per_s": round(n1 / el1, 2), "assembly_s": round(t_asm, 3)}
    errs = {}
    if m_final is not None:
        want = P.demag(m_final.astype(np.float64))
        errs["headline"] = rel_errors(hd_final, want)
    if batched:
        # the oracle's dense FP64 operator of the batched film (same geometry
        # and Ms), one product for all states
        A = oracle.assemble(batched["centers"], batched["sizes"])
        m32 = batched["m"].astype(np.float64)
        B = m32.shape[0]
        ref = -(batched["Ms"] * m32.reshape(B, -1)) @ A.T
        del A
        for name, hd in batched["hd"].items():
            errs["batched_" + name] = rel_errors(hd.reshape(B, -1), ref)
    return base, errs


def rel_errors(got, want):
    """Relative 2-norm and max-norm errors of a GPU result against the oracle."""
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    d = got - want
    return {"rel_err_2norm": float(np.linalg.norm(d) / np.linalg.norm(want)),
            "rel_err_max": float(np.abs(d).max() / np.abs(want).max())}


def batched_section(tmg, W, torch, attempts=60, profile_iters=20):
    """B = 128 states on the film geometry sharing one DENSE9 operator: one
    MFMA GEMM per right-hand side, in float32 and in bf16 / fp16 hi + lo
    split precision.  Returns the record and the GPU H_d of the initial
    states per precision, whose errors the oracle leg states."""
    wl = W.hysteresis_batch(B=128)
    n, B = wl.n, wl.batch
    ctx = tmg.Context(0)
    geom = tmg.Geometry(ctx, wl.centers, wl.sizes)
    m32 = wl.m0.astype(np.float32)
    Ha = torch.as_tensor(wl.Ha.astype(np.float32), device="cuda")
    out = {"workload": "hysteresis film 100x25x1 (N=2500), B=128 states, +80..-80 mT, DP45",
           "err_reference": "H_d of the initial states against the FP64 oracle (its dense operator, "
                            "one FP64 product on the host), stated by the cpu_baseline leg"}
    hds = {}
    peaks = {"fp32": 157.3, "bf16x3": 2500.0, "fp16x3": 2500.0}
    for prec, name in ((tmg.TM_PREC_FP32, "fp32"), (tmg.TM_PREC_BF16X3, "bf16x3"),
                       (tmg.TM_PREC_FP16X3, "fp16x3")):
        T = tmg.Tensor(ctx, geom, prec, tmg.TM_LAYOUT_DENSE9)
        p = tmg.Problem(ctx, geom, T, wl.Ms, wl.A, wl.alpha, wl.gamma0)
        ksplits, _ = tmg.tm_problem_tune(p.handle, B, 5)  # K splits of the product
        m = torch.as_tensor(m32, device="cuda")
        hds[name] = p.demag(m).cpu().numpy()
        rhs_ms, _ = tmg.tm_profile_field(p.handle, B, profile_iters)
        # inside an attempt every stage but the first reads the right operand
        # its previous stage wrote (no conversion pass)
        rhs_chain_ms, _ = tmg.tm_profile_field_mode(p.handle, B, 4, profile_iters)
        # a single layer: the operator is stored without its two zero blocks
        # (5 of the 9 components per block pair; bytes and products alike)
        comps = 5 if np.all(wl.centers[:, 2] == wl.centers[0, 2]) else 9
        flops = 2.0 * comps * n * n * B * (3 if name != "fp32" else 1)
        op_bytes = 4.0 * comps * n * n
        p.run(m, Ha, tmg.TM_DP45, dt=1e-14, max_steps=1 << 40, max_attempts=10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tt, dd, steps, st = p.run(m, Ha, tmg.TM_DP45, dt=1e-14, max_steps=1 << 40,
                                  max_attempts=attempts)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[name] = {"state_steps_per_s": round(B * attempts / el, 1),
                     "ms_per_step": round(el * 1e3 / attempts, 4),
                     "rhs_us": round(rhs_ms * 1e3, 2),
                     "rhs_in_attempt_us": round(rhs_chain_ms * 1e3, 2),
                     "mfma_tflops": round(flops / (rhs_ms * 1e-3) / 1e12, 2),
                     "mfma_frac": round(flops / (rhs_ms * 1e-3) / 1e12 / peaks[name], 4),
                     "operator_gbs": round(op_bytes / (rhs_ms * 1e-3) / 1e9, 1),
                     "k_splits_tuned": ksplits,
                     "accepted_min": int(st.accepted_min), "rejected": int(st.rejected)}
        p.close()
        T.close()
    geom.close()
    ctx.close()
    return out, {"centers": wl.centers, "sizes": wl.sizes, "Ms": wl.Ms, "m": m32, "hd": hds}


def tile_loads_choice(tmg, p, psym, forced, iters):
    """The pair-symmetric tile pass's operator loads: the autotuner's pick, or
    the one asked for (profiling runs: the profiler slows the timed
    candidates unevenly, so they name the pick of an unprofiled run)."""
    choice, _ = tmg.tm_problem_tune(p.handle, 1, iters)
    if psym and forced != "auto":
        choice = 1 if forced == "nontemporal" else 0
        tmg.tm_problem_apply(p.handle, choice)
    return choice


def cache_free_section(tmg, W, torch, layout, attempts=20, tile_loads="auto"):
    """The headline's operator pass on an operator larger than the 256 MB
    Infinity Cache: the SP4 film at [160, 40, 1] tiles (N = 6400; PSYM4
    327.7 MB, PSYM6 491.6 MB, SYM6 983 MB), timed inside DP45 steps like
    the headline."""
    wl = W.thin_film(nx=160, ny=40)
    n = wl.n
    ctx = tmg.Context(0)
    geom = tmg.Geometry(ctx, wl.centers, wl.sizes)
    T = tmg.Tensor(ctx, geom, tmg.TM_PREC_FP32, LAYOUT_CODE[layout])
    p = tmg.Problem(ctx, geom, T, wl.Ms, wl.A, wl.alpha, wl.gamma0)
    choice = tile_loads_choice(tmg, p, layout in ("psym4", "psym6"), tile_loads, 10)
    m = torch.as_tensor(wl.m0.astype(np.float32), device="cuda")
    Ha = torch.as_tensor(wl.Ha.astype(np.float32), device="cuda")
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt = torch.full((1,), 1e-14, dtype=torch.float64, device="cuda")
    p.run(m, Ha, tmg.TM_DP45, dt=dt, t=t, max_steps=1 << 40, max_attempts=5)
    op_ms, op_n = tmg.tm_profile_run(p.handle, n, tmg.TM_DP45, m, Ha, t, dt,
                                     tmg.tm_run_cfg(1 << 40, attempts, 0.0, 1e-6, 1e-6, 0.0, 0.0, 1, 0, 64))
    _, stored = tmg.tm_profile_field(p.handle, 1, 5)
    p.close()
    T.close()
    geom.close()
    ctx.close()
    if layout == "sym6":
        alg = 24 * n * n + 24 * n
    else:
        alg = n * (n + 1) // 2 * (4 if layout == "psym4" else 6) * 4 + 24 * n
    avg = op_ms / op_n
    return {"workload": "SP4 film [160,40,1] tiles (N=%d), %s operator %.1f MB as stored" % (n, layout.upper(), stored / 1e6),
            "tile_pass_loads" if layout != "sym6" else "stage_kernel_shape":
                (("nontemporal" if choice == 1 else "cached") if layout != "sym6" else choice),
            "avg_launch_us": round(avg * 1e3, 3), "launches_timed": op_n, "bytes_per_launch": alg,
            "achieved": round(alg / (avg * 1e-3) / 1e9, 1), "frac": round(alg / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def large_section(tmg, W, torch, attempts=20, profile_iters=10, with_oracle=True):
    """The 20000-tile refined slab (edges 2.5-20 nm, 1000 x 250 x 20 nm): FP64
    operator assembly on the GPU, the stage kernel streaming a 9.6 GB SYM6
    operator (no cache can hold it: the HBM roofline proper), a few single-state
    DP45 steps, and 32 states through the DENSE9 bf16 hi+lo GEMM path."""
    wl = W.refined_slab(n_target=20000, B=32)
    n = wl.n
    ctx = tmg.Context(0)
    geom = tmg.Geometry(ctx, wl.centers, wl.sizes)
    out = {"workload": "refined slab N=%d (%d ordered face pairs), alpha=0.1" % (n, geom.nfaces)}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T = tmg.Tensor(ctx, geom, tmg.TM_PREC_FP32, tmg.TM_LAYOUT_SYM6)
    torch.cuda.synchronize()
    asm = time.perf_counter() - t0
    out["assembly_ms"] = round(asm * 1e3, 1)
    out["assembly_gpairs_s"] = round(n * n / asm / 1e9, 2)
    if with_oracle:
        import oracle

        rows = np.arange(0, n, n // 64)[:64]
        t0 = time.perf_counter()
        oracle.demag_rows(wl.centers, wl.sizes, wl.Ms, wl.m0[0].astype(np.float64), rows)
        el = time.perf_counter() - t0
        out["oracle_tensor_gpairs_s"] = round(len(rows) * n / el / 1e9, 4)
        out["oracle_sample"] = "%d target rows x %d sources evaluated on the fly (%d threads)" % (
            len(rows), n, oracle.num_threads())
    p = tmg.Problem(ctx, geom, T, wl.Ms, wl.A, wl.alpha, wl.gamma0)
    shape, _ = tmg.tm_problem_tune(p.handle, 1, 3)
    out["stage_kernel_shape"] = shape
    ms, nb = tmg.tm_profile_field(p.handle, 1, profile_iters)
    out["stage_kernel_us"] = round(ms * 1e3, 1)
    out["stage_kernel_gbs"] = round(nb / (ms * 1e-3) / 1e9, 1)
    out["stage_kernel_hbm_frac"] = round(nb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    m = torch.as_tensor(wl.m0[:1].astype(np.float32), device="cuda")
    p.run(m, None, tmg.TM_DP45, dt=1e-14, max_steps=1 << 40, max_attempts=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p.run(m, None, tmg.TM_DP45, dt=1e-14, max_steps=1 << 40, max_attempts=attempts)
    torch.cuda.synchronize()
    out["single_steps_per_s"] = round(attempts / (time.perf_counter() - t0), 2)
    p.close()
    T.close()
    T9 = tmg.Tensor(ctx, geom, tmg.TM_PREC_BF16X3, tmg.TM_LAYOUT_DENSE9)
    p9 = tmg.Problem(ctx, geom, T9, wl.Ms, wl.A, wl.alpha, wl.gamma0)
    m = torch.as_tensor(wl.m0.astype(np.float32), device="cuda")
    out["batch32_k_splits_tuned"], _ = tmg.tm_problem_tune(p9.handle, 32, 5)
    ms, _ = tmg.tm_profile_field(p9.handle, 32, profile_iters)
    out["batch32_bf16x3_rhs_us"] = round(ms * 1e3, 1)
    out["batch32_bf16x3_operator_gbs"] = round(36.0 * n * n / (ms * 1e-3) / 1e9, 1)
    p9.run(m, None, tmg.TM_DP45, dt=1e-14, max_steps=1 << 40, max_attempts=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p9.run(m, None, tmg.TM_DP45, dt=1e-14, max_steps=1 << 40, max_attempts=attempts)
    torch.cuda.synchronize()
    out["batch32_state_steps_per_s"] = round(32 * attempts / (time.perf_counter() - t0), 2)
    p9.close()
    T9.close()
    geom.close()
    ctx.close()
    return out


def cube_section(tmg, W, torch, reps=5, with_oracle=True):
    """The 8 x 8 x 8 grid of 5 nm cubes (N = 512), RK4 at dt = 1e-13 s for
    200 steps with the float32 SYM6 operator (6 MB, cache-resident): a
    launch- and latency-bound case, run as captured graphs of four stage
    launches per step and as one persistent cooperative launch for the
    whole run (operator rows resident in LDS, a grid barrier per stage)."""
    wl = W.cube_grid()
    nsteps = wl.extra["steps"]
    ctx = tmg.Context(0)
    geom = tmg.Geometry(ctx, wl.centers, wl.sizes)
    T = tmg.Tensor(ctx, geom, tmg.TM_PREC_FP32, tmg.TM_LAYOUT_SYM6)
    p = tmg.Problem(ctx, geom, T, wl.Ms, wl.A, wl.alpha, wl.gamma0)
    m = torch.as_tensor(wl.m0.astype(np.float32), device="cuda")
    def best_of(persistent):
        p.run(m.clone(), None, tmg.TM_RK4, dt=wl.extra["dt"], max_steps=nsteps, persistent=persistent)
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(reps):
            mm = m.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p.run(mm, None, tmg.TM_RK4, dt=wl.extra["dt"], max_steps=nsteps, persistent=persistent)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return best

    best_graph = best_of(False)
    best_pers = best_of(True)
    best = min(best_graph, best_pers)
    ms, nb = tmg.tm_profile_field(p.handle, 1, 50)
    p.close()
    T.close()
    geom.close()
    ctx.close()
    out = {"workload": "8x8x8 cubes of 5 nm (N=512), alpha=0.5, RK4 dt=1e-13 s x %d steps, fp32 SYM6" % nsteps,
           "steps_per_s": round(nsteps / best, 1), "us_per_step": round(best / nsteps * 1e6, 2),
           "steps_per_s_graph": round(nsteps / best_graph, 1),
           "steps_per_s_persistent": round(nsteps / best_pers, 1),
           "stage_kernel_us": round(ms * 1e3, 2)}
    if with_oracle:
        import oracle

        t0 = time.perf_counter()
        P = oracle.Problem(wl.centers, wl.sizes, wl.Ms, wl.A, wl.alpha)
        t_asm = time.perf_counter() - t0
        t0 = time.perf_counter()
        P.rk4(wl.m0[0].astype(np.float32).astype(np.float64), [0, 0, 0], wl.extra["dt"], nsteps)
        el = time.perf_counter() - t0
        out["oracle"] = {"steps_per_s": round(nsteps / el, 1), "assembly_s": round(t_asm, 3),
                         "cores": oracle.num_threads(), "sample": "the full run (assembly + %d RK4 steps)" % nsteps}
    return out


def sp4_sweep_section(tmg, W, torch, attempts=300):
    """The standard-problem-4 film at [20n, 5n, 1] tiles (edges 25/n x 25/n x
    3 nm), n = 1..9 (N = 100 n^2): per-size stage-kernel time and bandwidth
    (fp32 SYM6, tuned launch shape) and single-state DP45 steps per second."""
    rows = []
    for nn in range(1, 10):
        wl = W.thin_film(nx=20 * nn, ny=5 * nn)
        ctx = tmg.Context(0)
        geom = tmg.Geometry(ctx, wl.centers, wl.sizes)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        T = tmg.Tensor(ctx, geom, tmg.TM_PREC_FP32, tmg.TM_LAYOUT_SYM6)
        torch.cuda.synchronize()
        asm = time.perf_counter() - t0
        p = tmg.Problem(ctx, geom, T, wl.Ms, wl.A, wl.alpha, wl.gamma0)
        shape, _ = tmg.tm_problem_tune(p.handle, 1, 10)
        ms, nb = tmg.tm_profile_field(p.handle, 1, 50)
        Ha = torch.as_tensor(wl.Ha.astype(np.float32), device="cuda")

        def steps_per_s(prob):
            m = torch.as_tensor(wl.m0.astype(np.float32), device="cuda")
            dt = torch.full((1,), 1e-14, dtype=torch.float64, device="cuda")
            prob.run(m, Ha, tmg.TM_DP45, dt=dt, max_steps=1 << 40, max_attempts=20)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            prob.run(m, Ha, tmg.TM_DP45, dt=dt, max_steps=1 << 40, max_attempts=attempts)
            torch.cuda.synchronize()
            return attempts / (time.perf_counter() - t0)

        row = {"n": nn, "tiles": wl.n, "assembly_ms": round(asm * 1e3, 2), "shape": shape,
               "stage_kernel_us": round(ms * 1e3, 2),
               "stage_kernel_gbs": round(nb / (ms * 1e-3) / 1e9, 1),
               "steps_per_s": round(steps_per_s(p), 1)}
        p.close()
        T.close()
        # the same film with the pair-symmetric operator (identical tiles)
        Tp = tmg.Tensor(ctx, geom, tmg.TM_PREC_FP32, tmg.TM_LAYOUT_PSYM6)
        pp = tmg.Problem(ctx, geom, Tp, wl.Ms, wl.A, wl.alpha, wl.gamma0)
        tmg.tm_problem_tune(pp.handle, 1, 10)
        msp, nbp = tmg.tm_profile_field(pp.handle, 1, 50)
        row.update({"psym6_field_us": round(msp * 1e3, 2), "psym6_steps_per_s": round(steps_per_s(pp), 1)})
        pp.close()
        Tp.close()
        # and with its four planes (one layer: xz = yz = 0)
        T4 = tmg.Tensor(ctx, geom, tmg.TM_PREC_FP32, tmg.TM_LAYOUT_PSYM4)
        p4 = tmg.Problem(ctx, geom, T4, wl.Ms, wl.A, wl.alpha, wl.gamma0)
        tmg.tm_problem_tune(p4.handle, 1, 10)
        ms4, _ = tmg.tm_profile_field(p4.handle, 1, 50)
        row.update({"psym4_field_us": round(ms4 * 1e3, 2), "psym4_steps_per_s": round(steps_per_s(p4), 1)})
        rows.append(row)
        p4.close()
        T4.close()
        geom.close()
        ctx.close()
    return {"workload": "SP4 film [20n,5n,1] tiles, n=1..9, one state, DP45, fp32 SYM6 (and PSYM6, PSYM4)", "sizes": rows}


def sp4_dynamics_section(tmg, W, torch, ns=range(1, 10), layouts=("psym4", "psym6", "sym6")):
    """The paper's standard-problem-4 timing experiment (Sec. 4.3, Fig. 5b):
    for each resolution [20n, 5n, 1] the s-state is prepared on the device
    (field staircase along [1, 1, 1], pure-damping relaxation; timed apart,
    as the paper leaves it out), then the dynamic part -- field 1 and field 2
    switched on at t = 0 with the paper's LL parameters, adaptive DP45 to
    1 ns -- is timed per operator layout."""
    from paper_2107_05364_amd import sp4

    rows = []
    t_all = time.perf_counter()
    for nn in ns:
        wl = W.sp4_film(nn)
        ctx = tmg.Context(0)
        geom = tmg.Geometry(ctx, wl.centers, wl.sizes)
        tensors = {name: tmg.Tensor(ctx, geom, tmg.TM_PREC_FP32, LAYOUT_CODE[name]) for name in layouts}
        t0 = time.perf_counter()
        m_s, levels = sp4.prepare_sstate(ctx, geom, tensors[layouts[0]], wl)
        torch.cuda.synchronize()
        row = {"n": nn, "tiles": wl.n,
               "sstate": {"seconds": round(time.perf_counter() - t0, 3), "layout": layouts[0],
                          "attempts": sum(lv["attempts"] for lv in levels),
                          "mean_m": [round(x, 6) for x in levels[-1]["mean_m"]]}}
        for name in layouts:
            rec = {}
            for field in (1, 2):
                m, st, wall, mean = sp4.dynamics(ctx, geom, tensors[name], wl, m_s, field, tune_iters=5)
                rec["field%d" % field] = {"seconds": round(wall, 4), "attempts": int(st.attempts),
                                          "accepted": int(st.accepted_max), "rejected": int(st.rejected),
                                          "mean_m_1ns": [round(float(x), 6) for x in mean]}
            rec["seconds_both_fields"] = round(rec["field1"]["seconds"] + rec["field2"]["seconds"], 4)
            row[name] = rec
        rows.append(row)
        for T in tensors.values():
            T.close()
        geom.close()
        ctx.close()
    return {"workload": "SP4 film [20n,5n,1], n=1..9: s-state (staircase 1000..0 mT along [1,1,1], pure "
                        "damping to max|dm/dt| < 1e-4 gamma0 Ms), then field 1 / field 2 for 1 ns with "
                        "c1 = 2.21e5, c2 = 4.42e3 (DP45, atol = rtol = 1e-6), one state, fp32",
            "sizes": rows, "seconds": round(time.perf_counter() - t_all, 1)}


def threshold_section(tmg, W, torch, attempts=300, fracs=(0.2, 0.4, 0.7)):
    """Thresholded operator on the SP4 film at [160, 40, 1] tiles (N = 6400),
    the paper's threshold study: for each removed fraction, the block-sparse
    operator's size, the sparse stage kernel's time and bandwidth (bytes as
    stored), the H_d error against the unthresholded float32 operator (random
    m), and single-state DP45 steps per second, beside the dense SYM6 path."""
    wl = W.thin_film(nx=160, ny=40)
    n = wl.n
    ctx = tmg.Context(0)
    geom = tmg.Geometry(ctx, wl.centers, wl.sizes)
    T = tmg.Tensor(ctx, geom, tmg.TM_PREC_FP32, tmg.TM_LAYOUT_SYM6)
    mr = torch.as_tensor(W.random_unit_vectors(9, n)[None].astype(np.float32), device="cuda")
    Ha = torch.as_tensor(wl.Ha.astype(np.float32), device="cuda")

    def measure(tensor, tune):
        p = tmg.Problem(ctx, geom, tensor, wl.Ms, wl.A, wl.alpha, wl.gamma0)
        if tune:
            tmg.tm_problem_tune(p.handle, 1, 10)
        ms, nb = tmg.tm_profile_field(p.handle, 1, 50)
        hd = p.demag(mr).cpu().numpy().astype(np.float64)
        m = torch.as_tensor(wl.m0.astype(np.float32), device="cuda")
        dt = torch.full((1,), 1e-14, dtype=torch.float64, device="cuda")
        p.run(m, Ha, tmg.TM_DP45, dt=dt, max_steps=1 << 40, max_attempts=20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p.run(m, Ha, tmg.TM_DP45, dt=dt, max_steps=1 << 40, max_attempts=attempts)
        torch.cuda.synchronize()
        sps = attempts / (time.perf_counter() - t0)
        p.close()
        return {"stage_kernel_us": round(ms * 1e3, 2), "bytes_per_launch": nb,
                "stage_kernel_gbs": round(nb / (ms * 1e-3) / 1e9, 1),
                "hbm_frac": round(nb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "steps_per_s": round(sps, 1)}, hd

    dense, hd_ref = measure(T, True)
    out = {"workload": "SP4 film [160,40,1] tiles of 3.125x3.125x3 nm (N=%d), one state, DP45" % n,
           "dense_sym6": dense, "thresholded": []}
    for f in fracs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Tt = T.threshold(f)
        torch.cuda.synchronize()
        build_ms = (time.perf_counter() - t0) * 1e3
        row, hd = measure(Tt, False)
        row.update({"frac": f, "threshold_ms": round(build_ms, 1), "blocks": Tt.nnzb,
                    "blocks_kept": round(Tt.nnzb / float(n * n), 4), "cut": Tt.cut,
                    "operator_bytes_vs_dense": round(Tt.nbytes / (24.0 * n * n), 4),
                    "hd_rel_err_vs_dense": float(np.linalg.norm(hd - hd_ref) / np.linalg.norm(hd_ref)),
                    "speedup_vs_dense": round(row["steps_per_s"] / dense["steps_per_s"], 3)})
        out["thresholded"].append(row)
        Tt.close()
    T.close()
    geom.close()
    ctx.close()
    return out


def sp3_section(tmg, W, torch, ns=(4, 6, 8, 10, 12, 16, 20)):
    """Standard problem 3: for each resolution n (n^3 cubic tiles, pair-
    symmetric operator), the edge L / l_ex at which the relaxed flower and
    vortex states have equal energy -- a scan in steps of 0.2 l_ex, then
    secant refinement of the sign change -- and the fit L(n) = a n^b + c whose
    c extrapolates to an infinitely fine mesh (the paper quotes 8.477 +- 0.007
    from its own runs, as context)."""
    from scipy.optimize import curve_fit

    out = {"workload": "cube with Ku = 0.1 Km (easy z), flower vs vortex (axis x) relaxed by pure damping "
                       "to max|dm/dt| < 1e-4 gamma0 Ms, batch of 2 states", "resolutions": []}
    t_all = time.perf_counter()
    for n in ns:
        t0 = time.perf_counter()
        w0 = W.sp3_cube(n, 8.5)
        ctx = tmg.Context(0)
        geom = tmg.Geometry(ctx, w0.centers, w0.sizes)
        T = tmg.Tensor(ctx, geom, tmg.TM_PREC_FP32, tmg.TM_LAYOUT_PSYM6)
        steps_total = 0

        def diff(lam):
            nonlocal steps_total
            w = W.sp3_cube(n, lam)
            ex = w.extra
            p = tmg.Problem(ctx, geom, T, w.Ms, w.A, w.alpha, w.gamma0, ll_form=1, Ku=ex["Ku"], easy=ex["easy"])
            m = torch.as_tensor(w.m0.astype(np.float32), device="cuda")
            _, _, steps, _ = p.run(m, None, tmg.TM_DP45, dt=1e-14, max_steps=20000, dmdt_stop=ex["dmdt_stop"])
            e = p.energy(m).sum(dim=1).cpu().numpy() / (ex["Km"] * ex["volume"])
            steps_total += int(steps.sum().item())
            p.close()
            return float(e[0] - e[1]), float(e[0]), float(e[1])

        lams = np.round(np.arange(7.4, 9.61, 0.2), 3)
        prev = None
        bracket = None
        for lam in lams:
            d = diff(lam)[0]
            if prev is not None and prev[1] < 0 <= d:
                bracket = (prev, (lam, d))
                break
            prev = (lam, d)
        row = {"n": n, "tiles": n ** 3}
        if bracket is None:
            row["crossing"] = None
        else:
            (a, fa), (b, fb) = bracket
            for _ in range(4):  # secant (regula falsi) on the energy difference
                c = b - fb * (b - a) / (fb - fa)
                fc = diff(c)[0]
                if fc < 0:
                    a, fa = c, fc
                else:
                    b, fb = c, fc
            row["crossing"] = round(b - fb * (b - a) / (fb - fa), 4)
        row["relax_steps"] = steps_total
        row["seconds"] = round(time.perf_counter() - t0, 2)
        out["resolutions"].append(row)
        T.close()
        geom.close()
        ctx.close()
    pts = [(r["n"], r["crossing"]) for r in out["resolutions"] if r["crossing"] is not None]
    for key, nmin in (("fit", 0), ("fit_n_ge_8", 8)):
        sel = [x for x in pts if x[0] >= nmin]
        if len(sel) < 4:
            continue
        nn = np.array([x[0] for x in sel], float)
        ll = np.array([x[1] for x in sel], float)
        try:
            (a, b, c), cov = curve_fit(lambda x, a, b, c: a * x ** b + c, nn, ll, p0=(-3.0, -1.0, 8.5), maxfev=20000)
            out[key] = {"a": round(float(a), 4), "b": round(float(b), 4), "L_inf": round(float(c), 4),
                        "L_inf_sd": round(float(np.sqrt(cov[2, 2])), 4)}
        except Exception as exc:  # a failed fit is reported, not fatal
            out[key] = {"error": str(exc)}
    out["paper_L_inf"] = "8.477 +- 0.007 (paper's fit over its own resolutions; context only)"
    out["seconds"] = round(time.perf_counter() - t_all, 1)
    return out


def peaks_section(torch, tmg):
    """Probe rates on this device for context (not ceilings): the library's
    own stream read (2 GiB) and register-only MFMA loops, a 4 GiB device copy
    (read + write bytes) and library GEMMs (torch.mm) in bf16 and fp32."""
    out = {}
    rd, mb, mf = tmg.tm_measure_peaks(0, 2 << 30)
    out["stream_read_gbs"] = round(rd, 1)
    out["mfma_bf16_32x32x16_tflops"] = round(mb, 1)
    out["mfma_fp32_16x16x4_tflops"] = round(mf, 1)
    src = torch.ones(1 << 30, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = 1e30
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    out["copy_gbs"] = round(2 * src.numel() * 4 / best / 1e9, 1)
    del src, dst
    for dt, name in ((torch.bfloat16, "bf16"), (torch.float32, "fp32")):
        a = torch.randn(8192, 8192, device="cuda").to(dt)
        b = torch.randn(8192, 8192, device="cuda").to(dt)
        c = torch.mm(a, b)
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            torch.mm(a, b, out=c)
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1) * 1e-3)
        out["library_gemm_%s_tflops" % name] = round(2 * 8192 ** 3 / best / 1e12, 1)
        del a, b, c
    torch.cuda.empty_cache()
    return out


def serving_section(tmg, W, torch, count=24, n_max=4000, max_steps=3000, slots=8, max_active=0, serial=True):
    """Poisson stream of relaxation requests (bounded sample of the serving
    workload: `count` requests, tile counts log-uniform in [500, n_max]):
    the continuous-batching server against serial FIFO plain-FP32 solves of
    the same requests (service times measured one by one, queueing from the
    same arrival times)."""
    Ms, A, alpha = 8.0e5, 1.3e-11, 0.5
    stop = 1e-4 * W.GAMMA0 * Ms
    reqs = W.serving_stream(count=count, n_max=n_max)
    kw = dict(Ms=Ms, A_exch=A, alpha=alpha, dmdt_stop=stop, max_steps=max_steps, dt0=1e-14)
    ctx = tmg.Context(0)
    srv = tmg.Server(ctx, max_slots=slots, max_groups=16, steps_per_round=64, max_active=max_active)
    t0 = time.perf_counter()
    tks = []
    for r in reqs:
        d = t0 + r.arrival - time.perf_counter()
        if d > 0:
            time.sleep(d)
        tks.append(srv.submit(r.centers, r.sizes, r.m0, r.Ha, **kw))
    res = [srv.poll(t)[0] for t in tks]
    span = time.perf_counter() - t0
    srv.close()
    lat = np.array([r.latency_ms for r in res])
    conv = sum(1 for r in res if r.status == 0)
    hits = sum(1 for r in res if r.cache_hit)
    out = {"workload": "Poisson stream 20 req/s, %d requests, N log-uniform 500-%d on 5x5x3 nm "
                       "grids, 30%% repeated geometries, relax to max|dm/dt| < 1e-4 gamma0 Ms "
                       "(cap %d steps)" % (count, n_max, max_steps),
           "server": {"throughput_req_s": round(count / span, 3),
                      "p50_ms": round(float(np.percentile(lat, 50)), 1),
                      "p99_ms": round(float(np.percentile(lat, 99)), 1),
                      "converged": conv, "cache_hits": hits, "slots": slots, "max_active": max_active}}
    if not serial:
        ctx.close()
        return out
    # serial FIFO baseline on the same device (operator cache kept, as a
    # plain solver would keep its operator between repeated geometries)
    svc = []
    cache = {}
    for r in reqs:
        ts = time.perf_counter()
        key = (r.centers.shape[0], r.centers.tobytes())
        if key not in cache:
            g = tmg.Geometry(ctx, r.centers, r.sizes)
            # the same operator layout the server picks: pair-symmetric for
            # identical tiles above 1200 tiles, with four planes for one layer
            same = bool(np.all(r.sizes == r.sizes[0])) and r.centers.shape[0] > 1200
            layer = bool(np.all(r.centers[:, 2] == r.centers[0, 2]))
            lay = (tmg.TM_LAYOUT_PSYM4 if layer else tmg.TM_LAYOUT_PSYM6) if same else tmg.TM_LAYOUT_SYM6
            T = tmg.Tensor(ctx, g, tmg.TM_PREC_FP32, lay)
            cache[key] = (g, T)
        g, T = cache[key]
        p = tmg.Problem(ctx, g, T, Ms, A, alpha)
        m = torch.as_tensor(r.m0[None].astype(np.float32), device="cuda")
        Ha = torch.as_tensor(np.asarray(r.Ha, np.float32)[None], device="cuda")
        p.run(m, Ha, tmg.TM_DP45, dt=1e-14, max_steps=max_steps, dmdt_stop=stop, check=False)
        torch.cuda.synchronize()
        p.close()
        svc.append(time.perf_counter() - ts)
    end, lat_s = 0.0, []
    for r, sv in zip(reqs, svc):
        start = max(r.arrival, end)
        end = start + sv
        lat_s.append((end - r.arrival) * 1e3)
    for g, T in cache.values():
        T.close()
        g.close()
    ctx.close()
    lat_s = np.array(lat_s)
    out["serial_fp32"] = {"throughput_req_s": round(count / end, 3),
                          "p50_ms": round(float(np.percentile(lat_s, 50)), 1),
                          "p99_ms": round(float(np.percentile(lat_s, 99)), 1)}
    return out


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
    if args.profile_only:
        # a plain copy of known size: the counters of this dispatch calibrate
        # FETCH_SIZE / WRITE_SIZE against 1 GiB read and 1 GiB written
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    wl = W.thin_film() if not args.profile_only or args.profile_film == "100x25" else W.thin_film(nx=160, ny=40)
    n = wl.n
    ctx = tmg.Context(0)
    geom = tmg.Geometry(ctx, wl.centers, wl.sizes)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    psym = args.layout in ("psym4", "psym6")
    T = tmg.Tensor(ctx, geom, tmg.TM_PREC_FP32, LAYOUT_CODE[args.layout])
    torch.cuda.synchronize()
    asm_ms = (time.perf_counter() - t0) * 1e3
    p = tmg.Problem(ctx, geom, T, wl.Ms, wl.A, wl.alpha, wl.gamma0)
    # project autotuner: fastest launch shape of the fused stage kernel for this N
    # (pair-symmetric layouts: cached or nontemporal operator loads in the tile pass)
    shape = tile_loads_choice(tmg, p, psym, args.tile_loads, 50)
    nt_loads = psym and shape == 1
    m = torch.as_tensor(wl.m0.astype(np.float32), device="cuda")
    Ha = torch.as_tensor(wl.Ha.astype(np.float32), device="cuda")
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt = torch.full((1,), 1e-14, dtype=torch.float64, device="cuda")
    big = 1 << 40

    if args.profile_only:
        # counter runs: the dominant kernel as it runs inside the steps (with
        # --profile-batch B: B states of the same film, each with its own
        # seeded in-plane applied field, integrated together)
        Bp = max(1, args.profile_batch)
        if Bp > 1:
            rng = np.random.default_rng(11)
            mb = np.repeat(wl.m0.astype(np.float32), Bp, axis=0)
            hb = np.repeat(wl.Ha.astype(np.float32), Bp, axis=0)
            hb[1:, :2] += rng.uniform(-2e4, 2e4, size=(Bp - 1, 2)).astype(np.float32)
            m = torch.as_tensor(mb, device="cuda")
            Ha = torch.as_tensor(hb, device="cuda")
            t = torch.zeros(Bp, dtype=torch.float64, device="cuda")
            dt = torch.full((Bp,), 1e-14, dtype=torch.float64, device="cuda")
        cfg = tmg.tm_run_cfg(big, args.profile_iters, 0.0, 1e-6, 1e-6, 0.0, 0.0, 1, 0, 64)
        op_ms, op_n = tmg.tm_profile_run(p.handle, n, tmg.TM_DP45, m, Ha, t, dt, cfg)
        print(json.dumps({"profile_only": True, "batch": Bp, "operator_pass_us": round(op_ms / op_n * 1e3, 3),
                          "launches": op_n}), flush=True)
        p.close()
        T.close()
        geom.close()
        ctx.close()
        return
    # warmup (graph capture happens here)
    p.run(m, Ha, tmg.TM_DP45, dt=dt, t=t, max_steps=big, max_attempts=max(1, args.warmup))
    steps_buf = torch.zeros(1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = tmg.tm_run(p.handle, n, tmg.TM_DP45, m, Ha, t, dt, steps_buf,
                    tmg.tm_run_cfg(big, args.steps, 0.0, 1e-6, 1e-6, 0.0, 0.0, 1, 1, 64))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    assert torch.isfinite(m).all().item(), "non-finite state after the timed run"
    accepted = int(steps_buf.cpu()[0])
    t_sim = float(t.cpu()[0])
    m_final = m.cpu().numpy()[0].copy()
    hd_final = p.demag(m).cpu().numpy()[0]

    # dominant kernel inside the step: the same number of attempts again from
    # the final state, every operator pass stamped with its own start and end
    # (kernel timestamps on the stream it runs on)
    op_ms, op_n = tmg.tm_profile_run(p.handle, n, tmg.TM_DP45, m, Ha, t, dt,
                                     tmg.tm_run_cfg(big, args.steps, 0.0, 1e-6, 1e-6, 0.0, 0.0, 1, 0, 64))
    avg_ms = op_ms / op_n
    eval_ms, stored_bytes = tmg.tm_profile_field(p.handle, 1, 20)
    if psym:
        planes = 4 if args.layout == "psym4" else 6
        alg_bytes = n * (n + 1) // 2 * planes * 4 + 24 * n
        alg_basis = "N(N+1)/2 blocks x %d planes x 4 B + 24 N (state in, slots out not counted)" % planes
        kname = "k_psym_tiles<true,true,%s,%d,false>" % ("true" if nt_loads else "false", planes)
        kdesc = (" (pair-symmetric tile pass of the demag product; the slot sum and epilogue run in "
                 "a second launch, included in field_evaluation_us)")
    else:
        alg_bytes = 24 * n * n + 24 * n
        alg_basis = "6 planes x N^2 x 4 B + 24 N"
        kname = "k_field<%d,%d,%d,%d,STAGE>" % tmg.tm_shape_info(shape)
        kdesc = " (fused demag matvec + H_eff + LL + stage update)"
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    traffic = counter_traffic(args.layout, kname)

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
                               "adaptive DP45, fp32 %s operator" % args.layout.upper(),
                   "n_tiles": n, "batch": 1, "integrator": "DP45", "operator": "fp32 " + args.layout,
                   "accepted_steps": accepted, "rejected_steps": int(st.rejected),
                   "stage_kernel_shape": -1 if psym else shape,
                   "tile_pass_loads": ("nontemporal" if nt_loads else "cached") if psym else None,
                   "simulated_ns": round(t_sim * 1e9, 4),
                   "assembly_ms": round(asm_ms, 2)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": kname + kdesc,
                     "avg_launch_us": round(avg_ms * 1e3, 3), "launches_timed": op_n,
                     "timing": "kernel start/end timestamps of every operator pass of %d further attempted "
                               "steps from the final state (tm_profile_run, direct launches)" % args.steps,
                     "bytes_per_launch": alg_bytes, "bytes_basis": "algorithmic: " + alg_basis,
                     "stored_bytes_per_launch": stored_bytes,
                     "cache_resident": stored_bytes < (256 << 20),
                     "field_evaluation_us": round(eval_ms * 1e3, 3)},
    }
    if stored_bytes < (256 << 20) and not args.no_cache_free:
        progress("cache-free roofline (N = 6400 film)")
        rec["roofline"]["cache_free"] = cache_free_section(tmg, W, torch, args.layout, tile_loads=args.tile_loads)
    p.close()
    T.close()
    geom.close()
    ctx.close()
    batched_data = None
    if not args.no_batched:
        progress("batched product (B = 128)")
        bat, batched_data = batched_section(tmg, W, torch)
        best = max(v["state_steps_per_s"] for k, v in bat.items() if isinstance(v, dict))
        bat["vs_single_fp32_solve"] = round(best / rec["value"], 2)
        rec["batched"] = bat
    if not args.no_large:
        progress("refined slab N = 20000")
        rec["large"] = large_section(tmg, W, torch, with_oracle=not args.no_cpu_baseline)
    if not args.no_cube:
        progress("cube RK4")
        rec["cube"] = cube_section(tmg, W, torch, with_oracle=not args.no_cpu_baseline)
    if not args.no_sweep:
        progress("SP4 sweep")
        rec["sp4_sweep"] = sp4_sweep_section(tmg, W, torch)
    if not args.no_sp4_dynamics:
        progress("SP4 dynamics")
        rec["sp4_dynamics"] = sp4_dynamics_section(tmg, W, torch)
    if not args.no_threshold:
        progress("thresholding")
        rec["threshold"] = threshold_section(tmg, W, torch)
    if not args.no_sp3:
        progress("standard problem 3")
        rec["sp3"] = sp3_section(tmg, W, torch)
    if not args.no_serving:
        progress("serving")
        rec["serving"] = serving_section(tmg, W, torch, count=args.serving_count, n_max=args.serving_nmax,
                                         max_active=args.serving_max_active)
    if not args.no_peaks:
        progress("probe rates")
        # context: what plain probes reach on this machine (not ceilings: the
        # slab's stage kernel streams at or above the read probe)
        rec["probe_rates"] = peaks_section(torch, tmg)
    if not args.no_cpu_baseline:
        progress("cpu baseline (oracle)")
        base, errs = cpu_baseline(wl, args.cpu_steps, m_final, hd_final, batched_data)
        rec["cpu_baseline"] = base
        rec["error_vs_oracle"] = dict(quantity="H_d of the timed run's final state against the FP64 oracle",
                                      tolerance=1e-5, **errs["headline"])
        if batched_data is not None:
            for name in batched_data["hd"]:
                e = errs["batched_" + name]
                rec["batched"][name]["hd_rel_err_2norm"] = e["rel_err_2norm"]
                rec["batched"][name]["hd_rel_err_max"] = e["rel_err_max"]
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
