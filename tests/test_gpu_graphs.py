"""Captured-graph replays against direct launches, for every operator layout.

tm_run replays a captured graph of 16 attempted steps (and one of a single
attempt for the remainder).  Each round below runs 37 attempts (two replays of
the 16-attempt graph, five of the single one) on one state copy and the same
attempts launched directly on another, with unrelated eager device work in
between; after every round the two copies must be bitwise equal (the kernels
are deterministic and graph replays must not change their inputs)."""
import sys

import numpy as np
import pytest

from gpu_helpers import close, device_state, tilemag
from paper_2107_05364_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tmg():
    return tilemag()


@pytest.fixture(scope="module")
def ctx(tmg):
    c = tmg.Context(0)
    yield c
    try:
        c.close()
    except tmg.TilemagError:
        pass


CASES = ["sym6", "psym6", "psym4", "bsr6", "dense9_fp32", "dense9_bf16x3", "dense9_fp16x3"]


@pytest.mark.parametrize("case", CASES)
def test_graph_replays_match_direct_launches(tmg, ctx, case):
    import torch

    print("graph replays %s" % case, flush=True)
    sys.stdout.flush()
    wl = W.hysteresis_batch(B=4, nx=40, ny=10)
    g = tmg.Geometry(ctx, wl.centers, wl.sizes)
    extra = []
    if case == "psym6":
        T = tmg.Tensor(ctx, g, tmg.TM_PREC_FP32, tmg.TM_LAYOUT_PSYM6)
    elif case == "psym4":  # the film is one layer of identical tiles
        T = tmg.Tensor(ctx, g, tmg.TM_PREC_FP32, tmg.TM_LAYOUT_PSYM4)
    elif case == "bsr6":
        T0 = tmg.Tensor(ctx, g)
        T = T0.threshold(0.4)
        extra.append(T0)
    elif case == "dense9_fp32":
        T = tmg.Tensor(ctx, g, tmg.TM_PREC_FP32, tmg.TM_LAYOUT_DENSE9)
    elif case == "dense9_bf16x3":
        T = tmg.Tensor(ctx, g, tmg.TM_PREC_BF16X3, tmg.TM_LAYOUT_DENSE9)
    elif case == "dense9_fp16x3":
        T = tmg.Tensor(ctx, g, tmg.TM_PREC_FP16X3, tmg.TM_LAYOUT_DENSE9)
    else:
        T = tmg.Tensor(ctx, g)
    p = tmg.Problem(ctx, g, T, wl.Ms, wl.A, wl.alpha, wl.gamma0)
    Ha = torch.as_tensor(wl.Ha.astype(np.float32), device="cuda")
    a = device_state(wl.m0)
    b = device_state(wl.m0)
    ta = torch.zeros(4, dtype=torch.float64, device="cuda")
    tb = torch.zeros(4, dtype=torch.float64, device="cuda")
    da = torch.full((4,), 1e-14, dtype=torch.float64, device="cuda")
    db = torch.full((4,), 1e-14, dtype=torch.float64, device="cuda")
    junk = torch.randn(1 << 20, device="cuda")
    for rnd in range(3):
        p.run(a, Ha, tmg.TM_DP45, dt=da, t=ta, max_steps=1 << 40, max_attempts=37, use_graph=True)
        junk = torch.sin(junk) * 1.5 + junk.sum() * 1e-9  # eager work between replays
        h = p.demag(device_state(wl.m0[::-1].copy()))
        torch.cuda.synchronize()
        p.run(b, Ha, tmg.TM_DP45, dt=db, t=tb, max_steps=1 << 40, max_attempts=37, use_graph=False)
        torch.cuda.synchronize()
        assert torch.equal(a, b), (case, rnd)
        assert torch.equal(ta, tb) and torch.equal(da, db), (case, rnd)
        assert torch.isfinite(h).all()
    close(g, T, p, *extra)


@pytest.mark.parametrize("case", ["sym6", "psym4", "bsr6", "dense9_bf16x3"])
def test_rk4_pairs_match_direct_launches(tmg, ctx, case):
    """RK4 runs replay graphs whose step pairs advance the control in their
    last stage (through the second set of control values) and whose odd last
    step uses the control pass: a run of 37 steps (graphs of 32, 4 and 1)
    then 6 more with t_end cutting the last step short, replayed three times,
    equals the same run from direct launches bit for bit (states, times,
    steps and step sizes)."""
    import torch

    print("rk4 pairs %s" % case, flush=True)
    wl = W.hysteresis_batch(B=3, nx=40, ny=10)
    g = tmg.Geometry(ctx, wl.centers, wl.sizes)
    extra = []
    if case == "psym4":
        T = tmg.Tensor(ctx, g, tmg.TM_PREC_FP32, tmg.TM_LAYOUT_PSYM4)
    elif case == "bsr6":
        T0 = tmg.Tensor(ctx, g)
        T = T0.threshold(0.4)
        extra.append(T0)
    elif case == "dense9_bf16x3":
        T = tmg.Tensor(ctx, g, tmg.TM_PREC_BF16X3, tmg.TM_LAYOUT_DENSE9)
    else:
        T = tmg.Tensor(ctx, g)
    p = tmg.Problem(ctx, g, T, wl.Ms, wl.A, wl.alpha, wl.gamma0)
    Ha = torch.as_tensor(wl.Ha.astype(np.float32), device="cuda")
    runs = {}
    for graph in (True, False):
        m = device_state(wl.m0)
        t = torch.zeros(3, dtype=torch.float64, device="cuda")
        dt = torch.full((3,), 2e-14, dtype=torch.float64, device="cuda")
        for rnd in range(3):
            s1 = p.run(m, Ha, tmg.TM_RK4, dt=dt, t=t, max_steps=37, use_graph=graph)[2]
            t_end = float(t.cpu().max()) + 5.5 * 2e-14
            s2 = p.run(m, Ha, tmg.TM_RK4, dt=dt, t=t, max_steps=6, t_end=t_end, use_graph=graph)[2]
        torch.cuda.synchronize()
        runs[graph] = (m.clone(), t.clone(), dt.clone(), s1.clone(), s2.clone())
    a, b = runs[True], runs[False]
    for x, y in zip(a, b):
        assert torch.equal(x, y), case
    assert torch.isfinite(a[0]).all()
    # one step per call (every step through the control pass) equals 37
    # steps in one call (pairs advancing the control in their last stage)
    m1 = device_state(wl.m0)
    m2 = device_state(wl.m0)
    t1 = torch.zeros(3, dtype=torch.float64, device="cuda")
    t2 = torch.zeros(3, dtype=torch.float64, device="cuda")
    dt1 = torch.full((3,), 2e-14, dtype=torch.float64, device="cuda")
    dt2 = torch.full((3,), 2e-14, dtype=torch.float64, device="cuda")
    p.run(m1, Ha, tmg.TM_RK4, dt=dt1, t=t1, max_steps=37)
    for _ in range(37):
        p.run(m2, Ha, tmg.TM_RK4, dt=dt2, t=t2, max_steps=1)
    torch.cuda.synchronize()
    assert torch.equal(m1, m2) and torch.equal(t1, t2), case
    close(g, T, p, *extra)
