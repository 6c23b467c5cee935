"""GPU parity at the full size of the large non-uniform mesh: the 20000-tile
refined slab (operator 60000 x 60000: 9.6 GB as six float32 planes, 14.5 GB
as bf16 hi + lo), in the launch configurations the benchmark times.  The
oracle computes H_d at sampled target tiles with the tensor evaluated on the
fly (no dense operator on the host).

Tolerances: float32 product 1e-5 (relative 2-norm and max-norm over the
sampled tiles), BF16X3 1e-3, as for the smaller meshes; over a few adaptive
steps |m| = 1 to 1e-6 and every value finite (the operator of a non-uniform
mesh is not symmetric, so the energy need not decrease)."""
import sys

import numpy as np
import pytest

from gpu_helpers import close, device_state, rel_errors, tilemag
from paper_2107_05364_amd import workloads as W

pytestmark = pytest.mark.gpu

ROWS = np.array([0, 1, 2, 517, 4999, 7777, 10000, 12345, 15000, 19000, 19998, 19999])


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


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


@pytest.fixture(scope="module")
def slab():
    return W.refined_slab(n_target=20000, B=32)


def test_large_slab_stage_kernel_rows(tmg, ctx, orc, slab):
    wl = slab
    _say("large slab N=%d sym6, tuned shape" % wl.n)
    g = tmg.Geometry(ctx, wl.centers, wl.sizes)
    T = tmg.Tensor(ctx, g, tmg.TM_PREC_FP32, tmg.TM_LAYOUT_SYM6)
    p = tmg.Problem(ctx, g, T, wl.Ms, wl.A, wl.alpha, wl.gamma0)
    shape, _ = tmg.tm_problem_tune(p.handle, 1, 2)  # as the benchmark does
    _say("large slab shape %d" % shape)
    m = wl.m0[:1].astype(np.float32)
    Hd = p.demag(device_state(m)).cpu().numpy()[0]
    want = orc.demag_rows(wl.centers, wl.sizes, wl.Ms, m[0].astype(np.float64), ROWS)
    e2, emax = rel_errors(Hd[ROWS], want)
    assert e2 <= 1e-5 and emax <= 1e-5, (e2, emax)
    # a few adaptive steps: norm and finiteness
    md = device_state(m)
    t, dt, steps, st = p.run(md, None, tmg.TM_DP45, dt=1e-14, max_steps=1 << 40, max_attempts=3)
    got = md.cpu().numpy()[0]
    assert np.isfinite(got).all() and int(steps.cpu()[0]) >= 1
    assert np.abs(np.linalg.norm(got, axis=1) - 1).max() < 1e-6
    close(g, T, p)


def test_large_slab_batched_bf16x3_rows(tmg, ctx, orc, slab):
    wl = slab
    _say("large slab N=%d dense9 bf16x3, B=32" % wl.n)
    g = tmg.Geometry(ctx, wl.centers, wl.sizes)
    T = tmg.Tensor(ctx, g, tmg.TM_PREC_BF16X3, tmg.TM_LAYOUT_DENSE9)
    p = tmg.Problem(ctx, g, T, wl.Ms, wl.A, wl.alpha, wl.gamma0)
    splits, _ = tmg.tm_problem_tune(p.handle, 32, 5)  # as the benchmark does
    _say("large slab bf16x3: %d K splits" % splits)
    m = wl.m0.astype(np.float32)
    Hd = p.demag(device_state(m)).cpu().numpy()
    for k in (0, 17, 31):
        want = orc.demag_rows(wl.centers, wl.sizes, wl.Ms, m[k].astype(np.float64), ROWS)
        e2, emax = rel_errors(Hd[k][ROWS], want)
        _say("state %d: %.3g %.3g" % (k, e2, emax))
        assert e2 <= 1e-3 and emax <= 1e-3, (k, e2, emax)
    close(g, T, p)
