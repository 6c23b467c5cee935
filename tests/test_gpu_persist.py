"""The persistent RK4 path (one cooperative launch for a whole run, operator
rows resident in LDS, a grid barrier per stage) against the FP64 oracle and
against the launch-per-stage path.

* the 8 x 8 x 8 cube grid (N = 512, eight target tiles per workgroup), 200
  RK4 steps of 1e-13 s: max |dm| <= 1e-4 against the oracle (the bound of the
  launch-per-stage RK4 test) and <= 1e-5 against the launch-per-stage path
  (both float32, different summation orders);
* a refined slab with per-tile Ms, anisotropy and an applied field (N = 701,
  768 padded tiles, four target tiles per workgroup), stopped by t_end in
  the middle of a step: the last step is shortened to land on t_end exactly,
  as in the launch-per-stage path; max |dm| <= 1e-4 against the oracle;
* the cases it does not take are refused before anything runs.
"""
import sys

import numpy as np
import pytest

from gpu_helpers import build, close, device_state, tilemag
from paper_2107_05364_amd import workloads as W

pytestmark = pytest.mark.gpu


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


def test_persistent_rk4_cube_200_steps(tmg, ctx, orc):
    wl = W.cube_grid()
    _say("persistent rk4 cube 200 steps")
    g, T, p = build(tmg, ctx, wl.centers, wl.sizes, alpha=wl.alpha)
    m0 = wl.m0.astype(np.float32)
    md = device_state(m0)
    t, dt, steps, st = p.run(md, None, tmg.TM_RK4, dt=1e-13, max_steps=200, persistent=True)
    got = md.cpu().numpy()[0]
    assert int(steps.cpu()[0]) == 200 and abs(float(t.cpu()[0]) - 200e-13) < 1e-20
    ref = device_state(m0)
    p.run(ref, None, tmg.TM_RK4, dt=1e-13, max_steps=200)
    P = orc.Problem(wl.centers, wl.sizes, wl.Ms, wl.A, wl.alpha)
    want = P.rk4(m0[0].astype(np.float64), [0, 0, 0], 1e-13, 200)
    _say("persistent vs oracle %.2e, vs launch-per-stage %.2e"
         % (np.abs(got - want).max(), np.abs(got - ref.cpu().numpy()[0]).max()))
    assert np.abs(got - want).max() <= 1e-4
    assert np.abs(got - ref.cpu().numpy()[0]).max() <= 1e-5
    assert np.abs(np.linalg.norm(got, axis=1) - 1).max() < 1e-6
    close(g, T, p)


def test_persistent_rk4_refined_t_end(tmg, ctx, orc):
    import torch

    slab = W.refined_slab(n_target=701, lx=200e-9, ly=60e-9, lz=20e-9)
    c, s = slab.centers, slab.sizes
    n = c.shape[0]
    Ms = np.linspace(6.0e5, 9.0e5, n)
    easy = W.random_unit_vectors(11, n)
    _say("persistent rk4 refined n=%d" % n)
    g, T, p = build(tmg, ctx, c, s, Ms=Ms, alpha=0.3, Ku=3.0e4, easy=easy)
    m0 = W.random_unit_vectors(31, n)[None].astype(np.float32)
    Ha = np.array([[2e4, -1e4, 5e3]], np.float32)
    dt0, t_end = 2e-14, 2.5e-13  # 12 full steps and a half step
    md = device_state(m0)
    t, dt, steps, st = p.run(md, torch.as_tensor(Ha, device="cuda"), tmg.TM_RK4, dt=dt0, max_steps=1000,
                             t_end=t_end, persistent=True)
    assert int(steps.cpu()[0]) == 13
    assert abs(float(t.cpu()[0]) - t_end) < 1e-24
    P = orc.Problem(c, s, Ms, 1.3e-11, 0.3, Ku=3.0e4, easy=easy)
    y = P.rk4(m0[0].astype(np.float64), Ha[0].astype(np.float64), dt0, 12)
    y = P.rk4(y, Ha[0].astype(np.float64), t_end - 12 * dt0, 1)
    got = md.cpu().numpy()[0]
    _say("persistent refined vs oracle %.2e" % np.abs(got - y).max())
    assert np.abs(got - y).max() <= 1e-4
    close(g, T, p)


def test_persistent_refuses_other_cases(tmg, ctx):
    import torch

    wl = W.cube_grid()
    g, T, p = build(tmg, ctx, wl.centers, wl.sizes, alpha=wl.alpha)
    m = device_state(np.concatenate([wl.m0, wl.m0]).astype(np.float32))
    st = p.run(m, None, tmg.TM_RK4, dt=1e-13, max_steps=5, persistent=True, check=False)[3]
    assert st.status == tmg.TM_EINVAL  # two states
    st = p.run(m[:1].contiguous(), None, tmg.TM_DP45, dt=1e-13, max_steps=5, persistent=True, check=False)[3]
    assert st.status == tmg.TM_EINVAL  # adaptive scheme
    close(g, T, p)
    c, s = W.grid(40, 30, 1, 5e-9, 5e-9, 3e-9)  # 1200 tiles
    g, T, p = build(tmg, ctx, c, s)
    m = device_state(W.random_unit_vectors(3, 1200)[None])
    st = p.run(m, None, tmg.TM_RK4, dt=1e-13, max_steps=5, persistent=True, check=False)[3]
    assert st.status == tmg.TM_EINVAL  # too many tiles for the LDS-resident rows
    assert torch.isfinite(m).all()
    close(g, T, p)
