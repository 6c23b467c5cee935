"""Standard problem 4 on the GPU against the FP64 oracle (paper Sec. 4.3):
the s-state preparation and the start of the reversal dynamics.

* s-state at [40, 10, 1]: the device protocol (staircase of [1, 1, 1] fields,
  pure-damping relaxation to the threshold, paper_2107_05364_amd.sp4) and the
  same protocol run on the oracle in the test end in the same state: mean
  magnetisation within 2e-3 per component (each side stops at its own first
  step below max|dm/dt| < 1e-4 gamma0 Ms, i.e. a residual torque field of
  80 A/m against restoring fields of ~1e4 A/m, so the two relaxed states may
  differ by ~1e-3 in m).
* s-state at [100, 25, 1]: the device protocol against the oracle's state
  stored in tests/golden/sp4_sstate_n5.json (written by make_sp4_sstate.py,
  oracle only), same bound.
* dynamics at [100, 25, 1]: from the stored oracle s-state (float32, the same
  array on both sides), field 1 and field 2 with the paper's LL parameters
  (c1 = 2.21e5, c2 = 4.42e3) for the first 10 ps, four-plane and six-plane
  operators: both sides land on t = 10 ps; max |dm| <= 5e-5 (the film
  trajectory bound of the other parity tests) and |d<m>| <= 1e-5.
"""
import base64
import json
import os
import sys

import numpy as np
import pytest

from gpu_helpers import close, tilemag
from paper_2107_05364_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "sp4_sstate_n5.json")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _golden():
    with open(GOLDEN) as fh:
        g = json.load(fh)
    m = np.frombuffer(base64.b64decode(g["m_float32_le_base64"]), dtype="<f4").reshape(g["n"], 3)
    return g, m.astype(np.float32)


def _oracle_relax(orc, wl):
    c1, c2 = wl.extra["relax_ll"]
    P = orc.Problem(wl.centers, wl.sizes, wl.Ms, wl.A, c2, gamma0=c1, ll_form=1)
    y = wl.m0[0].astype(np.float64).copy()
    for H in wl.extra["levels"]:
        k1 = P.rhs(y, H)
        dt, t = 1e-14, 0.0
        while True:
            ok, dt, t, _, dmx = P.dp45_attempt(y, k1, H, dt, t)
            if ok and dmx < wl.extra["relax_stop"]:
                break
    w = P.vol * P.Ms
    return (w[:, None] * y).sum(axis=0) / w.sum()


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


def _device_sstate(tmg, ctx, wl, layout):
    from paper_2107_05364_amd import sp4

    g = tmg.Geometry(ctx, wl.centers, wl.sizes)
    T = tmg.Tensor(ctx, g, tmg.TM_PREC_FP32, layout)
    m, levels = sp4.prepare_sstate(ctx, g, T, wl)
    close(g, T)
    return m, levels


def test_sstate_n2_matches_oracle(tmg, ctx, orc):
    wl = W.sp4_film(2)
    _say("sp4 s-state n=2 (N=%d)" % wl.n)
    m, levels = _device_sstate(tmg, ctx, wl, tmg.TM_LAYOUT_PSYM4)
    got = np.array(levels[-1]["mean_m"])
    want = _oracle_relax(orc, wl)
    _say("s-state n=2: device %s oracle %s" % (got, want))
    assert np.abs(got - want).max() <= 2e-3
    assert np.abs(np.linalg.norm(m.cpu().numpy()[0], axis=1) - 1).max() < 1e-6


def test_sstate_n5_matches_stored_oracle_state(tmg, ctx):
    g, _ = _golden()
    wl = W.sp4_film(5)
    _say("sp4 s-state n=5 (N=%d)" % wl.n)
    m, levels = _device_sstate(tmg, ctx, wl, tmg.TM_LAYOUT_PSYM4)
    got = np.array(levels[-1]["mean_m"])
    _say("s-state n=5: device %s stored oracle %s" % (got, g["mean_m_fp64"]))
    assert np.abs(got - np.array(g["mean_m_fp64"])).max() <= 2e-3


@pytest.mark.parametrize("field", [1, 2])
@pytest.mark.parametrize("layout", ["psym4", "sym6"])
def test_dynamics_first_10ps_match_oracle(tmg, ctx, orc, layout, field):
    import torch

    from paper_2107_05364_amd import sp4

    g, m0 = _golden()
    wl = W.sp4_film(5)
    t_end = 10e-12
    _say("sp4 dynamics n=5 field %d %s to %.0f ps" % (field, layout, t_end * 1e12))
    geom = tmg.Geometry(ctx, wl.centers, wl.sizes)
    lay = tmg.TM_LAYOUT_PSYM4 if layout == "psym4" else tmg.TM_LAYOUT_SYM6
    T = tmg.Tensor(ctx, geom, tmg.TM_PREC_FP32, lay)
    md = torch.as_tensor(m0[None], device="cuda")
    m, st, wall, mean = sp4.dynamics(ctx, geom, T, wl, md, field, t_end=t_end)
    got = m.cpu().numpy()[0]
    c1, c2 = wl.extra["dyn_ll"]
    P = orc.Problem(wl.centers, wl.sizes, wl.Ms, wl.A, c2, gamma0=c1, ll_form=1)
    H = wl.extra["fields"][field]
    y = m0.astype(np.float64).copy()
    k1 = P.rhs(y, H)
    dt, t = 1e-14, 0.0
    while t < t_end:
        _, dt, t, _, _ = P.dp45_attempt(y, k1, H, dt, t, 1e-6, 1e-6, True, t_end)
    w = P.vol * P.Ms
    want = (w[:, None] * y).sum(axis=0) / w.sum()
    dm = np.abs(got - y).max()
    _say("field %d %s: %d attempts, <m> device %s oracle %s, max|dm| %.2e"
         % (field, layout, st.attempts, mean, want, dm))
    assert dm <= 5e-5
    assert np.abs(mean - want).max() <= 1e-5
    close(geom, T)
