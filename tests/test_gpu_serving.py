"""GPU tests of the serving loop: continuous batching of relaxation requests
of different tile counts, the geometry-keyed tensor cache, admission by
device bytes, and the same result for a request alone and in a mix."""
import math
import sys

import numpy as np
import pytest

from gpu_helpers import build, close, device_state, tilemag
from paper_2107_05364_amd import workloads as W

pytestmark = pytest.mark.gpu

GAMMA0 = 2.21e5
MS = 8.0e5
STOP = 1e-4 * GAMMA0 * MS  # equilibrium: max_a |dm/dt|_a < 1e-4 gamma0 Ms


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


def _req(k, nx, ny, nz=1):
    c, s = W.grid(nx, ny, nz, 5e-9, 5e-9, 3e-9)
    m0 = W.random_unit_vectors(300 + k, c.shape[0])
    ang = 2 * math.pi * W.uniform(400 + k, 1)[0]
    Ha = (30e-3 / (4e-7 * math.pi)) * np.array([math.cos(ang), math.sin(ang), 0.0])
    return c, s, m0, Ha


def _submit(srv, r, max_steps=20000):
    c, s, m0, Ha = r
    return srv.submit(c, s, m0, Ha, Ms=MS, A_exch=1.3e-11, alpha=0.5, dmdt_stop=STOP,
                      max_steps=max_steps)


def test_requests_relax_to_equilibrium(tmg, ctx):
    srv = tmg.Server(ctx, max_slots=4, max_groups=4, steps_per_round=64)
    reqs = [_req(0, 12, 6), _req(1, 20, 5), _req(2, 12, 6), _req(3, 9, 9, 2)]
    tks = [_submit(srv, r) for r in reqs]
    res = [srv.poll(t) for t in tks]
    srv.close()
    for (c, s, m0, Ha), (r, m) in zip(reqs, res):
        assert r.status == 0 and r.steps > 0, (r.status, tmg.last_error())
        # verify the equilibrium criterion independently on the returned state
        g, T, p = build(tmg, ctx, c, s, alpha=0.5)
        import torch

        f = p.dmdt(device_state(m[None]), torch.tensor([Ha], dtype=torch.float32, device="cuda"))
        mx = f.norm(dim=2).max().item()
        close(g, T, p)
        assert mx < 1.05 * STOP, (mx, STOP)
        assert np.abs(np.linalg.norm(m, axis=1) - 1).max() < 1e-5
    # the third request repeats the first geometry: a cache hit
    assert res[2][0].cache_hit == 1
    _say("latencies ms: %s" % [round(r.latency_ms, 1) for r, _ in res])


def test_alone_equals_in_mix(tmg, ctx):
    target = _req(10, 16, 8)
    srv = tmg.Server(ctx, max_slots=4, max_groups=4, steps_per_round=32)
    r_alone, m_alone = srv.poll(_submit(srv, target))
    srv.close()
    srv = tmg.Server(ctx, max_slots=4, max_groups=4, steps_per_round=32)
    others = [_req(11, 16, 8), _req(12, 10, 10), _req(13, 16, 8)]
    others[0] = (target[0], target[1], others[0][2], others[0][3])  # same geometry, other state
    tks = [_submit(srv, others[0]), _submit(srv, others[1])]
    tk = _submit(srv, target)
    tks.append(_submit(srv, others[2]))
    r_mix, m_mix = srv.poll(tk)
    for t in tks:
        srv.poll(t)
    srv.close()
    assert r_alone.status == 0 and r_mix.status == 0
    assert r_alone.steps == r_mix.steps
    assert np.array_equal(m_alone, m_mix)


def test_admission_under_small_budget(tmg, ctx):
    """With room for about one operator at a time, requests queue and still
    all complete; a request larger than the whole budget is refused."""
    small = [_req(20 + k, 20, 10) for k in range(3)] + [_req(30, 24, 8)]
    tbytes = 6 * 200 * 200 * 4
    srv = tmg.Server(ctx, memory_budget=int(2.5 * tbytes + 4e6), max_slots=2, max_groups=8,
                     steps_per_round=64)
    big = _req(40, 60, 40)
    tks = [_submit(srv, r) for r in small]
    tb = _submit(srv, big)
    res = [srv.poll(t)[0] for t in tks]
    rb = srv.poll(tb)[0]
    srv.close()
    assert all(r.status == 0 for r in res), [r.status for r in res]
    assert rb.status == tmg.TM_ENOMEM


def test_pair_symmetric_groups_relax(tmg, ctx):
    """Above 1200 identical tiles the server streams the pair-symmetric
    operator: four planes for a single layer (1280 tiles), six for four
    layers (1600 tiles).  Both requests reach the equilibrium criterion,
    checked independently with the six-plane operator."""
    import torch

    reqs = [_req(50, 40, 32), _req(51, 20, 20, 4)]
    srv = tmg.Server(ctx, max_slots=2, max_groups=4, steps_per_round=64)
    tks = [_submit(srv, r, max_steps=40000) for r in reqs]
    res = [srv.poll(t) for t in tks]
    srv.close()
    for (c, s, m0, Ha), (r, m) in zip(reqs, res):
        _say("pair-symmetric group n=%d: status %d, %d steps, %.1f ms" % (c.shape[0], r.status, r.steps, r.latency_ms))
        assert r.status == 0 and r.steps > 0, (r.status, tmg.last_error())
        g, T, p = build(tmg, ctx, c, s, alpha=0.5)
        f = p.dmdt(device_state(m[None]), torch.tensor([Ha], dtype=torch.float32, device="cuda"))
        mx = f.norm(dim=2).max().item()
        close(g, T, p)
        assert mx < 1.05 * STOP, (mx, STOP)
        assert np.abs(np.linalg.norm(m, axis=1) - 1).max() < 1e-5
