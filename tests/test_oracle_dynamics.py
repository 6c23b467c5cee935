"""Pins of the oracle's time integration (paper Sec. 2.1 Landau-Lifshitz
equation, Sec. 3.1 explicit Runge-Kutta (4,5) integration).

A single cube tile in an applied field H z-hat has no demag torque (its self
field -Ms m/3 is parallel to m) and no exchange, so LL has the closed form
    m_z(t) = tanh(c2 H t + atanh m_z(0)),   phi(t) = phi(0) + c1 H t.
"""
import math

import numpy as np
import pytest

from paper_2107_05364_amd import workloads as W


def _macrospin(orc, alpha=0.1):
    c, s = np.zeros((1, 3)), np.full((1, 3), 5e-9)
    return orc.Problem(c, s, 8e5, 1.3e-11, alpha)


def _exact(P, m0, H, t):
    mz = math.tanh(P.c2 * H * t + math.atanh(m0[2]))
    phi = math.atan2(m0[1], m0[0]) + P.c1 * H * t
    r = math.sqrt(1 - mz * mz)
    return np.array([r * math.cos(phi), r * math.sin(phi), mz])


def test_macrospin_rk4_fourth_order(orc):
    P = _macrospin(orc)
    H = 2e5
    m0 = np.array([math.sin(2.5) * math.cos(0.3), math.sin(2.5) * math.sin(0.3), math.cos(2.5)])
    T = 40e-12
    errs = []
    for steps in (50, 100, 200):
        y = P.rk4(m0[None], [0, 0, H], T / steps, steps, renorm=False)
        errs.append(np.abs(y[0] - _exact(P, m0, H, T)).max())
    assert errs[-1] < 1e-7
    assert 13 < errs[0] / errs[1] < 19 and 13 < errs[1] / errs[2] < 19


def test_rk4_renormalisation(orc):
    P = _macrospin(orc)
    m0 = np.array([[0.6, 0.0, -0.8]])
    y = P.rk4(m0, [0, 0, 3e5], 2e-13, 100, renorm=False)
    drift = abs(np.linalg.norm(y) - 1)
    assert 1e-12 < drift < 1e-4
    y = P.rk4(m0, [0, 0, 3e5], 2e-13, 100, renorm=True)
    assert abs(np.linalg.norm(y) - 1) < 4e-16


def test_dp45_fifth_order_at_fixed_step(orc):
    """The propagated (fifth-order) solution converges like dt^5 and the
    embedded error estimate like dt^5 per step."""
    P = _macrospin(orc, alpha=0.2)
    H = 2e5
    m0 = np.array([math.sin(2.0), 0.0, math.cos(2.0)])
    T = 60e-12
    errs, ests = [], []
    for steps in (20, 40, 80):
        y = m0[None].copy()
        k1 = P.rhs(y, [0, 0, H])
        t, est = 0.0, 0.0
        dt = T / steps
        for _ in range(steps):
            ok, _, t, err, _ = P.dp45_attempt(y, k1, [0, 0, H], dt, t, atol=1e3, rtol=0.0,
                                              renorm=False)
            assert ok
            est = max(est, err * 1e3)
        errs.append(np.abs(y[0] - _exact(P, m0, H, T)).max())
        ests.append(est)
    assert 25 < errs[0] / errs[1] < 40 and 25 < errs[1] / errs[2] < 40
    assert 25 < ests[0] / ests[1] < 40 and 25 < ests[1] / ests[2] < 40


def test_dp45_adaptive_meets_tolerance(orc):
    P = _macrospin(orc, alpha=0.05)
    H = 1.5e5
    m0 = np.array([math.sin(2.8), 0.0, math.cos(2.8)])
    y, t, dt, att = P.dp45(m0[None], [0, 0, H], 1e-14, 200, atol=1e-8, rtol=1e-8)
    assert att >= 200
    assert np.abs(y[0] - _exact(P, m0, H, t)).max() < 1e-5
    assert abs(np.linalg.norm(y[0]) - 1) < 4e-16


def test_dp45_rejects_and_shrinks(orc):
    P = _macrospin(orc, alpha=0.05)
    m0 = np.array([[math.sin(1.0), 0.0, math.cos(1.0)]])
    y = m0.copy()
    k1 = P.rhs(y, [0, 0, 2e5])
    ok, dtn, t, err, _ = P.dp45_attempt(y, k1, [0, 0, 2e5], 5e-11, 0.0, 1e-8, 1e-8)
    assert not ok and err > 1 and t == 0.0 and np.array_equal(y, m0)
    assert 0.2 * 5e-11 - 1e-30 <= dtn < 0.9 * 5e-11
    ok, dtn2, t, err, _ = P.dp45_attempt(y, k1, [0, 0, 2e5], 1e-16, 0.0, 1e-8, 1e-8)
    assert ok and dtn2 == pytest.approx(5e-16) and t == 1e-16


def test_config1_energy_decreases(orc):
    """alpha > 0, static field, uniform mesh: the free energy never rises
    (paper Sec. 2.2) along 200 RK4 steps of dt = 1e-13 s."""
    wl = W.cube_grid()
    P = orc.Problem(wl.centers, wl.sizes, wl.Ms, wl.A, wl.alpha)
    y = wl.m0[0].copy()
    E = [P.energy(y).sum()]
    for _ in range(20):
        y = P.rk4(y, wl.Ha[0], 1e-13, 10)
        E.append(P.energy(y).sum())
    E = np.array(E)
    assert np.all(np.diff(E) <= 1e-12 * E[0])
    assert E[-1] < 0.5 * E[0]
    assert np.abs(np.linalg.norm(y, axis=1) - 1).max() < 1e-15
