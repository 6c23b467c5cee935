"""Pins of the oracle's effective field, energy and Landau-Lifshitz right-hand
side (paper Sec. 2.1-2.3 and the affine operator of Sec. 3.1)."""
import json
import math
import os

import numpy as np
import pytest

from paper_2107_05364_amd import workloads as W

MU0 = 4e-7 * math.pi


def _uniform_problem(orc, nx=6, ny=4, nz=3, d=(5e-9, 4e-9, 3e-9), alpha=0.5, Ku=0.0, easy=None):
    c, s = W.grid(nx, ny, nz, *d)
    return orc.Problem(c, s, 8.0e5, 1.3e-11, alpha, Ku=Ku, easy=easy)


def test_face_count_uniform_grid(orc):
    nx, ny, nz = 5, 4, 3
    c, s = W.grid(nx, ny, nz, 1.0, 2.0, 3.0)
    fa, fb, area, dist = orc.faces(c, s)
    want = 2 * ((nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1))
    assert fa.shape[0] == want
    # ordered pairs come in both directions with equal data
    key = {(a, b): (ar, di) for a, b, ar, di in zip(fa, fb, area, dist)}
    for (a, b), v in key.items():
        assert key[(b, a)] == v


def test_face_areas_close_every_tile_surface(orc):
    """On a non-conforming refined slab every tile face is either shared with
    neighbours or on the slab boundary, so shared + boundary area = surface."""
    wl = W.refined_slab(n_target=600, lx=200e-9, ly=50e-9, lz=20e-9)
    c, s = wl.centers, wl.sizes
    fa, fb, area, dist = orc.faces(c, s)
    n = c.shape[0]
    shared = np.zeros(n)
    np.add.at(shared, fa, area)
    lo, hi = (c - 0.5 * s).min(0), (c + 0.5 * s).max(0)
    bnd = np.zeros(n)
    for d in range(3):
        e1, e2 = (d + 1) % 3, (d + 2) % 3
        face = s[:, e1] * s[:, e2]
        bnd += face * (np.isclose(c[:, d] - 0.5 * s[:, d], lo[d], rtol=0, atol=1e-15))
        bnd += face * (np.isclose(c[:, d] + 0.5 * s[:, d], hi[d], rtol=0, atol=1e-15))
    surf = 2 * (s[:, 0] * s[:, 1] + s[:, 1] * s[:, 2] + s[:, 0] * s[:, 2])
    np.testing.assert_allclose(shared + bnd, surf, rtol=1e-12)
    # distance along the normal is the mean of the two edges
    assert len(np.unique(np.round(s / 1.25e-9))) > 1


def test_exchange_uniform_m_is_zero(orc):
    P = _uniform_problem(orc)
    m = np.tile([0.6, 0.0, 0.8], (P.n, 1))
    H = P.heff(m) - P.demag(m)
    assert np.abs(H).max() < 1e-9


def test_exchange_interior_eigenfunction(orc):
    """m = (cos kx, sin kx, 0) on a uniform grid: at tiles with both x
    neighbours the 3-point stencil gives (2A/mu0 Ms) (2cos(kh) - 2)/h^2 m."""
    nx, h = 12, 5e-9
    P = _uniform_problem(orc, nx=nx, ny=2, nz=1, d=(h, 4e-9, 3e-9))
    x = P.centers[:, 0]
    k = 2 * math.pi / (7.3 * h)
    m = np.stack([np.cos(k * x), np.sin(k * x), 0 * x], axis=1)
    Hex = P.heff(m) - P.demag(m)
    coef = 2 * 1.3e-11 / (MU0 * 8.0e5) * (2 * math.cos(k * h) - 2) / h**2
    ix = np.arange(P.n) % nx
    inner = (ix > 0) & (ix < nx - 1)
    np.testing.assert_allclose(Hex[inner], coef * m[inner], rtol=1e-10, atol=1e-6)
    # boundary tiles: one neighbour only (zero normal derivative)
    edge = ix == 0
    nb = np.where(ix == 1)[0]
    want = 2 * 1.3e-11 / (MU0 * 8.0e5) * (m[nb] - m[edge]) / h**2
    np.testing.assert_allclose(Hex[edge], want, rtol=1e-10, atol=1e-6)


def test_exchange_flux_conservation_nonuniform(orc):
    wl = W.refined_slab(n_target=500, lx=200e-9, ly=50e-9, lz=20e-9)
    P = orc.Problem(wl.centers, wl.sizes, 8.0e5, 1.3e-11, 0.1)
    m = W.random_unit_vectors(3, P.n)
    Hex = P.heff(m) - P.demag(m)
    tot = (P.vol[:, None] * Hex).sum(0)
    scale = (P.vol[:, None] * np.abs(Hex)).sum(0)
    assert np.all(np.abs(tot) < 1e-12 * scale)


def test_anisotropy_field_and_energy(orc):
    n = 1
    c, s = np.zeros((1, 3)), np.full((1, 3), 5e-9)
    e = np.array([[0.0, 0.6, 0.8]])
    K = 5e4
    P = orc.Problem(c, s, 8e5, 1.3e-11, 0.1, Ku=K, easy=e)
    m = np.array([[0.0, 0.6, 0.8]])
    H = P.heff(m)
    Hd = -8e5 * m / 3.0
    np.testing.assert_allclose(H - Hd, 2 * K / (MU0 * 8e5) * e, rtol=1e-13)
    E = P.energy(m)
    assert abs(E[2] + 125e-27 * K) < 1e-13 * 125e-27 * K
    assert n == 1


def test_energy_gradient_is_minus_field(orc):
    """H_eff = -(1/(mu0 Ms V)) dE/dm (paper Sec. 2.2): the four field terms
    against central differences of the four energy terms."""
    c, s = W.grid(4, 3, 2, 5e-9, 4e-9, 3e-9)
    n = c.shape[0]
    easy = W.random_unit_vectors(11, n)
    P = orc.Problem(c, s, 8.0e5, 1.3e-11, 0.5, Ku=3e4, easy=easy)
    m = W.random_unit_vectors(12, n)
    Ha = np.array([1.1e4, -2.3e4, 0.7e4])
    H = P.heff(m, Ha)
    rng = np.random.default_rng(0)
    for a in rng.choice(n, 6, replace=False):
        for i in range(3):
            eps = 1e-5
            mp_, mm_ = m.copy(), m.copy()
            mp_[a, i] += eps
            mm_[a, i] -= eps
            dE = (P.energy(mp_, Ha).sum() - P.energy(mm_, Ha).sum()) / (2 * eps)
            want = -dE / (MU0 * 8.0e5 * P.vol[a])
            assert abs(H[a, i] - want) < 1e-7 * np.abs(H).max(), (a, i, H[a, i], want)


def test_affine_operator(orc):
    """H_eff(m) - b is linear in m (paper Sec. 3.1), b being the applied field."""
    c, s = W.grid(3, 3, 2, 5e-9, 5e-9, 3e-9)
    n = c.shape[0]
    P = orc.Problem(c, s, 8.0e5, 1.3e-11, 0.5, Ku=2e4, easy=W.random_unit_vectors(1, n))
    Ha = np.array([3e4, 0.0, -1e4])
    m1, m2 = W.random_unit_vectors(2, n), W.random_unit_vectors(3, n)
    lam = 0.37
    lhs = P.heff(lam * m1 + m2, Ha) - Ha
    rhs = lam * (P.heff(m1, Ha) - Ha) + (P.heff(m2, Ha) - Ha)
    assert np.abs(lhs - rhs).max() < 1e-9 * np.abs(rhs).max()


def test_ll_rhs_properties(orc):
    """m . dm/dt = 0 (norm preservation, Sec. 2.1), dm/dt = 0 where m || H
    (Brown's first equation), and the damping term lowers the energy:
    dE/dt = -mu0 sum V Ms c2 |m x H|^2."""
    c, s = W.grid(4, 4, 2, 5e-9, 5e-9, 3e-9)
    n = c.shape[0]
    P = orc.Problem(c, s, 8.0e5, 1.3e-11, 0.3)
    m = W.random_unit_vectors(5, n)
    Ha = np.array([2e4, 1e4, 0.0])
    f = P.rhs(m, Ha)
    assert np.abs((m * f).sum(1)).max() < 1e-12 * np.abs(f).max()
    H = P.heff(m, Ha)
    mxh = np.cross(m, H)
    dEdt = -MU0 * (P.vol * P.Ms * P.c2 * (mxh**2).sum(1)).sum()
    eps = 1e-16
    dE = (P.energy(m + eps * f, Ha).sum() - P.energy(m - eps * f, Ha).sum()) / (2 * eps)
    assert abs(dE - dEdt) < 1e-6 * abs(dEdt)
    # a single cube tile in a field along its magnetisation: no torque
    P1 = orc.Problem(np.zeros((1, 3)), np.full((1, 3), 5e-9), 8e5, 1.3e-11, 0.3)
    mm = np.array([[0.0, 0.6, 0.8]])
    assert np.abs(P1.rhs(mm, 5e4 * mm[0])).max() < 1e-6


def test_ll_coefficients():
    import oracle

    c1, c2 = oracle.ll_coefficients(0.02, 2.21e5, 0)
    assert abs(c1 - 2.21e5 / 1.0004) < 1e-9 and abs(c2 - 0.02 * 2.21e5 / 1.0004) < 1e-9
    assert oracle.ll_coefficients(4.42e3, 2.21e5, 1) == (2.21e5, 4.42e3)


def test_sp4_parameters_match_paper():
    with open(os.path.join(os.path.dirname(__file__), "golden", "sp4_parameters.json")) as f:
        g = json.load(f)
    wl = W.thin_film()
    assert wl.A == g["A_exch_J_per_m"] and wl.Ms == g["Ms_A_per_m"]
    ext = (wl.centers + 0.5 * wl.sizes).max(0) - (wl.centers - 0.5 * wl.sizes).min(0)
    np.testing.assert_allclose(ext * 1e9, g["film_nm"], rtol=1e-12)
    assert len(np.unique(wl.centers[:, 2])) == g["tiles_through_thickness"]
    # the paper's LL damping is the Gilbert damping 0.02 times gamma:
    # alpha_LL / gamma_LL = 0.02 (the film's damping)
    assert abs(g["alpha_LL"] / g["gamma_LL"] - wl.alpha) < 1e-12
    assert wl.gamma0 == g["gamma_LL"]


def test_oracle_regression_fixture():
    """The oracle still produces the values frozen in tests/golden (written
    by tests/golden/make_oracle_regression.py from the oracle alone)."""
    import importlib.util

    here = os.path.join(os.path.dirname(__file__), "golden")
    spec = importlib.util.spec_from_file_location("mk", os.path.join(here, "make_oracle_regression.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    with open(os.path.join(here, "oracle_regression.json")) as f:
        want = json.load(f)
    got = mk.compute()
    for key in ("blocks",):
        for b in want[key]:
            np.testing.assert_allclose(got[key][b], want[key][b], rtol=1e-13, atol=1e-17)
    for key in ("demag_first_tiles", "energy", "rk4_10_steps_first_tiles"):
        np.testing.assert_allclose(got[key], want[key], rtol=1e-12, atol=1e-30)


def test_diagnostics_definitions(orc):
    """Mean magnetisation of a uniform state is that state; weights are the
    tile moments V Ms; max |dm/dt| is zero for a single tile magnetised along
    its field and positive otherwise; a NaN is flagged."""
    c, s = W.grid(3, 2, 2, 5e-9, 4e-9, 3e-9)
    n = c.shape[0]
    Ms = np.linspace(6e5, 9e5, n)
    P = orc.Problem(c, s, Ms, 1.3e-11, 0.5)
    u = np.array([0.28, -0.48, 0.83])
    u /= np.linalg.norm(u)
    D = P.diagnostics(np.tile(u, (n, 1)))
    np.testing.assert_allclose(D[4:7], u, rtol=0, atol=1e-15)
    np.testing.assert_allclose(D[:4], P.energy(np.tile(u, (n, 1))), rtol=1e-15)
    m = W.random_unit_vectors(4, n)
    D = P.diagnostics(m)
    w = P.vol * Ms
    np.testing.assert_allclose(D[4:7], (w[:, None] * m).sum(0) / w.sum(), rtol=1e-14)
    assert D[7] > 0 and D[8] == 0
    P1 = orc.Problem(np.zeros((1, 3)), np.full((1, 3), 5e-9), 8e5, 1.3e-11, 0.3)
    mm = np.array([[0.0, 0.6, 0.8]])
    assert P1.diagnostics(mm, 5e4 * mm[0])[7] < 1e-6
    bad = m.copy()
    bad[3, 1] = np.nan
    assert P.diagnostics(bad)[8] == 1.0
