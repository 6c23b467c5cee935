"""GPU parity of the pair-symmetric operators (PSYM6 and PSYM4: meshes of identical
tiles, where N^{ab} = N^{ba}, store each pair of blocks once) through the C
ABI, against the FP64 oracle's dense operator.

Tolerances (as for the float32 SYM6 path):
  stored blocks       |dN| <= 2^-24 |N| + 1e-14 against the oracle's N^{ab}
  H_d / H_eff         relative 2-norm and max-norm error <= 1e-5
  RK4, 200 steps      max |dm| <= 1e-4
The summation order of the product depends only on the tile count, so a
state's result is bitwise the same alone and in a batch.
"""
import sys

import numpy as np
import pytest

from gpu_helpers import build, close, device_state, rel_errors, tilemag
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


def _meshes():
    cube = W.cube_grid()
    return {
        "cube8": (cube.centers, cube.sizes),
        "grid13x5": W.grid(13, 5, 1, 5e-9, 4e-9, 3e-9),
        "grid7x5x3": W.grid(7, 5, 3, 4e-9, 4e-9, 6e-9),
        "single": (np.zeros((1, 3)), np.array([[5e-9, 4e-9, 3e-9]])),
    }


def _psym(tmg, ctx, c, s, alpha=0.5):
    return build(tmg, ctx, c, s, alpha=alpha, layout=tmg.TM_LAYOUT_PSYM6)


@pytest.mark.parametrize("name", ["cube8", "grid13x5", "grid7x5x3", "single"])
def test_psym_blocks_match_oracle(tmg, ctx, orc, name):
    c, s = _meshes()[name]
    _say("psym blocks %s n=%d" % (name, c.shape[0]))
    g = tmg.Geometry(ctx, c, s)
    T = tmg.Tensor(ctx, g, tmg.TM_PREC_FP32, tmg.TM_LAYOUT_PSYM6)
    got = T.dense()
    want = orc.assemble(c, s)
    assert np.all(np.abs(got - want) <= 2.0**-24 * np.abs(want) + 1e-14)
    # single blocks read back through the other entry point
    n = c.shape[0]
    for a, b in ((0, n - 1), (n - 1, 0), (n // 2, n // 3)):
        assert np.array_equal(T.block(a, b), got[3 * a:3 * a + 3, 3 * b:3 * b + 3])
    close(g, T)


@pytest.mark.parametrize("name,B", [("cube8", 1), ("grid13x5", 3), ("grid7x5x3", 2), ("single", 1)])
def test_psym_demag_and_heff(tmg, ctx, orc, name, B):
    c, s = _meshes()[name]
    n = c.shape[0]
    _say("psym demag %s n=%d B=%d" % (name, n, B))
    g, T, p = _psym(tmg, ctx, c, s)
    m = np.stack([W.random_unit_vectors(60 + k, n) for k in range(B)])
    md = device_state(m)
    Hd = p.demag(md).cpu().numpy()
    He = p.heff(md).cpu().numpy()
    P = orc.Problem(c, s, 8.0e5, 1.3e-11, 0.5)
    for k in range(B):
        mk = m[k].astype(np.float32).astype(np.float64)
        e2, emax = rel_errors(Hd[k], P.demag(mk))
        assert e2 <= 1e-5 and emax <= 1e-5, ("demag", k, e2, emax)
        e2, emax = rel_errors(He[k], P.heff(mk))
        assert e2 <= 1e-5 and emax <= 1e-5, ("heff", k, e2, emax)
    close(g, T, p)


def test_psym_film_full(tmg, ctx, orc):
    wl = W.thin_film()
    g, T, p = _psym(tmg, ctx, wl.centers, wl.sizes)
    m = wl.m0.astype(np.float32)
    Hd = p.demag(device_state(m)).cpu().numpy()[0]
    want = orc.demag(orc.assemble(wl.centers, wl.sizes), 8.0e5, m[0].astype(np.float64))
    e2, emax = rel_errors(Hd, want)
    assert e2 <= 1e-5 and emax <= 1e-5, (e2, emax)
    # about half the bytes of the six-plane layout
    assert T.nbytes < 0.53 * 24 * wl.n * wl.n
    close(g, T, p)


def test_psym_batch_invariance(tmg, ctx):
    c, s = _meshes()["grid7x5x3"]
    n = c.shape[0]
    g, T, p = _psym(tmg, ctx, c, s)
    m = np.stack([W.random_unit_vectors(80 + k, n) for k in range(4)])
    H4 = p.demag(device_state(m)).cpu().numpy()
    H1 = p.demag(device_state(m[2:3])).cpu().numpy()
    assert np.array_equal(H4[2], H1[0])
    close(g, T, p)


def test_psym_rk4_cube_grid(tmg, ctx, orc):
    wl = W.cube_grid()
    _say("psym rk4 cube grid 200 steps")
    g, T, p = _psym(tmg, ctx, wl.centers, wl.sizes, alpha=wl.alpha)
    m0 = wl.m0.astype(np.float32)
    md = device_state(m0)
    t, dt, steps, st = p.run(md, None, tmg.TM_RK4, dt=1e-13, max_steps=200)
    got = md.cpu().numpy()[0]
    P = orc.Problem(wl.centers, wl.sizes, wl.Ms, wl.A, wl.alpha)
    want = P.rk4(m0[0].astype(np.float64), [0, 0, 0], 1e-13, 200)
    assert int(steps.cpu()[0]) == 200
    assert np.abs(got - want).max() <= 1e-4
    assert np.abs(np.linalg.norm(got, axis=1) - 1).max() < 1e-6
    close(g, T, p)


def test_psym_dp45_one_step_film(tmg, ctx, orc):
    import torch

    wl = W.thin_film()
    g, T, p = _psym(tmg, ctx, wl.centers, wl.sizes, alpha=wl.alpha)
    m0 = wl.m0.astype(np.float32)
    Ha = wl.Ha.astype(np.float32)
    md = device_state(m0)
    t, dt, steps, st = p.run(md, torch.as_tensor(Ha, device="cuda"), tmg.TM_DP45, dt=2e-14,
                             max_steps=1, max_attempts=1)
    P = orc.Problem(wl.centers, wl.sizes, wl.Ms, wl.A, wl.alpha)
    y = m0[0].astype(np.float64).copy()
    k1 = P.rhs(y, Ha[0].astype(np.float64))
    ok, dtn, tn, err, _ = P.dp45_attempt(y, k1, Ha[0].astype(np.float64), 2e-14, 0.0)
    assert ok and int(steps.cpu()[0]) == 1
    assert float(t.cpu()[0]) == tn
    assert np.abs(md.cpu().numpy()[0] - y).max() <= 1e-5
    assert abs(float(dt.cpu()[0]) / dtn - 1) < 1e-3
    close(g, T, p)


def test_psym_dp45_film_matches_six_plane_path(tmg, ctx):
    """200 adaptive attempts on the film with PSYM6 and with SYM6: the two
    operators hold the same float32 values, so the trajectories agree to the
    float32 product's rounding (summation orders differ)."""
    import torch

    wl = W.thin_film()
    Ha = torch.as_tensor(wl.Ha.astype(np.float32), device="cuda")
    out = []
    for layout in (tmg.TM_LAYOUT_PSYM6, tmg.TM_LAYOUT_SYM6):
        g, T, p = build(tmg, ctx, wl.centers, wl.sizes, alpha=wl.alpha, layout=layout)
        md = device_state(wl.m0)
        t, dt, steps, st = p.run(md, Ha, tmg.TM_DP45, dt=1e-14, max_steps=1 << 40, max_attempts=200,
                                 t_end=2e-12)
        out.append((md.cpu().numpy()[0], float(t.cpu()[0])))
        close(g, T, p)
    assert abs(out[0][1] - out[1][1]) <= 1e-6 * out[1][1] or out[0][1] == out[1][1]
    assert np.abs(out[0][0] - out[1][0]).max() <= 1e-4


def test_psym_rejects_unlike_tiles(tmg, ctx):
    slab = W.refined_slab(n_target=300, lx=200e-9, ly=60e-9, lz=20e-9)
    g = tmg.Geometry(ctx, slab.centers, slab.sizes)
    with pytest.raises(tmg.TilemagError) as ei:
        tmg.Tensor(ctx, g, tmg.TM_PREC_FP32, tmg.TM_LAYOUT_PSYM6)
    assert ei.value.status == tmg.TM_EINVAL
    c, s = _meshes()["grid13x5"]
    g2 = tmg.Geometry(ctx, c, s)
    with pytest.raises(tmg.TilemagError):
        tmg.Tensor(ctx, g2, tmg.TM_PREC_FP64, tmg.TM_LAYOUT_PSYM6)
    close(g, g2)


def test_psym_streamed_size_rows(tmg, ctx, orc):
    """The SP4 film at [160, 40, 1] (N = 6400): the pair-symmetric operator
    (494 MB) exceeds the Infinity Cache and is streamed with nontemporal
    loads; sampled rows of H_d and H_eff against the oracle's rows."""
    wl = W.thin_film(nx=160, ny=40)
    g, T, p = _psym(tmg, ctx, wl.centers, wl.sizes, alpha=wl.alpha)
    assert T.nbytes > 192 * 2**20
    m = wl.m0.astype(np.float32)
    Hd = p.demag(device_state(m)).cpu().numpy()[0]
    rows = np.array([0, 1, 31, 32, 33, 159, 160, 3199, 3200, 6367, 6398, 6399])
    want = orc.demag_rows(wl.centers, wl.sizes, wl.Ms, m[0].astype(np.float64), rows)
    e2, emax = rel_errors(Hd[rows], want)
    assert e2 <= 1e-5 and emax <= 1e-5, (e2, emax)
    close(g, T, p)


# ---------------------------------------------------------------- PSYM4
# A single layer of identical tiles: every pair has a zero z offset, where
# the xz and yz components (odd in that offset) vanish, so four planes are
# stored.  Same tolerances as above; the oracle's dense operator (all nine
# components, computed from the closed form) is the reference, so the zero
# planes are checked against it too.

def _layers():
    film = W.thin_film()
    return {
        "grid13x5": W.grid(13, 5, 1, 5e-9, 4e-9, 3e-9),
        "grid45x7": W.grid(45, 7, 1, 5e-9, 5e-9, 3e-9),  # 315 tiles: ten tiles a side, ragged last
        "single": (np.zeros((1, 3)), np.array([[5e-9, 4e-9, 3e-9]])),
        "film": (film.centers, film.sizes),
    }


@pytest.mark.parametrize("name", ["grid13x5", "grid45x7", "single"])
def test_psym4_blocks_match_oracle(tmg, ctx, orc, name):
    c, s = _layers()[name]
    n = c.shape[0]
    _say("psym4 blocks %s n=%d" % (name, n))
    g = tmg.Geometry(ctx, c, s)
    T4 = tmg.Tensor(ctx, g, tmg.TM_PREC_FP32, tmg.TM_LAYOUT_PSYM4)
    T6 = tmg.Tensor(ctx, g, tmg.TM_PREC_FP32, tmg.TM_LAYOUT_PSYM6)
    got, six = T4.dense(), T6.dense()
    want = orc.assemble(c, s)
    assert np.all(np.abs(got - want) <= 2.0**-24 * np.abs(want) + 1e-14)
    # the vanishing components: zero as stored, and zero to rounding in the oracle
    for i, j in ((0, 2), (2, 0), (1, 2), (2, 1)):
        assert np.all(got[i::3, j::3] == 0.0)
        assert np.abs(want[i::3, j::3]).max() <= 1e-14
    # the four kept planes hold the six-plane layout's float32 values
    for i, j in ((0, 0), (0, 1), (1, 0), (1, 1), (2, 2)):
        assert np.array_equal(got[i::3, j::3], six[i::3, j::3])
    for a, b in ((0, n - 1), (n - 1, 0), (n // 2, n // 3)):
        assert np.array_equal(T4.block(a, b), got[3 * a:3 * a + 3, 3 * b:3 * b + 3])
    assert abs(T4.nbytes / T6.nbytes - 2.0 / 3.0) < 0.01
    close(g, T6, T4)


@pytest.mark.parametrize("name,B", [("grid13x5", 3), ("grid45x7", 2), ("single", 1)])
def test_psym4_demag_and_heff(tmg, ctx, orc, name, B):
    c, s = _layers()[name]
    n = c.shape[0]
    _say("psym4 demag %s n=%d B=%d" % (name, n, B))
    g, T, p = build(tmg, ctx, c, s, layout=tmg.TM_LAYOUT_PSYM4)
    m = np.stack([W.random_unit_vectors(90 + k, n) for k in range(B)])
    md = device_state(m)
    Hd = p.demag(md).cpu().numpy()
    He = p.heff(md).cpu().numpy()
    P = orc.Problem(c, s, 8.0e5, 1.3e-11, 0.5)
    for k in range(B):
        mk = m[k].astype(np.float32).astype(np.float64)
        e2, emax = rel_errors(Hd[k], P.demag(mk))
        assert e2 <= 1e-5 and emax <= 1e-5, ("demag", k, e2, emax)
        e2, emax = rel_errors(He[k], P.heff(mk))
        assert e2 <= 1e-5 and emax <= 1e-5, ("heff", k, e2, emax)
    if B > 1:  # a state's result does not depend on the batch
        H1 = p.demag(device_state(m[1:2])).cpu().numpy()
        assert np.array_equal(H1[0], Hd[1])
    close(g, T, p)


def test_psym4_film_full_and_one_dp45_step(tmg, ctx, orc):
    import torch

    wl = W.thin_film()
    _say("psym4 film demag + one DP45 step")
    g, T, p = build(tmg, ctx, wl.centers, wl.sizes, alpha=wl.alpha, layout=tmg.TM_LAYOUT_PSYM4)
    assert T.nbytes < 0.36 * 24 * wl.n * wl.n  # a third of the SYM6 bytes, plus the padded tail
    m0 = wl.m0.astype(np.float32)
    A = orc.assemble(wl.centers, wl.sizes)
    Hd = p.demag(device_state(m0)).cpu().numpy()[0]
    e2, emax = rel_errors(Hd, orc.demag(A, 8.0e5, m0[0].astype(np.float64)))
    assert e2 <= 1e-5 and emax <= 1e-5, (e2, emax)
    Ha = wl.Ha.astype(np.float32)
    md = device_state(m0)
    t, dt, steps, st = p.run(md, torch.as_tensor(Ha, device="cuda"), tmg.TM_DP45, dt=2e-14,
                             max_steps=1, max_attempts=1)
    P = orc.Problem(wl.centers, wl.sizes, wl.Ms, wl.A, wl.alpha)
    y = m0[0].astype(np.float64).copy()
    k1 = P.rhs(y, Ha[0].astype(np.float64))
    ok, dtn, tn, err, _ = P.dp45_attempt(y, k1, Ha[0].astype(np.float64), 2e-14, 0.0)
    assert ok and int(steps.cpu()[0]) == 1
    assert float(t.cpu()[0]) == tn
    assert np.abs(md.cpu().numpy()[0] - y).max() <= 1e-5
    assert abs(float(dt.cpu()[0]) / dtn - 1) < 1e-3
    close(g, T, p)


def test_psym4_dp45_film_matches_six_plane_path(tmg, ctx):
    """200 adaptive attempts on the film with PSYM4 and with PSYM6: the
    dropped planes hold values at the rounding level, so the trajectories
    agree to the float32 product's rounding."""
    import torch

    wl = W.thin_film()
    Ha = torch.as_tensor(wl.Ha.astype(np.float32), device="cuda")
    out = []
    for layout in (tmg.TM_LAYOUT_PSYM4, tmg.TM_LAYOUT_PSYM6):
        g, T, p = build(tmg, ctx, wl.centers, wl.sizes, alpha=wl.alpha, layout=layout)
        md = device_state(wl.m0)
        t, dt, steps, st = p.run(md, Ha, tmg.TM_DP45, dt=1e-14, max_steps=1 << 40, max_attempts=200,
                                 t_end=2e-12)
        out.append((md.cpu().numpy()[0], float(t.cpu()[0])))
        close(g, T, p)
    assert abs(out[0][1] - out[1][1]) <= 1e-6 * out[1][1] or out[0][1] == out[1][1]
    assert np.abs(out[0][0] - out[1][0]).max() <= 1e-4


def test_psym4_rejects_several_layers(tmg, ctx):
    c, s = _meshes()["grid7x5x3"]
    g = tmg.Geometry(ctx, c, s)
    with pytest.raises(tmg.TilemagError) as ei:
        tmg.Tensor(ctx, g, tmg.TM_PREC_FP32, tmg.TM_LAYOUT_PSYM4)
    assert ei.value.status == tmg.TM_EINVAL
    # one tile lifted off the layer
    c2, s2 = _layers()["grid13x5"]
    c2 = c2.copy()
    c2[7, 2] += 1e-12
    g2 = tmg.Geometry(ctx, c2, s2)
    with pytest.raises(tmg.TilemagError) as ei:
        tmg.Tensor(ctx, g2, tmg.TM_PREC_FP32, tmg.TM_LAYOUT_PSYM4)
    assert ei.value.status == tmg.TM_EINVAL
    c3, s3 = _layers()["grid13x5"]
    g3 = tmg.Geometry(ctx, c3, s3)
    with pytest.raises(tmg.TilemagError):
        tmg.Tensor(ctx, g3, tmg.TM_PREC_FP64, tmg.TM_LAYOUT_PSYM4)
    close(g, g2, g3)


def test_psym4_streamed_size_rows(tmg, ctx, orc):
    """The film at [160, 40, 1] (N = 6400): the four-plane operator (329 MB)
    exceeds the Infinity Cache and is streamed with nontemporal loads;
    sampled rows of H_d against the oracle's rows."""
    wl = W.thin_film(nx=160, ny=40)
    g, T, p = build(tmg, ctx, wl.centers, wl.sizes, alpha=wl.alpha, layout=tmg.TM_LAYOUT_PSYM4)
    assert T.nbytes > 192 * 2**20
    m = wl.m0.astype(np.float32)
    Hd = p.demag(device_state(m)).cpu().numpy()[0]
    rows = np.array([0, 1, 31, 32, 33, 159, 160, 3199, 3200, 6367, 6398, 6399])
    want = orc.demag_rows(wl.centers, wl.sizes, wl.Ms, m[0].astype(np.float64), rows)
    e2, emax = rel_errors(Hd[rows], want)
    assert e2 <= 1e-5 and emax <= 1e-5, (e2, emax)
    close(g, T, p)


def test_psym_tuned_loads_same_results(tmg, ctx):
    """tm_problem_tune on a pair-symmetric problem picks cached (0) or
    nontemporal (1) operator loads for the tile pass; the arithmetic is the
    same, so the field is bitwise unchanged."""
    for layout in (tmg.TM_LAYOUT_PSYM4, tmg.TM_LAYOUT_PSYM6):
        c, s = _layers()["grid45x7"]
        g, T, p = build(tmg, ctx, c, s, layout=layout)
        md = device_state(np.stack([W.random_unit_vectors(120 + k, c.shape[0]) for k in range(2)]))
        before = p.heff(md).cpu().numpy()
        chosen, ms = tmg.tm_problem_tune(p.handle, 2, 3)
        assert chosen in (0, 1) and ms > 0
        assert np.array_equal(p.heff(md).cpu().numpy(), before)
        close(g, T, p)


@pytest.mark.parametrize("layout", ["psym4", "psym6"])
def test_psym_batch_shares_tile_reads_film(tmg, ctx, orc, layout):
    """On the film (3160 tile pairs) one workgroup per pair applies its tile
    to every state of the batch; each state's field and DP45 steps are
    bitwise those it gets alone, and the field meets the oracle tolerance."""
    import torch

    wl = W.thin_film()
    lay = tmg.TM_LAYOUT_PSYM4 if layout == "psym4" else tmg.TM_LAYOUT_PSYM6
    _say("%s film batch of 3 sharing tile reads" % layout)
    g, T, p = build(tmg, ctx, wl.centers, wl.sizes, alpha=wl.alpha, layout=lay)
    m = np.stack([W.film_texture(wl.centers, 500e-9, 200 + k) for k in range(3)]).astype(np.float32)
    Ha = np.array([[2e4, 1e4, 0.0], [-3e4, 0.0, 0.0], [0.0, 2e4, 0.0]], np.float32)
    H3 = p.heff(device_state(m), torch.as_tensor(Ha, device="cuda")).cpu().numpy()
    P = orc.Problem(wl.centers, wl.sizes, wl.Ms, wl.A, wl.alpha)
    for k in range(3):
        one = p.heff(device_state(m[k:k + 1]), torch.as_tensor(Ha[k:k + 1], device="cuda")).cpu().numpy()
        assert np.array_equal(H3[k], one[0]), k
    e2, emax = rel_errors(H3[1], P.heff(m[1].astype(np.float64), Ha[1].astype(np.float64)))
    assert e2 <= 1e-5 and emax <= 1e-5, (e2, emax)
    md = device_state(m)
    t, dt, steps, st = p.run(md, torch.as_tensor(Ha, device="cuda"), tmg.TM_DP45, dt=1e-14, max_steps=1 << 30,
                             max_attempts=3)
    got3 = md.cpu().numpy()
    for k in range(3):
        mk = device_state(m[k:k + 1])
        p.run(mk, torch.as_tensor(Ha[k:k + 1], device="cuda"), tmg.TM_DP45, dt=1e-14, max_steps=1 << 30,
              max_attempts=3)
        assert np.array_equal(got3[k], mk.cpu().numpy()[0]), k
    close(g, T, p)
