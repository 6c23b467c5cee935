"""GPU parity of the batched path: many states sharing one operator, the
demag product as one MFMA GEMM (DENSE9 operator) in float32 or bf16 / fp16
hi + lo split precision with float32 accumulation.

Tolerances on H_d against the FP64 oracle (relative 2-norm and max-norm):
  FP32   <= 1e-5
  BF16X3 <= 1e-3 (three bf16 products carry ~16 significant bits)
  FP16X3 <= 2e-5 (three fp16 products with per-row scaling carry ~22 bits)
The measured errors are printed.
"""
import sys

import numpy as np
import pytest

from gpu_helpers import build, close, device_state, rel_errors, tilemag
from paper_2107_05364_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 1e-3, 2: 2e-5}
NAMES = {0: "fp32", 1: "bf16x3", 2: "fp16x3"}


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
def film_ref(orc):
    wl = W.hysteresis_batch(B=128)
    T = orc.assemble(wl.centers, wl.sizes)
    m = wl.m0.astype(np.float32)
    # FP64 oracle product for all states: one library matmul of the oracle's operator
    H = -(8.0e5 * m.astype(np.float64).reshape(128, -1)) @ T.T
    return wl, m, H.reshape(128, wl.n, 3)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_batched_demag_film_128_states(tmg, ctx, film_ref, prec):
    wl, m, H = film_ref
    _say("batched demag %s B=128 n=%d" % (NAMES[prec], wl.n))
    g, T, p = build(tmg, ctx, wl.centers, wl.sizes, alpha=wl.alpha, store=prec,
                    layout=tmg.TM_LAYOUT_DENSE9)
    got = p.demag(device_state(m)).cpu().numpy()
    e2, emax = rel_errors(got, H)
    _say("  %s: rel2 %.3e relmax %.3e" % (NAMES[prec], e2, emax))
    assert e2 <= TOL[prec] and emax <= TOL[prec]
    # and with the split count the benchmark tunes
    splits, _ = tmg.tm_problem_tune(p.handle, 128, 3)
    got = p.demag(device_state(m)).cpu().numpy()
    e2, emax = rel_errors(got, H)
    _say("  %s, %d K splits: rel2 %.3e relmax %.3e" % (NAMES[prec], splits, e2, emax))
    assert e2 <= TOL[prec] and emax <= TOL[prec]
    close(g, T, p)


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("B", [1, 3, 33])
def test_batched_demag_ragged(tmg, ctx, orc, prec, B):
    """Non-uniform tiles and per-tile Ms, a batch that is not a multiple of
    16 and a tile count that is not a multiple of 64."""
    wl = W.refined_slab(n_target=777, lx=200e-9, ly=60e-9, lz=20e-9)
    n = wl.n
    Ms = 8.0e5 * (0.75 + 0.5 * W.uniform(9, n))
    g, T, p = build(tmg, ctx, wl.centers, wl.sizes, Ms=Ms, store=prec, layout=tmg.TM_LAYOUT_DENSE9)
    m = np.stack([W.random_unit_vectors(40 + k, n) for k in range(B)]).astype(np.float32)
    got = p.demag(device_state(m)).cpu().numpy()
    Tref = orc.assemble(wl.centers, wl.sizes)
    for k in range(B):
        want = orc.demag(Tref, Ms, m[k].astype(np.float64))
        e2, emax = rel_errors(got[k], want)
        assert e2 <= TOL[prec] and emax <= TOL[prec], (k, e2, emax)
    close(g, T, p)


@pytest.mark.parametrize("prec", [0, 1])
def test_batched_state_is_batch_invariant(tmg, ctx, prec):
    """A state's demag field is bit-identical alone and in a batch of 40."""
    wl = W.thin_film(nx=40, ny=10)
    g, T, p = build(tmg, ctx, wl.centers, wl.sizes, store=prec, layout=tmg.TM_LAYOUT_DENSE9)
    m = np.stack([W.film_texture(wl.centers, 200e-9, k) for k in range(40)]).astype(np.float32)
    many = p.demag(device_state(m)).cpu().numpy()
    one = p.demag(device_state(m[17:18])).cpu().numpy()
    assert np.array_equal(many[17], one[0])
    close(g, T, p)


@pytest.mark.parametrize("prec", [0, 1])
def test_tuned_split_count(tmg, ctx, orc, prec):
    """tm_problem_tune on the batched product keeps one of its K-split
    candidates; after tuning H_d still meets the oracle tolerance, a repeat
    is bitwise identical, and a state is bit-identical alone and in the batch
    (the split count fixes the summation order)."""
    wl = W.thin_film(nx=40, ny=10)
    g, T, p = build(tmg, ctx, wl.centers, wl.sizes, store=prec, layout=tmg.TM_LAYOUT_DENSE9)
    m = np.stack([W.film_texture(wl.centers, 200e-9, k) for k in range(24)]).astype(np.float32)
    chosen, ms = tmg.tm_problem_tune(p.handle, 24, 2)
    _say("%s: %d K splits, %.1f us" % (NAMES[prec], chosen, ms * 1e3))
    assert chosen in (2, 3, 4, 5, 6, 8) and ms > 0
    H = p.demag(device_state(m)).cpu().numpy()
    P = orc.Problem(wl.centers, wl.sizes, 8.0e5, 1.3e-11, 0.5)
    for k in (0, 11, 23):
        e2, emax = rel_errors(H[k], P.demag(m[k].astype(np.float64)))
        assert e2 <= TOL[prec] and emax <= TOL[prec], (k, e2, emax)
    assert np.array_equal(H, p.demag(device_state(m)).cpu().numpy())
    one = p.demag(device_state(m[5:6])).cpu().numpy()
    assert np.array_equal(H[5], one[0])
    close(g, T, p)


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("mesh", ["film", "slab"])
def test_every_split_count(tmg, ctx, orc, prec, mesh):
    """Every work plan the autotuner can pick (applied with tm_problem_apply):
    the K-split counts, on a single layer (component-blocked operator: the z
    rows take fewer splits, and some counts leave work items short of a whole
    number per XCD) and on a three-layer mesh with per-tile Ms (dense form),
    and on the single layer the aligned plans (choice 100 + super-ranges,
    where the operator's parts fit them; items of two z parts whose
    operator rows switch row block mid-item): H_d against the oracle within
    the precision's tolerance, a repeat bitwise identical."""
    if mesh == "film":
        wl = W.thin_film(nx=40, ny=10)
        centers, sizes = wl.centers, wl.sizes
        Ms = np.full(wl.n, 8.0e5)
    else:
        centers, sizes = W.grid(12, 8, 3, 5e-9, 5e-9, 3e-9)
        Ms = 8.0e5 * (0.75 + 0.5 * W.uniform(3, centers.shape[0]))
    n = centers.shape[0]
    g, T, p = build(tmg, ctx, centers, sizes, Ms=Ms, store=prec, layout=tmg.TM_LAYOUT_DENSE9)
    m = np.stack([W.random_unit_vectors(60 + k, n) for k in range(37)]).astype(np.float32)
    Tref = orc.assemble(centers, sizes)
    want = [orc.demag(Tref, Ms, m[k].astype(np.float64)) for k in (0, 18, 36)]
    aligned = 0
    for splits in (2, 3, 4, 5, 6, 8) + tuple(100 + q for q in range(2, 9)):
        try:
            tmg.tm_problem_apply(p.handle, splits)
        except tmg.TilemagError:
            assert splits >= 100, splits  # only aligned plans can be refused here
            continue
        aligned += splits >= 100
        H = p.demag(device_state(m)).cpu().numpy()
        for k, w in zip((0, 18, 36), want):
            e2, emax = rel_errors(H[k], w)
            assert e2 <= TOL[prec] and emax <= TOL[prec], (splits, k, e2, emax)
        assert np.array_equal(H, p.demag(device_state(m)).cpu().numpy()), splits
        _say("  %s %s, %d K splits ok" % (mesh, NAMES[prec], splits))
    # the film (np = 512: 8 z chunks, 4 z row blocks) admits 2, 4 and 8
    # super-ranges; the three-layer mesh keeps the dense form, which has none
    assert aligned == (3 if mesh == "film" else 0), aligned
    close(g, T, p)


@pytest.mark.parametrize("plan", [0, 102])
def test_batched_dp45_matches_matvec_path(tmg, ctx, plan):
    """DP45 on 8 states to a common end time: the FP32 GEMM path and the FP32
    matvec path (different summation orders) agree within the float32
    resolution of the tolerance-1e-6 integration.  The stages inside an
    attempt read the right operand their previous stage wrote; plan 102 (the
    aligned plan with two K super-ranges: items of two z row blocks) runs it
    through the two-segment product."""
    import torch

    wl = W.hysteresis_batch(B=8, nx=40, ny=10)
    Ha = torch.as_tensor(wl.Ha.astype(np.float32), device="cuda")
    ga, Ta, pa = build(tmg, ctx, wl.centers, wl.sizes, alpha=wl.alpha, layout=tmg.TM_LAYOUT_DENSE9)
    if plan:
        tmg.tm_problem_apply(pa.handle, plan)
    gb, Tb, pb = build(tmg, ctx, wl.centers, wl.sizes, alpha=wl.alpha)
    ma, mb = device_state(wl.m0), device_state(wl.m0)
    ta, _, sa, _ = pa.run(ma, Ha, tmg.TM_DP45, dt=1e-14, max_steps=1 << 20, t_end=20e-12)
    tb, _, sb, _ = pb.run(mb, Ha, tmg.TM_DP45, dt=1e-14, max_steps=1 << 20, t_end=20e-12)
    assert torch.allclose(ta, tb, rtol=0, atol=1e-24)
    d = (ma - mb).abs().max().item()
    _say("gemm vs matvec path after 20 ps: max|dm| %.2e, steps %s / %s"
         % (d, sa.cpu().tolist(), sb.cpu().tolist()))
    assert d <= 2e-5
    close(ga, Ta, pa, gb, Tb, pb)


@pytest.mark.parametrize("prec", [1, 2])
def test_split_precision_hysteresis_run(tmg, ctx, prec):
    """A short batched hysteresis run in split precision stays within the
    tolerance-level distance of the FP32 run (same states, same end time)."""
    import torch

    wl = W.hysteresis_batch(B=16, nx=40, ny=10)
    Ha = torch.as_tensor(wl.Ha.astype(np.float32), device="cuda")
    g1, T1, p1 = build(tmg, ctx, wl.centers, wl.sizes, alpha=wl.alpha, layout=tmg.TM_LAYOUT_DENSE9)
    g2, T2, p2 = build(tmg, ctx, wl.centers, wl.sizes, alpha=wl.alpha, store=prec,
                       layout=tmg.TM_LAYOUT_DENSE9)
    a, b = device_state(wl.m0), device_state(wl.m0)
    p1.run(a, Ha, tmg.TM_DP45, dt=1e-14, max_steps=1 << 20, t_end=10e-12)
    p2.run(b, Ha, tmg.TM_DP45, dt=1e-14, max_steps=1 << 20, t_end=10e-12)
    d = (a - b).abs().max().item()
    _say("split vs fp32 hysteresis run, 10 ps: max|dm| %.2e" % d)
    assert d <= 1e-3
    close(g1, T1, p1, g2, T2, p2)


def test_profile_modes_run(tmg, ctx):
    """The field-timing modes on a batched problem: the stand-alone stage
    update (0) and the stage updates as inside an attempt (4, reading the
    right operand the previous stage wrote) both time; 5 is refused."""
    wl = W.hysteresis_batch(B=8, nx=40, ny=10)
    g, T, p = build(tmg, ctx, wl.centers, wl.sizes, alpha=wl.alpha, store=1, layout=tmg.TM_LAYOUT_DENSE9)
    for mode in (0, 4):
        ms, nbytes = tmg.tm_profile_field_mode(p.handle, 8, mode, 3)
        assert ms > 0 and nbytes > 0, (mode, ms, nbytes)
    with pytest.raises(tmg.TilemagError):
        tmg.tm_profile_field_mode(p.handle, 8, 5, 3)
    close(g, T, p)
