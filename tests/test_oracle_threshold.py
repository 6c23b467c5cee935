"""Pins of the oracle's thresholded operator (paper Sec. 4.3.1: the smallest
fraction of the nonzero tensor entries is truncated and the rest kept as a
sparse matrix).

Readings pinned here: magnitudes are ranked as float32 values, all 9 entries
of every block count, an entry is nonzero when its magnitude exceeds the
assembly's absolute accuracy (1e-14), the cut is the ceil(frac K)-th smallest
of the K nonzero magnitudes, entries at or below the cut go (ties included),
and self blocks are never truncated."""
import math

import numpy as np
import pytest

from paper_2107_05364_amd import workloads as W


def _mesh_uniform():
    return W.grid(4, 3, 2, 5e-9, 4e-9, 3e-9)


def _mesh_mixed():
    """Five non-overlapping cuboids of different shapes (no pair symmetry,
    few ties)."""
    c = np.array([[0.0, 0.0, 0.0], [9e-9, 1e-9, 0.0], [1e-9, 11e-9, 2e-9],
                  [-10e-9, 2e-9, -1e-9], [3e-9, -9e-9, 6e-9]])
    s = np.array([[5e-9, 5e-9, 5e-9], [4e-9, 7e-9, 3e-9], [8e-9, 3e-9, 5e-9],
                  [6e-9, 6e-9, 2e-9], [3e-9, 3e-9, 9e-9]])
    return c, s


FLOOR = float(np.float32(1e-14))


def _brute(T, frac):
    """Reference by counting, no sorting: the cut is the smallest magnitude x
    among the nonzero entries with #{|v| <= x} >= ceil(frac K)."""
    n = T.shape[0] // 3
    mags = [abs(float(np.float32(v))) for v in T.ravel()]
    nz = [v for v in mags if v > FLOOR]
    K = len(nz)
    r = math.ceil(frac * K)
    if r == 0:
        return np.ones(T.shape, bool)
    cut = None
    for x in nz:
        if sum(1 for v in nz if v <= x) >= r and (cut is None or x < cut):
            cut = x
    keep = np.zeros(T.shape, bool)
    for i in range(3 * n):
        for j in range(3 * n):
            keep[i, j] = (i // 3 == j // 3) or abs(float(np.float32(T[i, j]))) > cut
    return keep


def test_zero_fraction_is_identity(orc):
    c, s = _mesh_uniform()
    T = orc.assemble(c, s)
    t, cut = orc.threshold(T, 0.0)
    assert cut == -1.0
    assert np.array_equal(t, T)


@pytest.mark.parametrize("mesh", ["uniform", "mixed"])
@pytest.mark.parametrize("frac", [0.1, 0.25, 0.5, 0.77, 0.95])
def test_brute_force_rank(orc, mesh, frac):
    c, s = (W.grid(2, 2, 1, 5e-9, 5e-9, 3e-9) if mesh == "uniform" else _mesh_mixed())
    T = orc.assemble(c, s)
    t, _ = orc.threshold(T, frac)
    keep = _brute(T, frac)
    # removed entries are exactly zero, kept entries unchanged
    assert np.array_equal(t != 0, keep & (T != 0))
    assert np.array_equal(t[keep], T[keep])


def test_full_threshold_leaves_closed_form_self_terms(orc):
    """frac = 1 removes every entry outside the self blocks, so H_d at each
    tile is minus its own centre demagnetising tensor times Ms m, and that
    tensor is diagonal with the textbook closed form
    N_zz = (2/pi) atan(ab / (c sqrt(a^2 + b^2 + c^2))) (half-edges a, b, c)."""
    c, s = W.grid(3, 2, 2, 6e-9, 4e-9, 3e-9)
    n = c.shape[0]
    T = orc.assemble(c, s)
    t, _ = orc.threshold(T, 1.0)
    m = W.random_unit_vectors(7, n)
    Ms = 8.0e5
    a, b, cc = 3e-9, 2e-9, 1.5e-9

    def nzz(p, q, r):
        return 2.0 / math.pi * math.atan(p * q / (r * math.sqrt(p * p + q * q + r * r)))

    diag = np.array([nzz(b, cc, a), nzz(cc, a, b), nzz(a, b, cc)])
    want = -Ms * m * diag[None, :]
    np.testing.assert_allclose(orc.demag(t, Ms, m), want, rtol=1e-12, atol=1e-9)


def test_ties_at_the_cut_are_removed(orc):
    """On a uniform grid many magnitudes coincide by symmetry: when the cut
    falls inside a group of equal magnitudes the whole group goes, so more than
    ceil(frac K) entries may be removed, never fewer."""
    c, s = W.grid(4, 4, 1, 5e-9, 5e-9, 5e-9)
    T = orc.assemble(c, s)
    mags = np.abs(T.astype(np.float32)).astype(np.float64)
    K = int((mags > FLOOR).sum())
    self_blk = np.kron(np.eye(c.shape[0], dtype=bool), np.ones((3, 3), bool))
    hit_tie = False
    for frac in np.linspace(0.05, 0.95, 19):
        t, cut = orc.threshold(T, frac)
        removed = (T != 0) & (t == 0)
        assert not removed[self_blk].any()
        at_cut = (mags == cut) & ~self_blk
        assert removed[at_cut].all()
        lo = (mags <= cut) & (mags > FLOOR)
        assert lo.sum() >= math.ceil(frac * K)
        hit_tie |= at_cut.sum() > 1
    assert hit_tie


def test_rounding_noise_is_not_ranked(orc):
    """On the cube grid thousands of entries that vanish by symmetry come out
    of the float64 assembly as ~1e-17 noise: they count as zero, so K (and
    with it the cut) equals the count over magnitudes above 1e-14."""
    wl = W.cube_grid()
    T = orc.assemble(wl.centers, wl.sizes)
    mags = np.abs(T.astype(np.float32)).astype(np.float64)
    noise = (mags > 0) & (mags <= FLOOR)
    assert noise.sum() > 1000
    K = int((mags > FLOOR).sum())
    t, cut = orc.threshold(T, 0.3)
    srt = np.sort(mags[mags > FLOOR])
    assert cut == srt[math.ceil(0.3 * K) - 1]
    assert not (t[noise & (np.kron(np.eye(wl.n, dtype=bool), np.ones((3, 3), bool)) == 0)] != 0).any()


def test_monotone_in_fraction(orc):
    c, s = _mesh_uniform()
    T = orc.assemble(c, s)
    prev = np.ones(T.shape, bool)
    for frac in (0.0, 0.2, 0.4, 0.7, 1.0):
        t, _ = orc.threshold(T, frac)
        keep = t != 0
        assert not (keep & ~prev).any()
        prev = keep


def test_blocks_stay_symmetric(orc):
    """Each 3x3 block is symmetric, so its (i, j) and (j, i) entries share a
    magnitude and are kept or removed together."""
    c, s = _mesh_mixed()
    T = orc.assemble(c, s)
    n = c.shape[0]
    for frac in (0.3, 0.6):
        t, _ = orc.threshold(T, frac)
        for a in range(n):
            for b in range(n):
                blk = t[3 * a:3 * a + 3, 3 * b:3 * b + 3]
                assert np.array_equal(blk, blk.T)
