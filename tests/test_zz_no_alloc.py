"""tm_demag_noalloc (the demag field on the library's fixed scratch buffer,
for callers that cannot allocate) against tm_demag, through the C ABI.

Two calls in a row on the same device buffer, the second with a smaller
input (fewer tiles, fewer states, another operator layout), each compared
bitwise with tm_demag on the same problem and states (same kernels and
summation order) and with the FP64 oracle (relative 2-norm and max-norm
<= 1e-5, the float32 demag tolerance).  Also: the call changes no device
memory figure (nothing allocated), a batch beyond the buffer and a DENSE9
operator are refused before anything is enqueued, and a third call back at
the first size still matches (no state carried between calls).
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


def _noalloc_vs_demag(tmg, p, n, m, oracle_problem):
    import torch

    ref = p.demag(m)  # tm_demag (allocates its workspace on first use)
    torch.cuda.synchronize()
    out = torch.full_like(m, float("nan"))
    free0 = torch.cuda.mem_get_info()[0]
    tmg.tm_demag_noalloc(p.handle, n, m, out)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free0 == free1, "tm_demag_noalloc changed free device memory: %d -> %d" % (free0, free1)
    assert torch.equal(out, ref), "tm_demag_noalloc differs from tm_demag"
    got = out.cpu().numpy()
    mm = m.cpu().numpy()
    for k in range(m.shape[0]):
        e2, emax = rel_errors(got[k], oracle_problem.demag(mm[k].astype(np.float64)))
        assert e2 <= 1e-5 and emax <= 1e-5, (k, e2, emax)


def test_noalloc_matches_demag(orc):
    import torch

    tmg = tilemag()
    ctx = tmg.Context(0)
    # call 1: the film (N = 2500), four-plane pair-symmetric operator, 3 states
    wl = W.thin_film()
    _say("noalloc call 1: film N=%d psym4 B=3" % wl.n)
    g1, T1, p1 = build(tmg, ctx, wl.centers, wl.sizes, alpha=wl.alpha, layout=tmg.TM_LAYOUT_PSYM4)
    m1 = device_state(np.stack([W.random_unit_vectors(50 + k, wl.n) for k in range(3)]))
    P1 = orc.Problem(wl.centers, wl.sizes, wl.Ms, wl.A, wl.alpha)
    _noalloc_vs_demag(tmg, p1, wl.n, m1, P1)
    # call 2, smaller: 90 tiles in two layers, six-plane pair-symmetric, per-tile Ms, 2 states
    c2, s2 = W.grid(9, 5, 2, 5e-9, 5e-9, 3e-9)
    n2 = c2.shape[0]
    Ms2 = np.linspace(6.0e5, 9.0e5, n2)
    _say("noalloc call 2: n=%d psym6 B=2" % n2)
    g2, T2, p2 = build(tmg, ctx, c2, s2, Ms=Ms2, layout=tmg.TM_LAYOUT_PSYM6)
    m2 = device_state(np.stack([W.random_unit_vectors(60 + k, n2) for k in range(2)]))
    _noalloc_vs_demag(tmg, p2, n2, m2, orc.Problem(c2, s2, Ms2, 1.3e-11, 0.5))
    # call 3, smaller still: non-uniform refined slab, six planes, one state
    slab = W.refined_slab(n_target=150, lx=100e-9, ly=40e-9, lz=20e-9)
    n3 = slab.centers.shape[0]
    _say("noalloc call 3: refined n=%d sym6 B=1" % n3)
    g3, T3, p3 = build(tmg, ctx, slab.centers, slab.sizes)
    m3 = device_state(W.random_unit_vectors(70, n3)[None])
    _noalloc_vs_demag(tmg, p3, n3, m3, orc.Problem(slab.centers, slab.sizes, 8.0e5, 1.3e-11, 0.5))
    # back at the first size: nothing from the smaller calls leaks into it
    _say("noalloc call 4: film again")
    _noalloc_vs_demag(tmg, p1, wl.n, m1, P1)
    # refused before anything is enqueued: a batch beyond the buffer ...
    big = torch.zeros((14, wl.n, 3), dtype=torch.float32, device="cuda")
    out = torch.empty_like(big)
    r = tmg.tm_demag_noalloc(p1.handle, wl.n, big, out, check=False)
    assert r == tmg.TM_EINVAL
    assert "scratch" in tmg.tm_last_error()
    # ... and an operator it does not take (the batched DENSE9 product)
    g4, T4, p4 = build(tmg, ctx, c2, s2, layout=tmg.TM_LAYOUT_DENSE9)
    r = tmg.tm_demag_noalloc(p4.handle, n2, m2, torch.empty_like(m2), check=False)
    assert r == tmg.TM_EINVAL
    close(g4, T4, p4)
    close(g3, T3, p3)
    close(g2, T2, p2)
    close(g1, T1, p1)
    ctx.close()
