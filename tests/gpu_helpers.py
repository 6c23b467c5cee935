"""Shared helpers of the GPU parity tests: build library objects for a
workload and compare against the FP64 oracle."""
import numpy as np


def tilemag():
    from paper_2107_05364_amd import tilemag as tmg

    tmg.load()  # raises if the HIP library has not been built
    return tmg


def device_state(m, dtype=None):
    import torch

    return torch.as_tensor(np.ascontiguousarray(m, dtype=np.float32), device="cuda")


def build(tmg, ctx, centers, sizes, Ms=8.0e5, A=1.3e-11, alpha=0.5, gamma0=2.21e5, ll_form=0,
          Ku=None, easy=None, store=None, layout=None):
    store = tmg.TM_PREC_FP32 if store is None else store
    layout = tmg.TM_LAYOUT_SYM6 if layout is None else layout
    g = tmg.Geometry(ctx, centers, sizes)
    T = tmg.Tensor(ctx, g, store, layout)
    p = tmg.Problem(ctx, g, T, Ms, A, alpha, gamma0, ll_form, Ku, easy)
    return g, T, p


def close(*objs):
    for o in reversed(objs):
        o.close()


def rel_errors(got, want):
    """(relative 2-norm error, max-abs error / max-abs reference)."""
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    d = got - want
    return (np.linalg.norm(d) / np.linalg.norm(want), np.abs(d).max() / np.abs(want).max())


# The float32 states and slopes of the GPU path resolve the scaled error
# estimate of a Dormand-Prince attempt only to about one float32 ulp of a unit
# vector component (2^-24) over the tolerance scale atol + rtol |y| (about
# 0.03 for atol = rtol = 1e-6, measured deviations from the FP64 oracle
# 1e-4 .. 1.5e-3).  The next step h min(5, max(0.2, 0.9 err^-1/5)) is then
# known to lie between the proposals for err + d and err - d.
def dp_step_bounds(h, err, atol=1e-6, rtol=1e-6):
    d = 2.0 ** -24 / (atol + rtol)

    def proposal(e):
        return h * (5.0 if e <= 0.0 else min(5.0, max(0.2, 0.9 * e ** -0.2)))

    return proposal(err + d) * (1 - 1e-12), proposal(max(err - d, 0.0)) * (1 + 1e-12)
