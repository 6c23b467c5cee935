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
