"""Python binding of the tilemag C ABI (``include/tilemag.h``).

Argument marshalling only: every step of the computation runs in the HIP
library ``libtilemag.so``.  Device buffers are torch tensors on the GPU
(float32 states ``[B, n, 3]``, float32 fields ``[B, 3]``, float64 times),
and calls are ordered on torch's current stream.  There is no CPU fallback:
if the library is missing or no GPU is present the calls raise.

The module-level functions carry the C names (``tm_init``, ``tm_demag``,
...); the classes below wrap them with ownership.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtilemag.so")

TM_OK, TM_EINVAL, TM_ENOMEM, TM_EDEVICE = 0, -1, -2, -3
TM_ENONFINITE, TM_ESTEP, TM_EBUSY, TM_ENOTFOUND = -4, -5, -6, -7
TM_PREC_FP32, TM_PREC_BF16X3, TM_PREC_FP16X3, TM_PREC_FP64 = 0, 1, 2, 3
TM_LAYOUT_SYM6, TM_LAYOUT_DENSE9, TM_LAYOUT_BSR6, TM_LAYOUT_PSYM6, TM_LAYOUT_PSYM4 = 0, 1, 2, 3, 4
TM_RK4, TM_DP45 = 0, 1

_STATUS_NAMES = {0: "TM_OK", -1: "TM_EINVAL", -2: "TM_ENOMEM", -3: "TM_EDEVICE",
                 -4: "TM_ENONFINITE", -5: "TM_ESTEP", -6: "TM_EBUSY", -7: "TM_ENOTFOUND"}

# every symbol the header declares
EXPORTS = [
    "tm_last_error", "tm_version", "tm_measure_peaks", "tm_init", "tm_finalize", "tm_set_memory_budget",
    "tm_geometry_create", "tm_geometry_hash", "tm_geometry_info", "tm_geometry_destroy",
    "tm_tensor_assemble", "tm_tensor_threshold", "tm_tensor_sparse_info", "tm_tensor_sparse_get",
    "tm_tensor_get", "tm_tensor_rows", "tm_tensor_bytes", "tm_tensor_release",
    "tm_problem_create", "tm_problem_destroy", "tm_demag", "tm_demag_noalloc", "tm_heff", "tm_dmdt", "tm_energy",
    "tm_diagnostics",
    "tm_run", "tm_profile_run", "tm_profile_field", "tm_profile_field_mode", "tm_num_shapes", "tm_shape_info",
    "tm_problem_shape", "tm_problem_set_shape",
    "tm_problem_tune", "tm_problem_apply", "tm_tune_cache_save", "tm_tune_cache_load", "tm_tune_cache_clear",
    "tm_tune_cache_size", "tm_server_create", "tm_server_submit", "tm_server_poll", "tm_server_destroy",
]


class TilemagError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_STATUS_NAMES.get(status, str(status)), msg))
        self.status = status


class tm_material(C.Structure):
    _fields_ = [("Ms", C.POINTER(C.c_double)), ("A_exch", C.c_double),
                ("Ku", C.POINTER(C.c_double)), ("easy", C.POINTER(C.c_double)),
                ("alpha", C.c_double), ("gamma0", C.c_double), ("ll_form", C.c_int32)]


class tm_run_cfg(C.Structure):
    _fields_ = [("max_steps", C.c_int64), ("max_attempts", C.c_int64), ("t_end", C.c_double),
                ("atol", C.c_double), ("rtol", C.c_double), ("dt_min", C.c_double),
                ("dmdt_stop", C.c_double), ("renorm", C.c_int32), ("use_graph", C.c_int32),
                ("poll_every", C.c_int32), ("persistent", C.c_int32)]


class tm_run_stats(C.Structure):
    _fields_ = [("attempts", C.c_int64), ("accepted_min", C.c_int64), ("accepted_max", C.c_int64),
                ("rejected", C.c_int64), ("states_done", C.c_int32), ("states_failed", C.c_int32),
                ("elapsed_ms", C.c_double)]


class tm_server_cfg(C.Structure):
    _fields_ = [("memory_budget", C.c_int64), ("max_slots", C.c_int32), ("max_groups", C.c_int32),
                ("steps_per_round", C.c_int32), ("prec", C.c_int32), ("max_active", C.c_int32)]


class tm_request(C.Structure):
    _fields_ = [("n", C.c_int64), ("centers", C.POINTER(C.c_double)),
                ("sizes", C.POINTER(C.c_double)), ("mat", tm_material), ("Ha", C.c_double * 3),
                ("m0", C.POINTER(C.c_float)), ("dt0", C.c_double), ("atol", C.c_double),
                ("rtol", C.c_double), ("dmdt_stop", C.c_double), ("max_steps", C.c_int64)]


class tm_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("steps", C.c_int64), ("t", C.c_double),
                ("latency_ms", C.c_double), ("cache_hit", C.c_int32)]


_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libtilemag.so not found at %s; build it with "
                          "`python -m paper_2107_05364_amd.build`" % path)
    # torch ships its own HIP runtime under the same soname; importing torch
    # first makes the library bind to that runtime, so that torch's device
    # memory and stream handles belong to the runtime the library calls
    import torch  # noqa: F401

    L = C.CDLL(path)
    runtimes = _mapped_hip_runtimes()
    if len(runtimes) > 1:
        raise ImportError("two HIP runtimes are mapped in this process (%s); import torch "
                          "before anything else loads libamdhip64" % ", ".join(sorted(runtimes)))
    vp, i32, i64, u64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
    P = C.POINTER
    sig = {
        "tm_last_error": (C.c_char_p, []),
        "tm_version": (i32, []),
        "tm_measure_peaks": (i32, [i32, i64, P(d), P(d), P(d)]),
        "tm_init": (i32, [i32, P(vp)]),
        "tm_finalize": (i32, [vp]),
        "tm_set_memory_budget": (i32, [vp, i64]),
        "tm_geometry_create": (i32, [vp, i64, P(d), P(d), P(vp)]),
        "tm_geometry_hash": (i32, [vp, P(u64)]),
        "tm_geometry_info": (i32, [vp, P(i64), P(i64)]),
        "tm_geometry_destroy": (i32, [vp]),
        "tm_tensor_assemble": (i32, [vp, vp, i32, i32, vp, P(vp)]),
        "tm_tensor_threshold": (i32, [vp, vp, d, vp, P(vp)]),
        "tm_tensor_sparse_info": (i32, [vp, P(i64), P(d)]),
        "tm_tensor_sparse_get": (i32, [vp, P(i64), P(i32), P(C.c_float)]),
        "tm_tensor_get": (i32, [vp, i64, i64, P(d)]),
        "tm_tensor_rows": (i32, [vp, i64, i64, P(d)]),
        "tm_tensor_bytes": (i32, [vp, P(i64)]),
        "tm_tensor_release": (i32, [vp]),
        "tm_problem_create": (i32, [vp, vp, vp, P(tm_material), P(vp)]),
        "tm_problem_destroy": (i32, [vp]),
        "tm_demag": (i32, [vp, i64, vp, vp, vp]),
        "tm_demag_noalloc": (i32, [vp, i64, vp, vp, vp]),
        "tm_heff": (i32, [vp, i64, vp, vp, vp, vp]),
        "tm_dmdt": (i32, [vp, i64, vp, vp, vp, vp]),
        "tm_energy": (i32, [vp, i64, vp, vp, vp, vp]),
        "tm_diagnostics": (i32, [vp, i64, vp, vp, vp, vp]),
        "tm_run": (i32, [vp, i32, i64, vp, vp, vp, vp, vp, P(tm_run_cfg), P(tm_run_stats), vp]),
        "tm_profile_run": (i32, [vp, i32, i64, vp, vp, vp, vp, P(tm_run_cfg), P(d), P(i64), vp]),
        "tm_profile_field": (i32, [vp, i64, i32, vp, P(d), P(i64)]),
        "tm_profile_field_mode": (i32, [vp, i64, i32, i32, vp, P(d), P(i64)]),
        "tm_num_shapes": (i32, []),
        "tm_shape_info": (i32, [i32, P(i32), P(i32), P(i32), P(i32)]),
        "tm_problem_shape": (i32, [vp, P(i32)]),
        "tm_problem_set_shape": (i32, [vp, i32]),
        "tm_problem_tune": (i32, [vp, i64, i32, vp, P(i32), P(d)]),
        "tm_problem_apply": (i32, [vp, i32]),
        "tm_tune_cache_save": (i32, [C.c_char_p]),
        "tm_tune_cache_load": (i32, [C.c_char_p]),
        "tm_tune_cache_clear": (i32, []),
        "tm_tune_cache_size": (i32, [P(i64)]),
        "tm_server_create": (i32, [vp, P(tm_server_cfg), P(vp)]),
        "tm_server_submit": (i32, [vp, P(tm_request), P(u64)]),
        "tm_server_poll": (i32, [vp, u64, i32, P(tm_result), P(C.c_float)]),
        "tm_server_destroy": (i32, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _mapped_hip_runtimes() -> set:
    try:
        with open("/proc/self/maps") as f:
            return {ln.split()[-1] for ln in f if "libamdhip64" in ln}
    except OSError:
        return set()


def tm_last_error() -> str:
    return load().tm_last_error().decode()


def tm_version() -> int:
    return int(load().tm_version())


def tm_measure_peaks(device: int = 0, read_bytes: int = 2 << 30):
    """(stream read GB/s, bf16 32x32x16 MFMA TFLOP/s, fp32 16x16x4 MFMA TFLOP/s)."""
    r, b, f = C.c_double(), C.c_double(), C.c_double()
    _check(load().tm_measure_peaks(int(device), int(read_bytes), C.byref(r), C.byref(b), C.byref(f)))
    return r.value, b.value, f.value


last_error = tm_last_error


def _check(status: int) -> int:
    if status != TM_OK:
        raise TilemagError(status, last_error())
    return status


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _stream():
    import torch

    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype=None, name="tensor"):
    """Device pointer of a contiguous torch tensor on the GPU (or None)."""
    if t is None:
        return None
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a torch tensor on the GPU" % name)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return C.c_void_p(t.data_ptr())


# ----------------------------------------------------------------- C names

def tm_init(device: int = 0) -> C.c_void_p:
    out = C.c_void_p()
    _check(load().tm_init(device, C.byref(out)))
    return out


def tm_finalize(ctx) -> None:
    _check(load().tm_finalize(ctx))


def tm_set_memory_budget(ctx, nbytes: int) -> None:
    _check(load().tm_set_memory_budget(ctx, int(nbytes)))


def tm_geometry_create(ctx, centers, sizes) -> C.c_void_p:
    c, s = _f64(centers), _f64(sizes)
    if c.ndim != 2 or c.shape[1] != 3 or s.shape != c.shape:
        raise ValueError("centers and sizes must both be [n, 3]")
    out = C.c_void_p()
    _check(load().tm_geometry_create(ctx, c.shape[0], _dp(c), _dp(s), C.byref(out)))
    return out


def tm_geometry_hash(g) -> int:
    h = C.c_uint64()
    _check(load().tm_geometry_hash(g, C.byref(h)))
    return h.value


def tm_geometry_info(g):
    n, nf = C.c_int64(), C.c_int64()
    _check(load().tm_geometry_info(g, C.byref(n), C.byref(nf)))
    return n.value, nf.value


def tm_geometry_destroy(g) -> None:
    _check(load().tm_geometry_destroy(g))


def tm_tensor_assemble(ctx, g, store=TM_PREC_FP32, layout=TM_LAYOUT_SYM6) -> C.c_void_p:
    out = C.c_void_p()
    _check(load().tm_tensor_assemble(ctx, g, int(store), int(layout), _stream(), C.byref(out)))
    return out


def tm_tensor_threshold(ctx, T, frac: float) -> C.c_void_p:
    out = C.c_void_p()
    _check(load().tm_tensor_threshold(ctx, T, C.c_double(float(frac)), _stream(), C.byref(out)))
    return out


def tm_tensor_sparse_info(T):
    """(stored blocks, magnitude cut or -1)."""
    nb, cut = C.c_int64(), C.c_double()
    _check(load().tm_tensor_sparse_info(T, C.byref(nb), C.byref(cut)))
    return nb.value, cut.value


def tm_tensor_sparse_get(T, n: int):
    """(row_ptr int64 [n+1], col int32 [nnzb], vals float32 [6, nnzb])."""
    nnzb, _ = tm_tensor_sparse_info(T)
    rp = np.zeros(n + 1, np.int64)
    col = np.zeros(max(nnzb, 1), np.int32)
    vals = np.zeros((6, max(nnzb, 1)), np.float32)
    _check(load().tm_tensor_sparse_get(T, rp.ctypes.data_as(C.POINTER(C.c_int64)),
                                       col.ctypes.data_as(C.POINTER(C.c_int32)),
                                       vals.ctypes.data_as(C.POINTER(C.c_float))))
    return rp, col[:nnzb], vals[:, :nnzb]


def tm_tensor_get(T, a: int, b: int) -> np.ndarray:
    out = np.zeros(9)
    _check(load().tm_tensor_get(T, int(a), int(b), _dp(out)))
    return out.reshape(3, 3)


def tm_tensor_rows(T, n: int, a0: int, count: int) -> np.ndarray:
    """Blocks of target tiles [a0, a0+count) as float64 [count, n, 3, 3]."""
    out = np.zeros((count, n, 9))
    _check(load().tm_tensor_rows(T, int(a0), int(count), _dp(out)))
    return out.reshape(count, n, 3, 3)


def tm_tensor_bytes(T) -> int:
    v = C.c_int64()
    _check(load().tm_tensor_bytes(T, C.byref(v)))
    return v.value


def tm_tensor_release(T) -> None:
    _check(load().tm_tensor_release(T))


def make_material(n, Ms, A_exch, alpha, gamma0=2.21e5, ll_form=0, Ku=None, easy=None):
    """(tm_material, keep-alive arrays) for n tiles."""
    ms = _f64(np.broadcast_to(np.asarray(Ms, np.float64), (n,)))
    keep = [ms]
    ku_p = eas_p = None
    if Ku is not None:
        ku = _f64(np.broadcast_to(np.asarray(Ku, np.float64), (n,)))
        ea = _f64(np.broadcast_to(np.asarray(easy, np.float64), (n, 3)))
        keep += [ku, ea]
        ku_p, eas_p = _dp(ku), _dp(ea)
    mat = tm_material(_dp(ms), float(A_exch), ku_p, eas_p, float(alpha), float(gamma0), int(ll_form))
    return mat, keep


def tm_problem_create(ctx, g, T, mat: tm_material) -> C.c_void_p:
    out = C.c_void_p()
    _check(load().tm_problem_create(ctx, g, T, C.byref(mat), C.byref(out)))
    return out


def tm_problem_destroy(p) -> None:
    _check(load().tm_problem_destroy(p))


def _batch(m, n):
    if m.dim() != 3 or m.shape[1] != n or m.shape[2] != 3:
        raise ValueError("state must be [B, %d, 3], got %s" % (n, tuple(m.shape)))
    return m.shape[0]


def _shape(t, shape, name):
    """The kernels index device buffers by B and n: check every shape here."""
    if t is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))


def tm_demag(p, n, m, Hd) -> None:
    import torch

    B = _batch(m, n)
    _shape(Hd, m.shape, "Hd")
    _check(load().tm_demag(p, B, _dev(m, torch.float32, "m"), _dev(Hd, torch.float32, "Hd"), _stream()))


def tm_demag_noalloc(p, n, m, Hd, check=True) -> int:
    """tm_demag on the library's fixed scratch buffer (allocates nothing)."""
    import torch

    B = _batch(m, n)
    _shape(Hd, m.shape, "Hd")
    r = load().tm_demag_noalloc(p, B, _dev(m, torch.float32, "m"), _dev(Hd, torch.float32, "Hd"), _stream())
    if check:
        _check(r)
    return r


def tm_heff(p, n, m, Ha, H) -> None:
    import torch

    B = _batch(m, n)
    _shape(Ha, (B, 3), "Ha")
    _shape(H, m.shape, "H")
    _check(load().tm_heff(p, B, _dev(m, torch.float32, "m"), _dev(Ha, torch.float32, "Ha"),
                          _dev(H, torch.float32, "H"), _stream()))


def tm_dmdt(p, n, m, Ha, out) -> None:
    import torch

    B = _batch(m, n)
    _shape(Ha, (B, 3), "Ha")
    _shape(out, m.shape, "dmdt")
    _check(load().tm_dmdt(p, B, _dev(m, torch.float32, "m"), _dev(Ha, torch.float32, "Ha"),
                          _dev(out, torch.float32, "dmdt"), _stream()))


def tm_energy(p, n, m, Ha, E) -> None:
    import torch

    B = _batch(m, n)
    _shape(Ha, (B, 3), "Ha")
    _shape(E, (B, 4), "E")
    _check(load().tm_energy(p, B, _dev(m, torch.float32, "m"), _dev(Ha, torch.float32, "Ha"),
                            _dev(E, torch.float64, "E"), _stream()))


def tm_diagnostics(p, n, m, Ha, D) -> None:
    import torch

    B = _batch(m, n)
    _shape(Ha, (B, 3), "Ha")
    _shape(D, (B, 9), "D")
    _check(load().tm_diagnostics(p, B, _dev(m, torch.float32, "m"), _dev(Ha, torch.float32, "Ha"),
                                 _dev(D, torch.float64, "D"), _stream()))


def tm_run(p, n, integ, m, Ha, t, dt, steps_out, cfg: tm_run_cfg, check=True) -> tm_run_stats:
    import torch

    B = _batch(m, n)
    _shape(Ha, (B, 3), "Ha")
    _shape(t, (B,), "t")
    _shape(dt, (B,), "dt")
    _shape(steps_out, (B,), "steps")
    st = tm_run_stats()
    r = load().tm_run(p, int(integ), B, _dev(m, torch.float32, "m"), _dev(Ha, torch.float32, "Ha"),
                      _dev(t, torch.float64, "t"), _dev(dt, torch.float64, "dt"),
                      _dev(steps_out, torch.int64, "steps"), C.byref(cfg), C.byref(st), _stream())
    if check:
        _check(r)
    st.status = r
    return st


def tm_profile_run(p, n, integ, m, Ha, t, dt, cfg: tm_run_cfg):
    """(summed operator-pass duration [ms], operator-pass launches) of
    cfg.max_attempts attempted steps integrated in place."""
    import torch

    B = _batch(m, n)
    _shape(Ha, (B, 3), "Ha")
    _shape(t, (B,), "t")
    _shape(dt, (B,), "dt")
    ms, cnt = C.c_double(), C.c_int64()
    _check(load().tm_profile_run(p, int(integ), B, _dev(m, torch.float32, "m"), _dev(Ha, torch.float32, "Ha"),
                                 _dev(t, torch.float64, "t"), _dev(dt, torch.float64, "dt"), C.byref(cfg),
                                 C.byref(ms), C.byref(cnt), _stream()))
    return ms.value, cnt.value


def tm_profile_field(p, B: int, iters: int):
    """(mean ms per launch of the fused stage kernel, algorithmic bytes per launch)."""
    ms, nb = C.c_double(), C.c_int64()
    _check(load().tm_profile_field(p, int(B), int(iters), _stream(), C.byref(ms), C.byref(nb)))
    return ms.value, nb.value


def tm_profile_field_mode(p, B: int, mode: int, iters: int):
    ms, nb = C.c_double(), C.c_int64()
    _check(load().tm_profile_field_mode(p, int(B), int(mode), int(iters), _stream(), C.byref(ms),
                                        C.byref(nb)))
    return ms.value, nb.value


def tm_num_shapes() -> int:
    return int(load().tm_num_shapes())


def tm_shape_info(shape: int):
    """(threads per workgroup, target tiles per workgroup, nontemporal, waves cap)."""
    v = [C.c_int32() for _ in range(4)]
    _check(load().tm_shape_info(int(shape), *[C.byref(x) for x in v]))
    return tuple(x.value for x in v)


def tm_problem_shape(p) -> int:
    v = C.c_int32()
    _check(load().tm_problem_shape(p, C.byref(v)))
    return v.value


def tm_problem_set_shape(p, shape: int) -> None:
    _check(load().tm_problem_set_shape(p, int(shape)))


def tm_problem_tune(p, B: int = 1, iters: int = 20):
    """(chosen candidate, its mean ms per launch); iters < 0 times even when
    the autotuner's table holds a result for this key."""
    ch, ms = C.c_int32(), C.c_double()
    _check(load().tm_problem_tune(p, int(B), int(iters), _stream(), C.byref(ch), C.byref(ms)))
    return ch.value, ms.value


def tm_problem_apply(p, choice: int) -> None:
    """Applies a choice as tm_problem_tune reports it, without timing."""
    _check(load().tm_problem_apply(p, int(choice)))


def tm_tune_cache_save(path: str) -> None:
    _check(load().tm_tune_cache_save(os.fsencode(path)))


def tm_tune_cache_load(path: str) -> int:
    """Merges a saved table; returns the status (TM_ENOTFOUND if the file is missing)."""
    r = load().tm_tune_cache_load(os.fsencode(path))
    if r not in (TM_OK, TM_ENOTFOUND):
        _check(r)
    return r


def tm_tune_cache_clear() -> None:
    _check(load().tm_tune_cache_clear())


def tm_tune_cache_size() -> int:
    n = C.c_int64()
    _check(load().tm_tune_cache_size(C.byref(n)))
    return n.value


# ------------------------------------------------------------ convenience

class Context:
    """A device context (tensor cache + admission budget)."""

    def __init__(self, device: int = 0):
        self.handle = tm_init(device)
        self.device = device

    def close(self):
        if self.handle:
            tm_finalize(self.handle)
            self.handle = None

    def set_memory_budget(self, nbytes: int):
        tm_set_memory_budget(self.handle, nbytes)


class Geometry:
    def __init__(self, ctx, centers, sizes):
        self.centers, self.sizes = _f64(centers), _f64(sizes)
        self.n = self.centers.shape[0]
        self.handle = tm_geometry_create(None if ctx is None else ctx.handle, self.centers,
                                         self.sizes)

    @property
    def hash(self) -> int:
        return tm_geometry_hash(self.handle)

    @property
    def nfaces(self) -> int:
        return tm_geometry_info(self.handle)[1]

    def close(self):
        if self.handle:
            tm_geometry_destroy(self.handle)
            self.handle = None


class Tensor:
    def __init__(self, ctx: Context, geom: Geometry, store=TM_PREC_FP32, layout=TM_LAYOUT_SYM6):
        self.handle = tm_tensor_assemble(ctx.handle, geom.handle, store, layout)
        self.store, self.layout, self.n = store, layout, geom.n
        self.ctx = ctx

    def threshold(self, frac: float) -> "Tensor":
        """Thresholded copy (BSR6) of this FP32 SYM6 operator (paper Sec. 4.3.1)."""
        t = Tensor.__new__(Tensor)
        t.handle = tm_tensor_threshold(self.ctx.handle, self.handle, frac)
        t.store, t.layout, t.n, t.ctx = TM_PREC_FP32, TM_LAYOUT_BSR6, self.n, self.ctx
        return t

    def sparse(self):
        """(row_ptr, col, vals) of a BSR6 operator on the host."""
        return tm_tensor_sparse_get(self.handle, self.n)

    @property
    def nnzb(self) -> int:
        return tm_tensor_sparse_info(self.handle)[0]

    @property
    def cut(self) -> float:
        return tm_tensor_sparse_info(self.handle)[1]

    def block(self, a: int, b: int) -> np.ndarray:
        return tm_tensor_get(self.handle, a, b)

    def rows(self, a0: int, count: int) -> np.ndarray:
        return tm_tensor_rows(self.handle, self.n, a0, count)

    def dense(self) -> np.ndarray:
        """The whole operator as a float64 [3n, 3n] matrix (blocking)."""
        r = self.rows(0, self.n)
        return r.transpose(0, 2, 1, 3).reshape(3 * self.n, 3 * self.n)

    @property
    def nbytes(self) -> int:
        return tm_tensor_bytes(self.handle)

    def close(self):
        if self.handle:
            tm_tensor_release(self.handle)
            self.handle = None


class Problem:
    """Geometry + operator + material; field, right-hand side, energy and
    time integration of B states that share the operator."""

    def __init__(self, ctx: Context, geom: Geometry, tensor: Tensor, Ms, A_exch, alpha,
                 gamma0=2.21e5, ll_form=0, Ku=None, easy=None):
        self.n = geom.n
        mat, keep = make_material(self.n, Ms, A_exch, alpha, gamma0, ll_form, Ku, easy)
        self.handle = tm_problem_create(ctx.handle, geom.handle, tensor.handle, mat)
        self._keep = keep

    def _like(self, m):
        import torch

        return torch.empty_like(m)

    def demag(self, m):
        out = self._like(m)
        tm_demag(self.handle, self.n, m, out)
        return out

    def heff(self, m, Ha=None):
        out = self._like(m)
        tm_heff(self.handle, self.n, m, Ha, out)
        return out

    def dmdt(self, m, Ha=None):
        out = self._like(m)
        tm_dmdt(self.handle, self.n, m, Ha, out)
        return out

    def energy(self, m, Ha=None):
        import torch

        E = torch.empty((m.shape[0], 4), dtype=torch.float64, device=m.device)
        tm_energy(self.handle, self.n, m, Ha, E)
        return E

    def diagnostics(self, m, Ha=None):
        """[B, 9] float64: energy terms, <m>, max |dm/dt|, non-finite flag."""
        import torch

        D = torch.empty((m.shape[0], 9), dtype=torch.float64, device=m.device)
        tm_diagnostics(self.handle, self.n, m, Ha, D)
        return D

    def run(self, m, Ha=None, integ=TM_DP45, dt=1e-14, t=None, max_steps=1, max_attempts=0,
            atol=1e-6, rtol=1e-6, t_end=0.0, dt_min=0.0, dmdt_stop=0.0, renorm=True,
            use_graph=True, poll_every=64, check=True, persistent=False):
        """Integrates the states in place; returns (t, dt, steps, stats)."""
        import torch

        B = m.shape[0]
        dev = m.device
        tt = torch.zeros(B, dtype=torch.float64, device=dev) if t is None else t
        if isinstance(dt, torch.Tensor):
            dd = dt
        else:
            dd = torch.full((B,), float(dt), dtype=torch.float64, device=dev)
        steps = torch.zeros(B, dtype=torch.int64, device=dev)
        cfg = tm_run_cfg(int(max_steps), int(max_attempts), float(t_end), float(atol), float(rtol),
                         float(dt_min), float(dmdt_stop), int(bool(renorm)), int(bool(use_graph)),
                         int(poll_every), int(bool(persistent)))
        st = tm_run(self.handle, self.n, integ, m, Ha, tt, dd, steps, cfg, check=check)
        return tt, dd, steps, st

    def close(self):
        if self.handle:
            tm_problem_destroy(self.handle)
            self.handle = None


def tm_server_create(ctx, memory_budget=0, max_slots=8, max_groups=16, steps_per_round=64,
                     prec=TM_PREC_FP32, max_active=0) -> C.c_void_p:
    cfg = tm_server_cfg(int(memory_budget), int(max_slots), int(max_groups), int(steps_per_round),
                        int(prec), int(max_active))
    out = C.c_void_p()
    _check(load().tm_server_create(ctx, C.byref(cfg), C.byref(out)))
    return out


def tm_server_submit(srv, centers, sizes, m0, Ha, Ms, A_exch, alpha, gamma0=2.21e5, ll_form=0,
                     dt0=1e-14, atol=1e-6, rtol=1e-6, dmdt_stop=0.0, max_steps=100000, Ku=None,
                     easy=None) -> int:
    c, s = _f64(centers), _f64(sizes)
    n = c.shape[0]
    m = np.ascontiguousarray(np.asarray(m0, np.float32).reshape(n, 3))
    mat, keep = make_material(n, Ms, A_exch, alpha, gamma0, ll_form, Ku, easy)
    req = tm_request(n, _dp(c), _dp(s), mat, (C.c_double * 3)(*[float(v) for v in Ha]),
                     m.ctypes.data_as(C.POINTER(C.c_float)), float(dt0), float(atol), float(rtol),
                     float(dmdt_stop), int(max_steps))
    tk = C.c_uint64()
    _check(load().tm_server_submit(srv, C.byref(req), C.byref(tk)))
    del keep
    return tk.value


def tm_server_poll(srv, ticket: int, n: int = 0, wait: bool = True):
    """(tm_result, final state [n, 3] or None)."""
    res = tm_result()
    out = np.zeros((n, 3), np.float32) if n else None
    ptr = out.ctypes.data_as(C.POINTER(C.c_float)) if n else None
    _check(load().tm_server_poll(srv, C.c_uint64(ticket), int(bool(wait)), C.byref(res), ptr))
    return res, out


def tm_server_destroy(srv) -> None:
    _check(load().tm_server_destroy(srv))


class Server:
    """Continuous-batching server of LLG relaxation requests on one device."""

    def __init__(self, ctx: Context, memory_budget=0, max_slots=8, max_groups=16,
                 steps_per_round=64, max_active=0):
        self.handle = tm_server_create(ctx.handle, memory_budget, max_slots, max_groups,
                                       steps_per_round, max_active=max_active)
        self._n = {}

    def submit(self, centers, sizes, m0, Ha, **kw) -> int:
        tk = tm_server_submit(self.handle, centers, sizes, m0, Ha, **kw)
        self._n[tk] = np.asarray(centers).shape[0]
        return tk

    def poll(self, ticket: int, wait: bool = True):
        return tm_server_poll(self.handle, ticket, self._n[ticket], wait)

    def close(self):
        if self.handle:
            tm_server_destroy(self.handle)
            self.handle = None

