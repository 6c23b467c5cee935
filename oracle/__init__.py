"""FP64 CPU oracle for the tile micromagnetics hot path (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It wraps ``oracle.c`` (plain C, FP64)
through ctypes and shares nothing with the HIP library.

Physics follows Bjork et al., "MagTense: a micromagnetic framework using the
analytical demagnetization tensor" (JMMM 2021): the Landau-Lifshitz equation
(Sec. 2.1), the four effective-field terms (Sec. 2.3), the tile discretisation
with the analytical cuboid tensor evaluated at tile centres (Sec. 3) and the
affine effective-field operator integrated with an explicit Runge-Kutta (4,5)
pair (Sec. 3.1).  Readings of points the paper leaves open are listed in the
repository's design notes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
MU0 = 4.0e-7 * np.pi

_lib = None


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (FP64, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        d = C.POINTER(C.c_double)
        i64 = C.c_int64
        L.orc_prism_tensor.argtypes = [d, d, d, d]
        L.orc_assemble.argtypes = [i64, d, d, d]
        L.orc_demag.argtypes = [i64, d, d, d, d]
        L.orc_demag_rows.argtypes = [i64, d, d, d, d, i64, C.POINTER(i64), d]
        L.orc_threshold.argtypes = [i64, d, C.c_double]
        L.orc_threshold.restype = C.c_double
        L.orc_faces.argtypes = [i64, d, d, i64, C.POINTER(i64), C.POINTER(i64), d, d]
        L.orc_faces.restype = i64
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        P = C.POINTER(_Problem)
        L.orc_heff.argtypes = [P, d, d, d]
        L.orc_ll_rhs.argtypes = [P, d, d, d, d]
        L.orc_rk4_step.argtypes = [P, d, d, C.c_double, C.c_int]
        L.orc_dp45_attempt.argtypes = [P, d, d, d, d, d, C.c_double, C.c_double, C.c_int,
                                       C.c_double, d, d]
        L.orc_dp45_attempt.restype = C.c_int
        L.orc_energy.argtypes = [P, d, d, d]
        _lib = L
    return _lib


class _Problem(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("T", C.POINTER(C.c_double)),
        ("vol", C.POINTER(C.c_double)),
        ("Ms", C.POINTER(C.c_double)),
        ("A", C.c_double),
        ("Ku", C.POINTER(C.c_double)),
        ("easy", C.POINTER(C.c_double)),
        ("nfaces", C.c_int64),
        ("fa", C.POINTER(C.c_int64)),
        ("fb", C.POINTER(C.c_int64)),
        ("area", C.POINTER(C.c_double)),
        ("dist", C.POINTER(C.c_double)),
        ("c1", C.c_double),
        ("c2", C.c_double),
    ]


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def set_num_threads(n: int) -> None:
    """Threads of the oracle's outer loops from now on (for timing)."""
    lib().orc_set_num_threads(int(n))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def prism_tensor(r, c, s) -> np.ndarray:
    """Tensor of the cuboid (centre c, full edges s) at point r; returns the
    symmetric 3x3 matrix N so that the tile's field is H = -N M."""
    r, c, s = _f64(r), _f64(c), _f64(s)
    out = np.zeros(6)
    lib().orc_prism_tensor(_p(r), _p(c), _p(s), _p(out))
    xx, xy, xz, yy, yz, zz = out
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


def assemble(centers, sizes) -> np.ndarray:
    """Dense [3n, 3n] FP64 demag operator; block (a, b) is tile b's tensor at
    the centre of tile a (paper Sec. 3)."""
    centers, sizes = _f64(centers), _f64(sizes)
    n = centers.shape[0]
    T = np.empty((3 * n, 3 * n))
    lib().orc_assemble(n, _p(centers), _p(sizes), _p(T))
    return T


def demag(T, Ms, m) -> np.ndarray:
    """H_d = -N (Ms m) for m of shape [n, 3]; returns [n, 3] in A/m."""
    m = _f64(m)
    n = m.shape[0]
    Ms = _f64(np.broadcast_to(Ms, (n,)))
    T = _f64(T)
    out = np.empty((n, 3))
    lib().orc_demag(n, _p(T), _p(Ms), _p(m), _p(out))
    return out


ZERO_FLOOR = 1e-14  # magnitudes at or below this (as float32) count as zero when thresholding


def threshold(T, frac: float):
    """Copy of the dense operator with the smallest ``frac`` of its nonzero
    entries (float32 magnitudes above ZERO_FLOOR, ties at the cut included)
    set to zero and self blocks kept (paper Sec. 4.3.1); returns (operator,
    cut), cut = -1 when nothing is removed."""
    if not 0.0 <= frac <= 1.0:
        raise ValueError("threshold fraction must lie in [0, 1]")
    out = np.array(T, dtype=np.float64, order="C", copy=True)
    n = out.shape[0] // 3
    cut = lib().orc_threshold(n, _p(out), float(frac))
    return out, float(cut)


def demag_rows(centers, sizes, Ms, m, rows) -> np.ndarray:
    """H_d at the target tiles ``rows`` only, tensor evaluated on the fly."""
    centers, sizes, m = _f64(centers), _f64(sizes), _f64(m)
    n = centers.shape[0]
    Ms = _f64(np.broadcast_to(Ms, (n,)))
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    out = np.empty((rows.shape[0], 3))
    lib().orc_demag_rows(n, _p(centers), _p(sizes), _p(Ms), _p(m), rows.shape[0],
                         rows.ctypes.data_as(C.POINTER(C.c_int64)), _p(out))
    return out


def faces(centers, sizes):
    """Ordered face pairs (a, b, shared area, centre distance along the normal)."""
    centers, sizes = _f64(centers), _f64(sizes)
    n = centers.shape[0]
    L = lib()
    cnt = L.orc_faces(n, _p(centers), _p(sizes), 0, None, None, None, None)
    fa = np.zeros(cnt, np.int64)
    fb = np.zeros(cnt, np.int64)
    area = np.zeros(cnt)
    dist = np.zeros(cnt)
    i64p = C.POINTER(C.c_int64)
    L.orc_faces(n, _p(centers), _p(sizes), cnt, fa.ctypes.data_as(i64p), fb.ctypes.data_as(i64p),
                _p(area), _p(dist))
    return fa, fb, area, dist


def ll_coefficients(alpha: float, gamma0: float, ll_form: int = 0):
    """(c1, c2) of dm/dt = -c1 m x H - c2 m x (m x H).

    ll_form 0: alpha is the dimensionless Gilbert damping,
               c1 = gamma0/(1+alpha^2), c2 = gamma0 alpha/(1+alpha^2);
    ll_form 1: (gamma0, alpha) are the paper's LL parameters, used as is."""
    if ll_form == 1:
        return float(gamma0), float(alpha)
    return gamma0 / (1.0 + alpha * alpha), gamma0 * alpha / (1.0 + alpha * alpha)


class Problem:
    """A tiled magnet with material data; holds the FP64 operator and faces."""

    def __init__(self, centers, sizes, Ms, A, alpha, gamma0=2.21e5, ll_form=0, Ku=None,
                 easy=None, T=None):
        self.centers = _f64(centers)
        self.sizes = _f64(sizes)
        n = self.n = self.centers.shape[0]
        self.Ms = _f64(np.broadcast_to(Ms, (n,)))
        self.A = float(A)
        self.Ku = _f64(np.zeros(n) if Ku is None else np.broadcast_to(Ku, (n,)))
        if easy is None:
            easy = np.tile([0.0, 0.0, 1.0], (n, 1))
        self.easy = _f64(np.broadcast_to(easy, (n, 3)))
        self.vol = _f64(np.prod(self.sizes, axis=1))
        self.T = assemble(self.centers, self.sizes) if T is None else _f64(T)
        self.fa, self.fb, self.area, self.dist = faces(self.centers, self.sizes)
        self.c1, self.c2 = ll_coefficients(alpha, gamma0, ll_form)
        i64p = C.POINTER(C.c_int64)
        self._s = _Problem(n, _p(self.T), _p(self.vol), _p(self.Ms), self.A, _p(self.Ku),
                           _p(self.easy), self.fa.shape[0], self.fa.ctypes.data_as(i64p),
                           self.fb.ctypes.data_as(i64p), _p(self.area), _p(self.dist),
                           self.c1, self.c2)

    def heff(self, m, Ha=(0.0, 0.0, 0.0)) -> np.ndarray:
        m, Ha = _f64(m), _f64(Ha)
        H = np.empty((self.n, 3))
        lib().orc_heff(C.byref(self._s), _p(m), _p(Ha), _p(H))
        return H

    def demag(self, m) -> np.ndarray:
        return demag(self.T, self.Ms, m)

    def rhs(self, m, Ha=(0.0, 0.0, 0.0)) -> np.ndarray:
        m, Ha = _f64(m), _f64(Ha)
        out = np.empty((self.n, 3))
        hb = np.empty((self.n, 3))
        lib().orc_ll_rhs(C.byref(self._s), _p(m), _p(Ha), _p(out), _p(hb))
        return out

    def rk4(self, m, Ha, dt, steps, renorm=True) -> np.ndarray:
        y = _f64(m).copy()
        Ha = _f64(Ha)
        for _ in range(steps):
            lib().orc_rk4_step(C.byref(self._s), _p(y), _p(Ha), float(dt), int(renorm))
        return y

    def dp45_attempt(self, m, k1, Ha, dt, t, atol=1e-6, rtol=1e-6, renorm=True, t_end=0.0):
        """One attempted adaptive step; m and k1 are updated in place on
        acceptance.  Returns (accepted, dt_next, t, err, max|dm/dt|)."""
        Ha = _f64(Ha)
        dtp = C.c_double(dt)
        tp = C.c_double(t)
        err = C.c_double(0.0)
        dmx = C.c_double(0.0)
        acc = lib().orc_dp45_attempt(C.byref(self._s), _p(m), _p(k1), _p(Ha), C.byref(dtp),
                                     C.byref(tp), atol, rtol, int(renorm), t_end, C.byref(err),
                                     C.byref(dmx))
        return bool(acc), dtp.value, tp.value, err.value, dmx.value

    def dp45(self, m, Ha, dt0, steps, atol=1e-6, rtol=1e-6, renorm=True, max_attempts=None):
        """Integrate until ``steps`` accepted steps; returns (m, t, dt, attempts)."""
        y = _f64(m).copy()
        k1 = self.rhs(y, Ha)
        dt, t, acc_n, att = float(dt0), 0.0, 0, 0
        while acc_n < steps:
            ok, dt, t, _, _ = self.dp45_attempt(y, k1, Ha, dt, t, atol, rtol, renorm)
            acc_n += int(ok)
            att += 1
            if max_attempts is not None and att >= max_attempts:
                break
        return y, t, dt, att

    def diagnostics(self, m, Ha=(0.0, 0.0, 0.0)) -> np.ndarray:
        """[E_demag, E_ex, E_anis, E_Z, <m>_x, <m>_y, <m>_z, max_a |dm/dt|_a,
        non-finite flag]: the energy terms, the moment-weighted mean
        magnetisation sum V Ms m / sum V Ms, and the largest LL right-hand
        side (Sec. 2.1-2.3)."""
        m = _f64(m)
        bad = not np.isfinite(m).all()
        out = np.zeros(9)
        with np.errstate(all="ignore"):
            out[:4] = self.energy(m, Ha)
            w = self.vol * self.Ms
            out[4:7] = (w[:, None] * m).sum(axis=0) / w.sum()
            k = self.rhs(m, Ha)
            bad = bad or not np.isfinite(k).all()
            out[7] = 0.0 if bad else np.sqrt((k * k).sum(axis=1)).max()
        out[8] = 1.0 if bad else 0.0
        return out

    def energy(self, m, Ha=(0.0, 0.0, 0.0)) -> np.ndarray:
        """[demag, exchange, anisotropy, Zeeman] energies in J."""
        m, Ha = _f64(m), _f64(Ha)
        E = np.empty(4)
        lib().orc_energy(C.byref(self._s), _p(m), _p(Ha), _p(E))
        return E
