"""Seeded synthetic inputs (tile meshes, initial states, applied fields).

This module only *generates inputs*; it holds none of the method's arithmetic
and is shared by the tests, the benchmark and the FP64 oracle checks so that
both sides of every comparison see the same arrays.

Random numbers come from one counter-based generator, splitmix64: draw ``i``
of stream ``seed`` is ``mix(seed * 0x9E3779B97F4A7C15 + (i+1) * 0x9E3779B97F4A7C15)``
with the splitmix64 finaliser; the top 53 bits give a uniform in [0, 1).
Normals use Box-Muller on two consecutive uniforms; random unit vectors are
normalised Gaussian triples.

Geometry follows the paper's workloads: Cartesian meshes of cuboid tiles
(paper Sec. 3), the thin film of standard problem 4 (Sec. 4.3: 500 x 125 x 3 nm,
one tile thick, A = 1.3e-11 J/m, Ms = 8.0e5 A/m), and a seeded non-uniform
refinement of a slab.  All lengths are in metres, fields in A/m.
"""
from __future__ import annotations

import heapq
import math
from dataclasses import dataclass, field

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
MU0 = 4.0e-7 * math.pi          # only to state inputs: mT -> A/m, the energy density Km of problem 3
GAMMA0 = 2.21e5                 # gyromagnetic constant of standard problem 4 [m/(A s)]
NM = 1e-9


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def uniform(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """``count`` uniforms in [0, 1) from stream ``seed`` starting at draw ``offset``."""
    with np.errstate(over="ignore"):
        base = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) * _GOLDEN
        idx = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
        z = _mix(base + idx * _GOLDEN)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def normal(seed: int, count: int) -> np.ndarray:
    u = uniform(seed, 2 * count).reshape(count, 2)
    r = np.sqrt(-2.0 * np.log1p(-u[:, 0]))
    return r * np.cos(2.0 * math.pi * u[:, 1])


def random_unit_vectors(seed: int, n: int) -> np.ndarray:
    g = normal(seed, 3 * n).reshape(n, 3)
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def grid(nx: int, ny: int, nz: int, dx: float, dy: float, dz: float, origin=(0.0, 0.0, 0.0)):
    """Cartesian mesh of identical cuboids, x fastest: a = ix + nx (iy + ny iz)."""
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    c = np.stack([(ix.ravel() + 0.5) * dx, (iy.ravel() + 0.5) * dy, (iz.ravel() + 0.5) * dz], axis=1)
    c = c + np.asarray(origin, dtype=np.float64)
    s = np.tile([dx, dy, dz], (c.shape[0], 1)).astype(np.float64)
    return np.ascontiguousarray(c), np.ascontiguousarray(s)


@dataclass
class Workload:
    name: str
    centers: np.ndarray          # [n, 3] m
    sizes: np.ndarray            # [n, 3] full edges, m
    m0: np.ndarray               # [B, n, 3] unit vectors
    Ha: np.ndarray               # [B, 3] applied field, A/m
    Ms: float = 8.0e5
    A: float = 1.3e-11
    alpha: float = 0.5
    gamma0: float = GAMMA0
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.centers.shape[0]

    @property
    def batch(self) -> int:
        return self.m0.shape[0]


def cube_grid(seed: int = 0, n_side: int = 8, edge: float = 5 * NM) -> Workload:
    """Regular n_side^3 grid of cubic tiles, random unit m0, zero field
    (plain-method FP64 configuration: 8 x 8 x 8 cubes of 5 nm)."""
    c, s = grid(n_side, n_side, n_side, edge, edge, edge)
    m0 = random_unit_vectors(seed, c.shape[0])[None]
    return Workload("cube_grid_%d" % n_side, c, s, m0, np.zeros((1, 3)), alpha=0.5,
                    extra={"dt": 1e-13, "steps": 200})


def film_texture(centers: np.ndarray, length: float, seed: int, theta_e_deg: float = 30.0,
                 ell: float = 50 * NM, noise_deg: float = 5.0) -> np.ndarray:
    """Near-saturated in-plane texture of a film along x: in-plane angle
    theta(x) = theta_e (exp(-x/ell) + exp(-(L-x)/ell)) from +x, plus per-tile
    uniform in-plane noise and out-of-plane tilt of +-noise_deg."""
    n = centers.shape[0]
    x = centers[:, 0]
    th = math.radians(theta_e_deg) * (np.exp(-x / ell) + np.exp(-(length - x) / ell))
    u = uniform(seed, 2 * n).reshape(n, 2)
    th = th + math.radians(noise_deg) * (2.0 * u[:, 0] - 1.0)
    ph = math.radians(noise_deg) * (2.0 * u[:, 1] - 1.0)
    return np.stack([np.cos(ph) * np.cos(th), np.cos(ph) * np.sin(th), np.sin(ph)], axis=1)


def thin_film(nx: int = 100, ny: int = 25, seed_m: int = 0, seed_h: int = 1) -> Workload:
    """Standard-problem-4 film, 500 x 125 x 3 nm, one tile thick (5 x 5 x 3 nm
    tiles at nx = 100), alpha = 0.02; seeded in-plane field of 10-50 mT."""
    L, W, t = 500 * NM, 125 * NM, 3 * NM
    c, s = grid(nx, ny, 1, L / nx, W / ny, t)
    m0 = film_texture(c, L, seed_m)[None]
    u = uniform(seed_h, 2)
    ang = 2.0 * math.pi * u[0]
    b = (10.0 + 40.0 * u[1]) * 1e-3 / MU0
    Ha = np.array([[b * math.cos(ang), b * math.sin(ang), 0.0]])
    return Workload("thin_film_%dx%dx1" % (nx, ny), c, s, m0, Ha, alpha=0.02,
                    extra={"steps": 20000, "dt0": 1e-14, "atol": 1e-6, "rtol": 1e-6})


def sp3_cube(n: int, lam: float, Ms: float = 8.0e5, edge: float = 20 * NM) -> Workload:
    """Standard problem 3 (paper Sec. 4.2): a cube of edge L = lam * l_ex cut
    into n^3 cubic tiles, with l_ex = sqrt(A / Km), Km = mu0 Ms^2 / 2 and a
    uniaxial anisotropy Ku = 0.1 Km along z.  The edge is held at `edge` and
    A = Km (edge / lam)^2 sets L / l_ex = lam (the demag tensor depends only on
    shape, so one geometry serves every lam).  Two starting states:
    m0[0] flower start, uniform along the easy axis; m0[1] vortex start,
    circulating in the y-z planes about the x axis through the cube's centre
    (the vortex axis perpendicular to the easy axis), tilting toward +x near
    the axis.  Relaxation is pure damping (LL with c1 = 0, c2 = gamma0)."""
    Km = 0.5 * MU0 * Ms * Ms
    A = Km * (edge / lam) ** 2
    c, s = grid(n, n, n, edge / n, edge / n, edge / n)
    flower = np.tile([0.0, 0.0, 1.0], (c.shape[0], 1))
    y, z = c[:, 1] - 0.5 * edge, c[:, 2] - 0.5 * edge
    v = np.stack([np.full_like(y, 0.1 * edge), -z, y], axis=1)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return Workload("sp3_cube_n%d_L%.3f" % (n, lam), c, s, np.stack([flower, v]), np.zeros((2, 3)),
                    Ms=Ms, A=A, alpha=GAMMA0, gamma0=0.0,
                    extra={"Ku": 0.1 * Km, "easy": np.array([0.0, 0.0, 1.0]), "Km": Km, "lam": lam,
                           "ll_form": 1, "volume": edge ** 3, "dmdt_stop": 1e-4 * GAMMA0 * Ms})


# Standard problem 4 (paper Sec. 4.3): the s-state is prepared by saturating
# along [1, 1, 1] and removing that field slowly; here a staircase of fields
# along [1, 1, 1] (mT), each level relaxed by pure damping (LL with c1 = 0,
# c2 = gamma0) until max_a |dm/dt|_a < SP4_RELAX_STOP.  The dynamics then use
# the paper's LL parameters (ll_form 1: c1 = gamma = 2.21e5, c2 = alpha = 4.42e3)
# under field 1 or field 2, switched on at t = 0, for SP4_DYN_TIME.
SP4_LEVELS_MT = (1000.0, 300.0, 100.0, 30.0, 10.0, 3.0, 0.0)
SP4_RELAX_STOP = 1e-4 * GAMMA0 * 8.0e5
SP4_FIELDS_MT = {1: (-24.6, 4.3, 0.0), 2: (-35.5, -6.3, 0.0)}
SP4_DYN_TIME = 1e-9


def sp4_film(n: int) -> Workload:
    """Standard-problem-4 film at resolution [20n, 5n, 1] (tiles of
    25/n x 25/n x 3 nm), Ms = 8.0e5 A/m, A = 1.3e-11 J/m, starting saturated
    along [1, 1, 1].  extra: the s-state staircase (applied fields [A/m] per
    level), the relaxation LL parameters, the dynamics LL parameters and the
    two reversal fields [A/m]."""
    c, s = grid(20 * n, 5 * n, 1, 25 * NM / n, 25 * NM / n, 3 * NM)
    d = np.ones(3) / math.sqrt(3.0)
    m0 = np.tile(d, (c.shape[0], 1))[None]
    levels = [d * (b * 1e-3 / MU0) for b in SP4_LEVELS_MT]
    fields = {k: np.array(v) * 1e-3 / MU0 for k, v in SP4_FIELDS_MT.items()}
    return Workload("sp4_film_n%d" % n, c, s, m0, np.zeros((1, 3)), Ms=8.0e5, A=1.3e-11,
                    alpha=4.42e3, gamma0=GAMMA0,
                    extra={"n": n, "levels": levels, "relax_stop": SP4_RELAX_STOP,
                           "relax_ll": (0.0, GAMMA0),  # (c1, c2): pure damping
                           "dyn_ll": (GAMMA0, 4.42e3), "ll_form": 1, "fields": fields,
                           "dyn_time": SP4_DYN_TIME})


def hysteresis_batch(B: int = 128, nx: int = 100, ny: int = 25, seed_axis: int = 2) -> Workload:
    """B independent states on the film geometry: fields evenly spaced from
    +80 mT to -80 mT along one seeded in-plane axis; state k starts from the
    film texture with noise stream k."""
    L, W, t = 500 * NM, 125 * NM, 3 * NM
    c, s = grid(nx, ny, 1, L / nx, W / ny, t)
    ang = 2.0 * math.pi * uniform(seed_axis, 1)[0]
    axis = np.array([math.cos(ang), math.sin(ang), 0.0])
    b = np.linspace(80e-3, -80e-3, B) / MU0
    Ha = b[:, None] * axis[None, :]
    m0 = np.stack([film_texture(c, L, k) for k in range(B)])
    return Workload("hysteresis_film_B%d" % B, c, s, m0, Ha, alpha=0.02, extra={"axis": axis})


def refined_slab(n_target: int = 20000, seed: int = 4, seed_m: int = 0, B: int = 1,
                 lx=1000 * NM, ly=250 * NM, lz=20 * NM, root=(20 * NM, 10 * NM, 20 * NM),
                 min_edge=5 * NM, jitter=2 * NM) -> Workload:
    """Seeded adaptive refinement of a slab: start from a grid of root cuboids
    and repeatedly halve the tile of highest priority along its longest edge
    (ties x, y, z) while that edge >= min_edge; priority is minus the distance
    of the tile centre to the nearest lateral face plus a uniform jitter in
    [0, jitter) (one draw per tile, in creation order); priority ties go to the
    lowest index.  Stops at exactly n_target tiles.  Tiles are finally sorted
    by (z, y, x) of their centres."""
    nx, ny, nz = int(round(lx / root[0])), int(round(ly / root[1])), int(round(lz / root[2]))
    c, s = grid(nx, ny, nz, *root)
    cs = [list(v) for v in c]
    ss = [list(v) for v in s]
    draws = iter(uniform(seed, 4 * n_target + 16))

    def prio(i):
        x, y = cs[i][0], cs[i][1]
        return -min(x, lx - x, y, ly - y) + jitter * next(draws)

    heap = [(-prio(i), i) for i in range(len(cs))]
    heapq.heapify(heap)
    while len(cs) < n_target and heap:
        _, i = heapq.heappop(heap)
        e = ss[i]
        d = int(np.argmax(e))  # first maximal edge: x before y before z
        if e[d] < min_edge * (1 - 1e-12):
            continue
        half = 0.5 * e[d]
        lo = list(cs[i]); hi = list(cs[i])
        lo[d] -= 0.5 * half; hi[d] += 0.5 * half
        sz = list(e); sz[d] = half
        cs[i] = lo; ss[i] = sz
        cs.append(hi); ss.append(list(sz))
        j = len(cs) - 1
        heapq.heappush(heap, (-prio(i), i))
        heapq.heappush(heap, (-prio(j), j))
    c = np.array(cs); s = np.array(ss)
    order = np.lexsort((c[:, 0], c[:, 1], c[:, 2]))
    c = np.ascontiguousarray(c[order]); s = np.ascontiguousarray(s[order])
    m0 = np.stack([random_unit_vectors(seed_m + k, c.shape[0]) for k in range(B)])
    return Workload("refined_slab_%d" % c.shape[0], c, s, m0, np.zeros((B, 3)), alpha=0.1,
                    extra={"steps": 5000})


@dataclass
class Request:
    arrival: float               # s since stream start
    centers: np.ndarray
    sizes: np.ndarray
    m0: np.ndarray               # [n, 3]
    Ha: np.ndarray               # [3] A/m
    repeat_of: int               # index of the earlier request whose geometry is reused, or -1


def serving_stream(count: int = 200, rate: float = 20.0, seed: int = 5, n_min: int = 500,
                   n_max: int = 20000, repeat_frac: float = 0.3) -> list:
    """Poisson arrivals of relaxation requests on grids of 5 x 5 x 3 nm tiles
    with a log-uniform tile count and a seeded aspect ratio; about
    ``repeat_frac`` of the requests reuse an earlier request's geometry."""
    u = uniform(seed, 8 * count).reshape(count, 8)
    t = np.cumsum(-np.log1p(-u[:, 0]) / rate)
    reqs = []
    for k in range(count):
        rep = -1
        if k > 0 and u[k, 1] < repeat_frac:
            rep = int(u[k, 2] * k)
            while reqs[rep].repeat_of >= 0:
                rep = reqs[rep].repeat_of
            c, s = reqs[rep].centers, reqs[rep].sizes
        else:
            ntile = math.exp(math.log(n_min) + (math.log(n_max) - math.log(n_min)) * u[k, 3])
            nz = 1 if u[k, 4] < 0.7 else 2
            aspect = 1.0 + 3.0 * u[k, 5]
            ny = max(1, int(round(math.sqrt(ntile / (nz * aspect)))))
            nx = max(1, int(round(ntile / (nz * ny))))
            c, s = grid(nx, ny, nz, 5 * NM, 5 * NM, 3 * NM)
        ang = 2.0 * math.pi * u[k, 6]
        b = 50e-3 * u[k, 7] / MU0
        Ha = np.array([b * math.cos(ang), b * math.sin(ang), 0.0])
        m0 = random_unit_vectors(1000 + k, c.shape[0])
        reqs.append(Request(float(t[k]), c, s, m0, Ha, rep))
    return reqs
