"""Seeded synthetic inputs: meshes, advecting-field descriptors, initial data.

This module is shared by the CPU oracle's tests and the GPU path's tests and
benchmark.  It holds no part of the method itself (no foot tracking, no point
location, no interpolation, no mesh adjacency): it only draws node coordinates,
triangle vertex lists, field *descriptors* (a kind plus parameters; each side
evaluates the field with its own code) and nodal values of analytic initial
data.

The paper runs on Delaunay meshes from an external generator, on the square
with a rotating field (Section 4).  Those meshes are not available, so the
workloads below are jittered or graded structured grids of the same sizes
and shapes; the triangle numbering of a cell follows the paper's Courant grid
(two triangles per cell, Section 4, direct location on a structured grid),
0-based.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field as dc_field

import numpy as np

# Field kinds.  The numeric codes are part of the C interface of both sides.
FIELD_CONSTANT = 0     # f = (p0, p1)
FIELD_SOLID_BODY = 1   # f = p0 * (-(y - p2), x - p1)
FIELD_SWIRL = 2        # f = cos(pi t / p0) (sin^2(pi x) sin(2 pi y), -sin^2(pi y) sin(2 pi x))
FIELD_PAPER_ROT = 3    # f = (cos(p0 |x - c| + p1 t), sin(p0 |x - c| + p1 t)), c = (p2, p3)
FIELD_AFFINE = 4       # f = [[p0, p1], [p2, p3]] (x - (p4, p5)) + (p6, p7)

SCHEME_EULER = 0
SCHEME_RK2 = 1


@dataclass
class Field:
    """An advecting field f(x, t) given by kind and up to 8 parameters."""
    kind: int
    p: tuple = ()

    def params8(self) -> np.ndarray:
        out = np.zeros(8, dtype=np.float64)
        out[: len(self.p)] = self.p
        return out


def solid_body(omega=2.0 * math.pi, cx=0.5, cy=0.5) -> Field:
    return Field(FIELD_SOLID_BODY, (omega, cx, cy))


def swirl(period=1.0) -> Field:
    return Field(FIELD_SWIRL, (period,))


def constant(ax, ay) -> Field:
    return Field(FIELD_CONSTANT, (ax, ay))


def paper_rot(c0=2.0 * math.pi, c1=2.0 * math.pi, cx=0.0, cy=0.0) -> Field:
    return Field(FIELD_PAPER_ROT, (c0, c1, cx, cy))


def affine(a11, a12, a21, a22, cx=0.0, cy=0.0, bx=0.0, by=0.0) -> Field:
    return Field(FIELD_AFFINE, (a11, a12, a21, a22, cx, cy, bx, by))


# ---------------------------------------------------------------------------
# Meshes
# ---------------------------------------------------------------------------

def grid_triangles(n: int) -> np.ndarray:
    """Triangles of an n x n node grid, node (l, m) -> m*n + l.

    Cell c = (n-1)*m + l is split by its diagonal (l,m)-(l+1,m+1):
    triangle 2c = (v00, v11, v01) lies above the diagonal and 2c+1 =
    (v00, v10, v11) below it, both counter-clockwise.
    """
    l, m = np.meshgrid(np.arange(n - 1), np.arange(n - 1), indexing="xy")
    l = l.ravel().astype(np.int64)
    m = m.ravel().astype(np.int64)
    v00 = m * n + l
    v10 = v00 + 1
    v01 = v00 + n
    v11 = v01 + 1
    tri = np.empty((2 * (n - 1) ** 2, 3), dtype=np.int32)
    tri[0::2] = np.stack([v00, v11, v01], axis=1)
    tri[1::2] = np.stack([v00, v10, v11], axis=1)
    return tri


def grid_nodes(n: int, x0=0.0, x1=1.0) -> np.ndarray:
    """Unjittered n x n nodes on [x0, x1]^2, row-major with x fastest."""
    s = np.linspace(x0, x1, n)
    # make the last coordinate exactly x1 and the grid exactly symmetric
    s[-1] = x1
    x, y = np.meshgrid(s, s, indexing="xy")
    return np.stack([x.ravel(), y.ravel()], axis=1).astype(np.float64)


def jittered_grid(n: int, seed: int, jitter: float = 0.2, x0=0.0, x1=1.0):
    """n x n grid on [x0,x1]^2 with interior nodes moved by U(-jitter*h, jitter*h).

    Boundary nodes move only along their boundary side and the four corners
    stay fixed, so the domain is exactly the square and every boundary edge
    lies on x or y in {x0, x1}.  With jitter <= 0.2 no triangle inverts (the
    largest displacement, 0.2*sqrt(2) h, is below half the smallest
    vertex-to-opposite-edge distance h/sqrt(2)).
    """
    xy = grid_nodes(n, x0, x1)
    h = (x1 - x0) / (n - 1)
    rng = np.random.default_rng(seed)
    d = rng.uniform(-jitter * h, jitter * h, size=xy.shape)
    l = np.tile(np.arange(n), n)
    m = np.repeat(np.arange(n), n)
    on_x = (l == 0) | (l == n - 1)
    on_y = (m == 0) | (m == n - 1)
    d[on_x, 0] = 0.0
    d[on_y, 1] = 0.0
    xy = xy + d
    return xy, grid_triangles(n)


def _drop_cells(xy: np.ndarray, tri: np.ndarray, n: int, keep_cell):
    """The triangles of the cells (l, m) with keep_cell(l, m) (grid_triangles
    numbering: triangles 2c, 2c + 1 of cell c = (n-1) m + l), the unused nodes
    removed and the rest renumbered in order."""
    c = np.arange(tri.shape[0]) // 2
    l, m = c % (n - 1), c // (n - 1)
    t = tri[keep_cell(l, m)]
    used = np.unique(t)
    new = np.full(xy.shape[0], -1, dtype=np.int64)
    new[used] = np.arange(used.size)
    return np.ascontiguousarray(xy[used]), new[t].astype(np.int32)


def l_shaped(n: int, seed: int, jitter: float = 0.2):
    """The unit square without its upper-right quarter (an L, one reflex
    corner at (1/2, 1/2)), from the jittered n x n grid (n odd); the nodes of
    the notch's sides keep the jitter of interior nodes."""
    xy, tri = jittered_grid(n, seed, jitter)
    half = (n - 1) // 2
    return _drop_cells(xy, tri, n, lambda l, m: ~((l >= half) & (m >= half)))


def square_with_hole(n: int, seed: int, jitter: float = 0.2):
    """The unit square without the square hole [3/8, 5/8]^2 (two boundary
    loops), from the jittered n x n grid (n - 1 divisible by 8)."""
    xy, tri = jittered_grid(n, seed, jitter)
    a, b = 3 * (n - 1) // 8, 5 * (n - 1) // 8
    return _drop_cells(xy, tri, n, lambda l, m: ~((l >= a) & (l < b) & (m >= a) & (m < b)))


def _graded_S(rho, rho0, A, delta):
    return rho + A * np.tanh((rho - rho0) / delta) + A * np.tanh(rho0 / delta)


def graded_grid(n: int, A: float = 0.4, ratio: float = 100.0):
    """n x n grid refined towards the circle of radius 1/4 about (1/2, 1/2).

    A computational point s has p = s - c, rho = 2 |p|_inf in [0, 1] and
    rho0 = |p|_inf / (2 |p|) (where the ray through p meets the circle).
    The physical radius psi solves S(psi) = rho with
    S(r) = [r + A tanh((r - rho0)/delta) + A tanh(rho0/delta)] / Z,
    Z chosen so S(1) = 1 and delta = A/(ratio-1), which makes the radial
    spacing near the circle `ratio` times finer than far from it.  The node is
    c + p * psi / rho.  Boundary nodes (rho = 1) stay fixed.
    """
    delta = A / (ratio - 1.0)
    s = grid_nodes(n)
    c = np.array([0.5, 0.5])
    p = s - c
    pinf = np.max(np.abs(p), axis=1)
    p2 = np.sqrt(np.sum(p * p, axis=1))
    rho = 2.0 * pinf
    center = pinf == 0.0
    rho0 = np.where(center, 0.5, 0.5 * pinf / np.where(center, 1.0, p2))
    Z = _graded_S(np.ones_like(rho0), rho0, A, delta)
    target = rho * Z
    lo = np.zeros_like(rho)
    hi = np.ones_like(rho)
    for _ in range(64):
        mid = 0.5 * (lo + hi)
        below = _graded_S(mid, rho0, A, delta) < target
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    psi = 0.5 * (lo + hi)
    psi = np.where(rho == 1.0, 1.0, psi)
    scale = np.where(center, 0.0, psi / np.where(center, 1.0, rho))
    xy = c + p * scale[:, None]
    # keep the boundary exact
    bnd = rho == 1.0
    xy[bnd] = s[bnd]
    tri = grid_triangles(n)
    a, b, cc = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    area2 = (b[:, 0] - a[:, 0]) * (cc[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (cc[:, 0] - a[:, 0])
    if not (area2 > 0).all():
        raise ValueError(f"graded grid folds at n={n} (needs n >= 81)")
    return xy, tri


def permute_mesh(xy: np.ndarray, tri: np.ndarray, seed: int):
    """Random relabelling of nodes and triangles (same geometry)."""
    rng = np.random.default_rng(seed)
    pn = rng.permutation(xy.shape[0])          # new id -> old id
    inv = np.empty_like(pn)
    inv[pn] = np.arange(pn.size)              # old id -> new id
    pt = rng.permutation(tri.shape[0])
    xy2 = xy[pn]
    tri2 = inv[tri[pt]].astype(np.int32)
    return xy2, tri2


def morton_order_mesh(xy: np.ndarray, tri: np.ndarray):
    """Relabel nodes and triangles in Z-order of node / centroid position.

    This is an input-order option of the workloads (a user who already
    stores the mesh sorted), independent of any reordering the library does.
    """
    def key(p):
        lo = p.min(axis=0)
        span = max(float((p.max(axis=0) - lo).max()), 1e-300)
        q = np.clip(((p - lo) / span * 65535.0).astype(np.int64), 0, 65535)
        k = np.zeros(p.shape[0], dtype=np.int64)
        for b in range(16):
            k |= ((q[:, 0] >> b) & 1) << (2 * b)
            k |= ((q[:, 1] >> b) & 1) << (2 * b + 1)
        return k
    pn = np.argsort(key(xy), kind="stable")
    inv = np.empty_like(pn)
    inv[pn] = np.arange(pn.size)
    tri2 = inv[tri].astype(np.int32)
    cen = xy[pn][tri2].mean(axis=1)
    pt = np.argsort(key(cen), kind="stable")
    return xy[pn], tri2[pt]


# ---------------------------------------------------------------------------
# Initial data
# ---------------------------------------------------------------------------

def gaussian_hill(xy: np.ndarray, cx=0.5, cy=0.75, sigma=0.05, amp=1.0) -> np.ndarray:
    d2 = (xy[:, 0] - cx) ** 2 + (xy[:, 1] - cy) ** 2
    return amp * np.exp(-d2 / (2.0 * sigma * sigma))


@dataclass
class Hills:
    cx: np.ndarray
    cy: np.ndarray
    sigma: np.ndarray
    amp: np.ndarray

    def values(self, xy: np.ndarray, dtype=np.float64) -> np.ndarray:
        """Node-major [n_points][K] values, one Gaussian hill per field."""
        out = np.empty((xy.shape[0], self.cx.size), dtype=np.float64)
        for k in range(self.cx.size):
            out[:, k] = gaussian_hill(xy, self.cx[k], self.cy[k], self.sigma[k], self.amp[k])
        return out.astype(dtype)


def random_hills(k: int, seed: int) -> Hills:
    rng = np.random.default_rng(seed)
    return Hills(cx=rng.uniform(0.15, 0.85, k), cy=rng.uniform(0.15, 0.85, k),
                 sigma=rng.uniform(0.02, 0.08, k), amp=rng.uniform(0.5, 1.0, k))


def linear_data(xy: np.ndarray, a=0.3, b=-1.7, c=0.25) -> np.ndarray:
    return a + b * xy[:, 0] + c * xy[:, 1]


def quadratic_data(xy: np.ndarray) -> np.ndarray:
    x, y = xy[:, 0], xy[:, 1]
    return 0.5 - 1.25 * x + 0.75 * y + 2.0 * x * x - 1.5 * x * y + 0.625 * y * y


# ---------------------------------------------------------------------------
# Workload recipes
# ---------------------------------------------------------------------------

def courant_dt(alpha: float, h: float, t_final: float = 1.0):
    """Largest dt <= alpha*h/max|f| (max|f| = 1) that divides t_final."""
    steps = int(math.ceil(t_final / (alpha * h) - 1e-12))
    return t_final / steps, steps


@dataclass
class Workload:
    name: str
    xy: np.ndarray
    tri: np.ndarray
    field: Field
    scheme: int
    dt: float
    steps: int
    v0: np.ndarray            # [N][K] initial nodal values (vertex DOFs)
    h: float
    extra: dict = dc_field(default_factory=dict)


def small_rotation(n: int = 33, seed: int = 1001) -> Workload:
    """33x33 jittered unit square (2048 triangles), solid-body rotation of a
    Gaussian hill, Euler feet, dt = 0.05, 20 steps (one full turn)."""
    xy, tri = jittered_grid(n, seed)
    v0 = gaussian_hill(xy)[:, None]
    return Workload("rotation_33x33_jittered", xy, tri, solid_body(), SCHEME_EULER,
                    0.05, 20, v0, 1.0 / (n - 1))


def swirl_500(alpha: float = 5.0, order: str = "random", seed: int = 1002,
              perm_seed: int = 2002, n: int = 500) -> Workload:
    """500x500 jittered unit square (498,002 triangles), time-dependent swirl
    with period 1, Courant number alpha; nodes and triangles in seeded random
    order or Morton order."""
    xy, tri = jittered_grid(n, seed)
    if order == "random":
        xy, tri = permute_mesh(xy, tri, perm_seed)
    elif order == "morton":
        xy, tri = morton_order_mesh(xy, tri)
    h = 1.0 / (n - 1)
    dt, steps = courant_dt(alpha, h)
    v0 = gaussian_hill(xy)[:, None]
    return Workload(f"swirl_{n}x{n}_jittered_{order}_a{alpha:g}", xy, tri, swirl(1.0),
                    SCHEME_EULER, dt, steps, v0, h, {"alpha": alpha})


def graded_swirl(alpha: float = 5.0, n: int = 1415, k_fields: int = 16,
                 hill_seed: int = 3003, steps: int = 50) -> Workload:
    """n x n grid graded towards the circle r = 1/4 (100x spacing ratio;
    n = 1415 gives 3,998,792 triangles), swirl with period 1, RK2 feet,
    Courant number alpha on the computational spacing 1/(n-1), K Gaussian
    hills sharing one location."""
    xy, tri = graded_grid(n)
    h = 1.0 / (n - 1)
    dt, _ = courant_dt(alpha, h)
    hills = random_hills(k_fields, hill_seed)
    v0 = hills.values(xy, np.float32)
    return Workload(f"graded_{n}x{n}_swirl_rk2_a{alpha:g}_K{k_fields}", xy, tri, swirl(1.0),
                    SCHEME_RK2, dt, steps, v0, h, {"alpha": alpha, "hills": hills})


def batch_meshes(count: int = 64, size_seed: int = 4004, period_seed: int = 4005,
                 tmin: float = 1e4, tmax: float = 5e5, alpha: float = 5.0):
    """Uneven batch: triangle counts log-uniform in [tmin, tmax], jittered
    grids with n = round(1 + sqrt(t/2)) nodes a side, swirl periods U[0.5, 2]."""
    rng = np.random.default_rng(size_seed)
    t = np.exp(rng.uniform(math.log(tmin), math.log(tmax), count))
    ns = np.rint(1.0 + np.sqrt(t / 2.0)).astype(int)
    periods = np.random.default_rng(period_seed).uniform(0.5, 2.0, count)
    out = []
    for k in range(count):
        xy, tri = jittered_grid(int(ns[k]), 4100 + k)
        h = 1.0 / (ns[k] - 1)
        dt = alpha * h
        out.append(Workload(f"batch_{k}_{ns[k]}", xy, tri, swirl(float(periods[k])), SCHEME_EULER,
                            dt, 100, gaussian_hill(xy)[:, None].astype(np.float32), h))
    return out


def random_points(m: int, seed: int, lo=-0.05, hi=1.05) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, size=(m, 2))
