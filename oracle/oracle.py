"""CPU oracle for the semi-Lagrangian foot-location + interpolation path.

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
benchmark's CPU-baseline leg are the only callers.  The GPU library never
imports, links or runs anything here, and this module imports nothing from
the GPU package (only its seeded input generators are shared, by the
callers).

Paper: Cacace & Ferretti, arXiv 2104.09189.  What is computed, and where it
is defined:

* feet: explicit Euler backward in time, eq. (eulero); the explicit
  midpoint rule as the higher-order ODE solver that Section 3 (before
  Algorithm 1) leaves open.
* location: the walk of Section 2.2 stops in a triangle where every
  barycentric coordinate is non-negative, i.e. a closed triangle containing
  the point.  The oracle returns that result by definition, without a walk:
  the smallest triangle id among all closed containers, decided with exact
  orientation signs; -1 (outside) when there is none.
* weights: eq. (barycoords) in double precision.
* values: P1 as in the Remark after eq. (barycoords), P2 with the standard
  quadratic Lagrange basis; one step of eq. (schema_trasp) / Algorithm 2.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_LIB_PATH = _HERE / "liborc.so"
_lib = None


def build(force: bool = True) -> Path:
    """Compile liborc.so with gcc (no FP contraction, OpenMP): the oracle
    (orc.c) and the paper's walk on the host (walk.c)."""
    if force or not _LIB_PATH.exists():
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", str(_LIB_PATH) + ".tmp",
               str(_HERE / "orc.c"), str(_HERE / "walk.c"), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(str(_LIB_PATH) + ".tmp", _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not _LIB_PATH.exists():
            build(force=False)
        L = ctypes.CDLL(str(_LIB_PATH))
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        i64 = ctypes.c_int64
        L.orc_orient_sign.restype = ctypes.c_int
        L.orc_orient_sign.argtypes = [ctypes.c_double] * 6
        L.orc_orient_sign_exact.restype = ctypes.c_int
        L.orc_orient_sign_exact.argtypes = [ctypes.c_double] * 6
        L.orc_orient_sign_batch.restype = None
        L.orc_orient_sign_batch.argtypes = [dp, i64, ctypes.POINTER(ctypes.c_int8), ctypes.c_int]
        L.orc_locate.restype = ctypes.c_int
        L.orc_locate.argtypes = [dp, i64, ip, i64, dp, i64, ip, dp, ctypes.c_int]
        L.orc_containers.restype = ctypes.c_int
        L.orc_containers.argtypes = [dp, i64, ip, i64, ctypes.c_double, ctypes.c_double, ip, ctypes.c_int]
        L.orc_field.restype = None
        L.orc_field.argtypes = [ctypes.c_int, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.orc_feet.restype = None
        L.orc_feet.argtypes = [dp, i64, ctypes.c_int, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp]
        L.orc_p2_edges.restype = i64
        L.orc_p2_edges.argtypes = [ip, i64, ip, ip]
        L.orc_interp.restype = None
        L.orc_interp.argtypes = [ctypes.c_int, ip, i64, ip, i64, ip, dp, i64, dp, ctypes.c_int,
                                 ctypes.c_double, dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# --------------------------------------------------------------------------
# predicates

def orient_sign(a, b, c) -> int:
    return lib().orc_orient_sign(float(a[0]), float(a[1]), float(b[0]), float(b[1]),
                                 float(c[0]), float(c[1]))


def orient_sign_exact(a, b, c) -> int:
    return lib().orc_orient_sign_exact(float(a[0]), float(a[1]), float(b[0]), float(b[1]),
                                       float(c[0]), float(c[1]))


def orient_sign_batch(pts: np.ndarray, use_filter: bool = True) -> np.ndarray:
    pts = _f64(pts).reshape(-1, 6)
    out = np.empty(pts.shape[0], dtype=np.int8)
    lib().orc_orient_sign_batch(_d(pts), pts.shape[0],
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), int(use_filter))
    return out


# --------------------------------------------------------------------------
# location

def locate(xy, tri, q, brute: bool = False):
    """(elem, bary): smallest-id closed container of each query, -1 outside."""
    xy, tri, q = _f64(xy), _i32(tri), _f64(q).reshape(-1, 2)
    m = q.shape[0]
    elem = np.empty(m, dtype=np.int32)
    bary = np.empty((m, 3), dtype=np.float64)
    rc = lib().orc_locate(_d(xy), xy.shape[0], _i(tri), tri.shape[0], _d(q), m, _i(elem), _d(bary),
                          int(brute))
    if rc != 0:
        raise ValueError("orc_locate: bad arguments")
    return elem, bary


def containers(xy, tri, q, cap: int = 64):
    xy, tri = _f64(xy), _i32(tri)
    out = np.empty(cap, dtype=np.int32)
    c = lib().orc_containers(_d(xy), xy.shape[0], _i(tri), tri.shape[0], float(q[0]), float(q[1]),
                             _i(out), cap)
    return out[: min(c, cap)].copy()


# --------------------------------------------------------------------------
# feet

def field(fld, x, y, t):
    out = np.empty(2, dtype=np.float64)
    p = _f64(fld.params8())
    lib().orc_field(int(fld.kind), _d(p), float(x), float(y), float(t), _d(out))
    return out


def feet(xy, fld, t_np1: float, dt: float, scheme: int) -> np.ndarray:
    xy = _f64(xy)
    out = np.empty_like(xy)
    p = _f64(fld.params8())
    lib().orc_feet(_d(xy), xy.shape[0], int(fld.kind), _d(p), float(t_np1), float(dt), int(scheme),
                   _d(out))
    return out


# --------------------------------------------------------------------------
# P2 degrees of freedom

class P2Dofs:
    """Vertices first (node ids), then edge midpoints in lexicographic
    (min, max) vertex-pair order."""

    def __init__(self, xy, tri):
        xy, tri = _f64(xy), _i32(tri)
        nt = tri.shape[0]
        edges = np.empty((max(3 * nt, 1), 2), dtype=np.int32)
        te = np.empty((nt, 3), dtype=np.int32)
        ne = lib().orc_p2_edges(_i(tri), nt, _i(edges), _i(te))
        self.n_vert = xy.shape[0]
        self.edges = edges[:ne].copy()
        self.tri_edges = te
        mid = (xy[self.edges[:, 0]] + xy[self.edges[:, 1]]) * 0.5
        self.xy = np.concatenate([xy, mid], axis=0)

    @property
    def ndof(self):
        return self.xy.shape[0]


def interp(order: int, tri, elem, bary, v, n_vert: int, tri_edges=None, outside_value: float = 0.0):
    tri, elem, bary = _i32(tri), _i32(elem), _f64(bary)
    v = _f64(v)
    if v.ndim == 1:
        v = v[:, None]
    k = v.shape[1]
    m = elem.shape[0]
    out = np.empty((m, k), dtype=np.float64)
    if tri_edges is None:
        tri_edges = np.zeros((tri.shape[0], 3), dtype=np.int32)
    tri_edges = _i32(tri_edges)
    lib().orc_interp(int(order), _i(tri), tri.shape[0], _i(tri_edges), int(n_vert), _i(elem), _d(bary),
                     m, _d(v), k, float(outside_value), _d(out))
    return out


# --------------------------------------------------------------------------
# variable step at the boundary (remark after eq. (eulero)): a characteristic
# that leaves the domain stops on the boundary, where Dirichlet data apply

def boundary_edges(xy, tri) -> np.ndarray:
    """Boundary edges (a, b), each directed with the domain on its left: the
    edges that belong to one triangle only, taken in that triangle's
    counter-clockwise order."""
    xy, t = _f64(xy), np.array(tri, dtype=np.int64)
    a, b, c = xy[t[:, 0]], xy[t[:, 1]], xy[t[:, 2]]
    cw = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]) < 0
    t[cw] = t[cw][:, [0, 2, 1]]
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    _, inv, cnt = np.unique(np.sort(e, axis=1), axis=0, return_inverse=True, return_counts=True)
    return e[cnt[inv.ravel()] == 1]


def boundary_crossing(xy, edges, x, q):
    """theta in [0, 1] such that p = x + theta (q - x) is where the segment
    from x (in the closed domain) to q leaves the domain, and p; found as the
    smallest parameter over every boundary edge that the segment crosses
    from inside to outside (edge parameter lambda in [0, 1]).  NaN where
    there is none."""
    xy, x, q = _f64(xy), _f64(x).reshape(-1, 2), _f64(q).reshape(-1, 2)
    A, B = xy[edges[:, 0]], xy[edges[:, 1]]
    e = B - A                                        # (nb, 2)
    w = q - x                                        # (m, 2)
    r = A[None, :, :] - x[:, None, :]                # (m, nb, 2)
    den = w[:, None, 0] * e[None, :, 1] - w[:, None, 1] * e[None, :, 0]     # w x e > 0: outwards
    with np.errstate(divide="ignore", invalid="ignore"):
        th = (r[..., 0] * e[None, :, 1] - r[..., 1] * e[None, :, 0]) / den
        la = (r[..., 0] * w[:, None, 1] - r[..., 1] * w[:, None, 0]) / den
    ok = (den > 0) & (la >= 0) & (la <= 1) & (th >= -1e-12) & (th <= 1 + 1e-12)
    th = np.where(ok, np.clip(th, 0.0, 1.0), np.inf)
    theta = th.min(axis=1)
    theta[~np.isfinite(theta)] = np.nan
    p = x + theta[:, None] * w
    return theta, p


def boundary_value(bc, px, py, t):
    """Dirichlet data: bc = (kind, params), kind 1 constant p0, kind 2
    p0 + p1 x + p2 y + p3 t."""
    kind, p = bc
    p = list(p) + [0.0] * (4 - len(p))
    if kind == 1:
        return np.full_like(px, p[0])
    return p[0] + p[1] * px + p[2] * py + p[3] * t


# --------------------------------------------------------------------------
# one step and a run of eq. (schema_trasp) / Algorithm 2

def sl_step(xy, tri, v, fld, t_n: float, dt: float, scheme: int, order: int = 1,
            p2: P2Dofs | None = None, outside_value: float = 0.0, q=None, bc=None):
    """v^{n+1}_i = I[V^n](X^Delta(x_i, t_{n+1}; t_n)); returns (v_new, q, elem, bary).

    For order 2, `p2` gives the DOFs; feet are taken at every DOF.  If q is
    given it replaces the computed feet (index parity on identical points).
    With boundary data bc = (kind, params), a DOF whose foot is outside the
    domain gets g(p, t_{n+1} - theta dt) at the point p where the segment
    from the DOF to its foot leaves the domain (for every field); else
    outside_value.
    """
    pts = xy if order == 1 else p2.xy
    if q is None:
        q = feet(pts, fld, t_n + dt, dt, scheme)
    elem, bary = locate(xy, tri, q)
    te = None if order == 1 else p2.tri_edges
    v_new = interp(order, tri, elem, bary, v, xy.shape[0], te, outside_value)
    if bc is not None and bc[0] != 0:
        out = np.nonzero((elem < 0) & np.isfinite(q).all(axis=1))[0]
        if out.size:
            theta, p = boundary_crossing(xy, boundary_edges(xy, tri), _f64(pts)[out], _f64(q)[out])
            g = boundary_value(bc, p[:, 0], p[:, 1], t_n + dt - theta * dt)
            hit = np.isfinite(theta)
            v_new[out[hit]] = g[hit][:, None]
    return v_new, q, elem, bary


def sl_run(xy, tri, v0, fld, dt: float, steps: int, scheme: int, order: int = 1,
           p2: P2Dofs | None = None, outside_value: float = 0.0, t0: float = 0.0):
    v = _f64(v0)
    if v.ndim == 1:
        v = v[:, None]
    for n in range(steps):
        v, _, _, _ = sl_step(xy, tri, v, fld, t0 + n * dt, dt, scheme, order, p2, outside_value)
    return v
