"""CPU-side tests of the HIP library: it loads, exports every entry point the
header declares, and its host-side mesh validation accepts valid meshes and
rejects invalid ones with the documented status codes.  No kernel runs."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2104_09189_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def S():
    from paper_2104_09189_amd import slwalk
    return slwalk


def test_library_exports_every_declared_symbol(S):
    hdr = open(os.path.join(ROOT, "include", "slwalk.h")).read()
    declared = set(re.findall(r"\b(slw_[a-z0-9_]+)\s*\(", hdr))
    assert len(declared) >= 15
    lib = ctypes.CDLL(str(S.LIB_PATH))
    missing = [n for n in sorted(declared) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(S.EXPORTED) == declared


def test_status_strings(S):
    for code in range(11):
        assert S._lib.slw_status_string(code).decode()


def test_valid_meshes_pass(S):
    xy, tri = I.jittered_grid(33, 1001)
    info = S.slw_mesh_check(xy, tri, S.P2)
    assert info["n_nodes"] == 1089 and info["n_tris"] == 2048
    assert info["n_edges"] == 1089 + 2048 - 1
    assert info["n_dofs"] == 1089 + info["n_edges"]
    xy, tri = I.permute_mesh(*I.graded_grid(81), 3)
    assert S.slw_mesh_check(xy, tri)["n_tris"] == 2 * 80 * 80
    # clockwise triangles are accepted (flipped internally)
    tri2 = tri.copy()
    tri2[::2] = tri2[::2][:, [0, 2, 1]]
    S.slw_mesh_check(xy, tri2)


def _code(S, xy, tri, flags=0):
    try:
        S.slw_mesh_check(xy, tri, flags)
    except S.SlwError as e:
        return e.name
    return "SLW_OK"


def test_invalid_meshes_are_rejected(S):
    xy, tri = I.jittered_grid(6, 3)
    t = tri.copy()
    t[4, 1] = 999
    assert _code(S, xy, t) == "SLW_E_MESH_INDEX"
    t = tri.copy()
    t[4, 1] = t[4, 0]
    assert _code(S, xy, t) == "SLW_E_MESH_DEGENERATE"
    # zero-area triangle: three collinear nodes
    x2 = xy.copy()
    a, b, c = tri[7]
    x2[c] = 0.5 * (x2[a] + x2[b])
    assert _code(S, x2, tri) in ("SLW_E_MESH_DEGENERATE", "SLW_E_MESH_NONCONFORMING", "SLW_E_MESH_NONCONVEX")
    # an unused node
    x3 = np.concatenate([xy, [[0.5, 0.5]]])
    assert _code(S, x3, tri) == "SLW_E_MESH_DEGENERATE"
    # a triangle listed twice: an edge in more than two triangles
    assert _code(S, xy, np.concatenate([tri, tri[:1]])) == "SLW_E_MESH_NONCONFORMING"
    # a hole (one interior triangle removed) and a reflex corner (one corner
    # cell's triangle removed): accepted, marked non-convex
    n = 6
    hole = (n - 1) * 2 + 2
    info = S.slw_mesh_check(xy, np.delete(tri, [2 * hole], axis=0))
    assert info["nonconvex"] and info["boundary_loops"] == 2
    info = S.slw_mesh_check(xy, np.delete(tri, [1], axis=0))
    assert info["nonconvex"] and info["boundary_loops"] == 1
    assert not S.slw_mesh_check(xy, tri)["nonconvex"]
    # a boundary that passes twice through a node: two triangles meeting at a vertex only
    xb = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [-1.0, 0.0], [0.0, -1.0]])
    assert _code(S, xb, np.array([[0, 1, 2], [0, 3, 4]], np.int32)) == "SLW_E_MESH_NONCONVEX"
    # the L and the square with a hole of the input generators
    for xy2, tri2, loops in (I.l_shaped(17, 4) + (1,), I.square_with_hole(17, 5) + (2,)):
        info = S.slw_mesh_check(xy2, tri2)
        assert info["nonconvex"] and info["boundary_loops"] == loops
    # coordinates outside the exactness domain
    x4 = xy.copy()
    x4[0, 0] = np.nan
    assert _code(S, x4, tri) == "SLW_E_MESH_RANGE"
    x4 = xy.copy()
    x4[8, 0] = 1e-200
    assert _code(S, x4, tri) == "SLW_E_MESH_RANGE"
    assert _code(S, xy, tri, 0x100) == "SLW_E_ARG"
    assert _code(S, xy[:2], tri[:0]) == "SLW_E_ARG"


def test_context_on_a_missing_device_is_an_error(S):
    h = ctypes.c_void_p()
    rc = S._lib.slw_ctx_create(99, None, ctypes.byref(h))
    assert rc in (1, 7) and not h.value   # SLW_E_ARG, or SLW_E_HIP without a device
    assert S._lib.slw_ctx_create(0, None, None) == 1


def _predicate_cases(rng, m):
    """Triples (a, b) in the mesh exactness domain and any query c: random,
    near-collinear (rounded points of the line a-b, one-ulp nudges of exact
    lattice points), and queries with tiny or subnormal coordinates."""
    out = []
    for _ in range(m):
        kind = int(rng.integers(0, 5))
        a = rng.uniform(-1, 1, 2)
        b = rng.uniform(-1, 1, 2)
        if kind == 0:
            c = rng.uniform(-1, 1, 2)
        elif kind == 1:
            c = a + rng.uniform(-2, 3) * (b - a)
        elif kind == 2:
            s = 2.0 ** -int(rng.integers(0, 60))
            a = rng.integers(-50, 50, 2) * s
            d = rng.integers(-7, 8, 2) * s
            b = a + d
            c = (a + int(rng.integers(-5, 6)) * d).astype(float)
            i = int(rng.integers(0, 2))
            c[i] = np.nextafter(c[i], np.inf if rng.integers(0, 2) else -np.inf)
        elif kind == 3:
            # a vertical or horizontal edge through 0 and a query at a tiny offset
            t = rng.uniform(0.1, 0.9)
            a = np.array([0.0, rng.uniform(0.0, 0.4)])
            b = np.array([0.0, rng.uniform(0.6, 1.0)])
            tiny = float(rng.choice([5e-324, -5e-324, 1e-310, -1e-300, 1e-200, -2.0 ** -1000]))
            c = np.array([tiny, t])
            if rng.integers(0, 2):
                a, b, c = a[::-1].copy(), b[::-1].copy(), c[::-1].copy()
        else:
            # large coordinates at the top of the domain
            base = rng.uniform(-2.0 ** 90, 2.0 ** 90, 2)
            a = base + rng.uniform(-1e10, 1e10, 2)
            b = base + rng.uniform(-1e10, 1e10, 2)
            c = a + rng.uniform(-2, 3) * (b - a)
        out.append(np.concatenate([a, b, c]))
    return np.array(out)


def test_library_predicate_matches_oracle_exact_sign(S, orc):
    rng = np.random.default_rng(77)
    pts = _predicate_cases(rng, 40000)
    want = orc.orient_sign_batch(pts, use_filter=False)
    assert (S.slw_orient_sign_host(pts, 0) == want).all()
    assert (S.slw_orient_sign_host(pts, 1) == want).all()
    assert (want == 0).sum() > 1000 and (want != 0).sum() > 10000
    # float pipeline: exact on the inputs rounded to float
    p32 = pts.astype(np.float32).astype(np.float64)
    assert (S.slw_orient_sign_host(pts, 2) == orc.orient_sign_batch(p32, use_filter=False)).all()


def _filter_cases(rng, m, scale, h):
    """Walk-like triples: an edge a-b of length ~h somewhere in a box of
    half-width `scale` about 0.5, and a query q at distances from the edge's
    line that range from ~h down to zero (points exactly on the line, and
    points a few float ulps off it)."""
    c = np.array([0.5, 0.5])
    a = c + rng.uniform(-scale, scale, (m, 2))
    ang = rng.uniform(0, 2 * np.pi, m)
    b = a + h * np.stack([np.cos(ang), np.sin(ang)], axis=1)
    t = rng.uniform(-1.5, 2.5, m)[:, None]
    on = a + t * (b - a)
    nrm = np.stack([-np.sin(ang), np.cos(ang)], axis=1)
    off = h * 10.0 ** rng.uniform(-12, 0, m)[:, None] * rng.choice([-1.0, 1.0], (m, 1))
    q = on + off
    k = m // 4
    q[:k] = on[:k]                              # rounded points of the line (near-zero determinants)
    q[k:2 * k] = np.nextafter(on[k:2 * k], np.inf)
    return np.concatenate([a, b, q], axis=1)


def test_walk_float_filter_never_certifies_a_wrong_sign(S, orc):
    rng = np.random.default_rng(5)
    for scale, h in ((0.5, 7e-4), (0.5, 1.3e-5), (0.5, 0.05), (3.0e3, 2.0), (1e-3, 1e-6)):
        pts = _filter_cases(rng, 60000, scale, h)
        cmax = float(np.abs(pts - 0.5).max())
        got = S.slw_float_filter_host(pts, 0.5, 0.5, cmax)
        exact = orc.orient_sign_batch(pts, use_filter=False)
        cert = got != 2
        assert (got[cert] == exact[cert]).all(), (scale, h)
        # it does certify the larger offsets (the share shrinks as h/scale does)
        assert cert.mean() > 0.05, (scale, h, cert.mean())
    # float meshes: inputs already float, the plain static bound
    pts = _filter_cases(rng, 60000, 0.5, 7e-4).astype(np.float32).astype(np.float64)
    got = S.slw_float_filter_host(pts, 0.0, 0.0, 0.0, f32=True)
    exact = orc.orient_sign_batch(pts, use_filter=False)
    cert = got != 2
    assert (got[cert] == exact[cert]).all()
    assert cert.mean() > 0.1


def test_walk_float_filter_certifies_typical_walk_tests(S, orc):
    # queries uniformly around a triangle of size h: nearly always certified
    rng = np.random.default_rng(6)
    h = 1.0 / 1414
    a = rng.uniform(0, 1, (50000, 2))
    b = a + rng.uniform(-h, h, (50000, 2))
    q = a + rng.uniform(-3 * h, 3 * h, (50000, 2))
    pts = np.concatenate([a, b, q], axis=1)
    got = S.slw_float_filter_host(pts, 0.5, 0.5, 0.5)
    exact = orc.orient_sign_batch(pts, use_filter=False)
    cert = got != 2
    assert (got[cert] == exact[cert]).all()
    assert cert.mean() > 0.99, cert.mean()


def _decode_codes(words):
    """Neighbour codes of the walk records: code k in bits [21k, 21k + 21) of
    the 64-bit word hi:lo, two's complement."""
    w = words[:, 0].astype(np.uint64) | (words[:, 1].astype(np.uint64) << np.uint64(32))
    out = np.empty((words.shape[0], 3), dtype=np.int64)
    for k in range(3):
        c = ((w >> np.uint64(21 * k)) & np.uint64((1 << 21) - 1)).astype(np.int64)
        out[:, k] = np.where(c >= 1 << 20, c - (1 << 21), c)
    return out


@pytest.mark.parametrize("bits", [2, 5, 12, 21])
def test_walk_record_neighbour_codes(S, bits):
    # neighbour triples with every kind of offset: boundary, +-1, near the
    # code limits, far (escapes), the largest ids
    rng = np.random.default_rng(bits)
    n = 1 << 22
    t = np.concatenate([rng.integers(0, n, 20000), [0, 1, n - 1, n - 2, 1 << 20, (1 << 20) + 7]])
    t = np.unique(t)
    off = rng.choice([-1, 1, -(1 << 19), (1 << 19), -(1 << 20) + 1, (1 << 20) - 1, -(1 << 20), 1 << 20,
                      -(1 << bits - 1) + 1, (1 << bits - 1) - 1, -(1 << bits - 1), 1 << bits - 1, 3, -3],
                     size=(t.size, 3))
    nb = t[:, None] + off
    nb = np.where((nb < 0) | (nb >= n) | (rng.random(nb.shape) < 0.1), -1, nb)
    # triangles listed densely: ids 0..len-1 map to t via a full table
    full = -np.ones((n, 3), dtype=np.int64)
    full[t] = nb
    words = S.slw_walk_codes_host(full.astype(np.int32), bits)
    codes = _decode_codes(words)[t]
    lim = 1 << (bits - 1)
    d = nb - t[:, None]
    fits = (nb >= 0) & (d > -lim) & (d < lim)
    assert np.array_equal(codes == 0, nb < 0)
    assert np.array_equal(codes == -(1 << 20), (nb >= 0) & ~fits)
    assert np.array_equal(np.where(fits, t[:, None] + codes, -7), np.where(fits, nb, -7))
    assert np.all(words[:, 1] >> 31 == 0)
