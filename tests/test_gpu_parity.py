"""Parity of the HIP path (through the C-ABI) with the CPU oracle.

Indices must match bit for bit on identical query points; values within
1e-12 (FP64 values) or 1e-5 (FP32 values) relative to max(|v_ref|, |V^n|_inf).
Feet computed on both sides agree bit for bit for polynomial fields (the
same IEEE operations in the same order, no contraction) and within a few
ulp for the trigonometric ones.
"""
import numpy as np
import pytest

from paper_2104_09189_amd import inputs as I
from gpu_util import ctx as _ctx, dev, host, rel_err

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module")
def S():
    from paper_2104_09189_amd import slwalk
    return slwalk


@pytest.fixture(scope="module")
def C(S):
    return _ctx()


def _queries(xy, tri, seed, m=4000):
    """Random points (some outside), every vertex, edge midpoints and
    points at 1/4 along edges: exercises interior, edge and vertex cases."""
    rng = np.random.default_rng(seed)
    a, b = xy[tri[:, 0]], xy[tri[:, 1]]
    q = [I.random_points(m, seed, -0.1, 1.1), xy, (a + b) * 0.5, a + 0.25 * (b - a),
         xy[tri].mean(axis=1)[rng.integers(0, tri.shape[0], 500)]]
    return np.concatenate(q)


@pytest.mark.parametrize("flags", [0, 0x4, 0x8])  # Morton (default), no reorder, internal order
def test_locate_bitexact_small(S, C, orc, flags):
    xy, tri = I.permute_mesh(*I.jittered_grid(33, 1001), 7)
    tri = tri.copy()
    tri[::5] = tri[::5][:, [0, 2, 1]]  # clockwise input triangles
    q = _queries(xy, tri, 3)
    mesh = S.Mesh(C, xy, tri, flags)
    elem, bary, steps = mesh.locate(dev(q), want_steps=True)
    e_ref, b_ref = orc.locate(xy, tri, q)
    e, b = host(elem), host(bary)
    assert (e == e_ref).all(), np.nonzero(e != e_ref)[0][:10]
    inside = e_ref >= 0
    assert np.abs(b[inside] - b_ref[inside]).max() < 1e-12
    assert np.isnan(b[~inside]).all()
    assert (~inside).sum() > 100 and inside.sum() > 5000


def test_locate_with_given_starts_is_start_independent(S, C, orc):
    xy, tri = I.jittered_grid(40, 5)
    q = _queries(xy, tri, 4, 2000)
    mesh = S.Mesh(C, xy, tri)
    e_ref, _ = orc.locate(xy, tri, q)
    rng = np.random.default_rng(1)
    for trial in range(3):
        start = rng.integers(0, tri.shape[0], q.shape[0]).astype(np.int32)
        elem, _, steps = mesh.locate(dev(q), start=dev(start), want_steps=True)
        assert (host(elem) == e_ref).all()
    # invalid start ids fall back to the bucket-grid start
    bad = np.full(q.shape[0], -5, dtype=np.int32)
    bad[::2] = tri.shape[0] + 7
    elem, _, _ = mesh.locate(dev(q), start=dev(bad))
    assert (host(elem) == e_ref).all()


def test_locate_fp32_mesh_bitexact_on_rounded_inputs(S, C, orc):
    xy, tri = I.jittered_grid(50, 11)
    q = _queries(xy, tri, 5).astype(np.float32)
    mesh = S.Mesh(C, xy, tri, S.COORDS_F32)
    elem, bary, _ = mesh.locate(dev(q))
    xy32 = xy.astype(np.float32).astype(np.float64)
    e_ref, b_ref = orc.locate(xy32, tri, q.astype(np.float64))
    e = host(elem)
    assert (e == e_ref).all()
    inside = e_ref >= 0
    assert np.abs(host(bary)[inside] - b_ref[inside]).max() < 1e-5


def test_locate_empty_and_degenerate_queries(S, C, orc):
    import torch
    xy, tri = I.jittered_grid(20, 2)
    mesh = S.Mesh(C, xy, tri)
    elem, bary, _ = mesh.locate(torch.empty((0, 2), dtype=torch.float64, device="cuda:0"))
    assert elem.numel() == 0
    q = np.array([[np.nan, 0.5], [0.5, np.inf], [-np.inf, -np.inf], [1e300, 0.5], [1e-300, 0.5],
                  [0.0, 0.0], [1.0, 1.0], [0.5, -1e-320]])
    elem, bary, _ = mesh.locate(dev(q))
    e = host(elem)
    e_ref, _ = orc.locate(xy, tri, q)
    assert e[:4].tolist() == [-1, -1, -1, -1]
    # tiny and subnormal query coordinates are decided exactly as well
    assert (e == e_ref).all()
    assert e_ref[7] == -1 and e_ref[4] >= 0


def test_locate_feet_given_feet_bitexact(S, C, orc):
    # swirl feet (trigonometric): computed once by the oracle, passed to both
    w = I.swirl_500(alpha=5.0, order="random", n=80)
    p2 = orc.P2Dofs(w.xy, w.tri)
    for flags, pts in ((0, w.xy), (S.P2, p2.xy)):
        mesh = S.Mesh(C, w.xy, w.tri, flags)
        feet = orc.feet(pts, w.field, 0.3 + w.dt, w.dt, I.SCHEME_RK2)
        out = mesh.locate_feet(feet=dev(feet), feet_in=True, want_steps=True, stats=True)
        e_ref, b_ref = orc.locate(w.xy, w.tri, feet)
        e = host(out["elem"])
        assert (e == e_ref).all()
        inside = e_ref >= 0
        assert np.abs(host(out["bary"])[inside] - b_ref[inside]).max() < 1e-12
        assert out["stats"]["feet"] == pts.shape[0]
        assert out["stats"]["outside"] == int((~inside).sum())


def test_feet_match_oracle(S, C, orc):
    w = I.swirl_500(alpha=5.0, order="morton", n=60)
    mesh = S.Mesh(C, w.xy, w.tri)
    for fld in (w.field, I.solid_body(), I.paper_rot(8.0, 2.0, 0.5, 0.5), I.affine(0.3, -1.1, 0.7, 0.2, 0.4, 0.6, 0.1, 0.0),
                I.constant(0.25, -0.5)):
        for scheme in (I.SCHEME_EULER, I.SCHEME_RK2):
            out = mesh.locate_feet(fld, 0.37, 0.013, scheme, want_feet=True)
            f_gpu = host(out["feet"])
            f_ref = orc.feet(w.xy, fld, 0.37, 0.013, scheme)
            if fld.kind in (I.FIELD_CONSTANT, I.FIELD_SOLID_BODY, I.FIELD_AFFINE):
                assert (f_gpu == f_ref).all()            # same operations, same rounding
                e_ref, _ = orc.locate(w.xy, w.tri, f_ref)
                assert (host(out["elem"]) == e_ref).all()
            else:
                assert np.abs(f_gpu - f_ref).max() < 8 * 2.0 ** -52


def test_step_rotation_33_end_to_end(S, C, orc):
    """33x33 jittered grid, solid-body rotation, Euler, dt = 0.05, 20 steps,
    P1, FP64: element indices bit-exact at every step, values within 1e-12."""
    w = I.small_rotation()
    mesh = S.Mesh(C, w.xy, w.tri)
    v = dev(w.v0)
    v_ref = w.v0.astype(np.float64)
    for n in range(w.steps):
        t_n = n * w.dt
        out = mesh.locate_feet(w.field, t_n + w.dt, w.dt, w.scheme)
        v_new, q, e_ref, _ = orc.sl_step(w.xy, w.tri, v_ref, w.field, t_n, w.dt, w.scheme)
        assert (host(out["elem"]) == e_ref).all(), n
        v, st = mesh.step(w.field, t_n, w.dt, w.scheme, v, stats=True)
        v_ref = v_new
        assert rel_err(host(v), v_ref) < TOL64, n
    assert st["feet"] == w.xy.shape[0]


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("flags", [0, 0x8])
def test_step_swirl_p1_p2_from_identical_values(S, C, orc, order, flags):
    w = I.swirl_500(alpha=5.0, order="random", n=70)
    mesh = S.Mesh(C, w.xy, w.tri, flags | (S.P2 if order == 2 else 0))
    p2 = orc.P2Dofs(w.xy, w.tri)
    pts = w.xy if order == 1 else p2.xy
    v0 = I.gaussian_hill(pts)[:, None]
    perm = mesh.dof_order() if flags & S.INTERNAL_ORDER else None
    for n in (0, 7):
        t_n = n * w.dt
        v_in = v0 if perm is None else v0[perm]
        v_out = host(mesh.step(w.field, t_n, w.dt, I.SCHEME_RK2, dev(v_in), order=order))
        ref, _, _, _ = orc.sl_step(w.xy, w.tri, v0, w.field, t_n, w.dt, I.SCHEME_RK2, order, p2)
        if perm is not None:
            ref = ref[perm]
        assert rel_err(v_out, ref, np.abs(v0).max()) < TOL64


def test_step_fp32_values_k16_graded(S, C, orc):
    """Graded mesh, RK2, 16 Gaussian-hill fields sharing one location, FP32
    values on FP64 coordinates; per step from identical V^n."""
    w = I.graded_swirl(alpha=5.0, n=101, k_fields=16)
    mesh = S.Mesh(C, w.xy, w.tri)
    v0 = w.v0.astype(np.float32)
    out = host(mesh.step(w.field, 0.2, w.dt, I.SCHEME_RK2, dev(v0)))
    ref, _, _, _ = orc.sl_step(w.xy, w.tri, v0.astype(np.float64), w.field, 0.2, w.dt, I.SCHEME_RK2)
    assert rel_err(out, ref, np.abs(v0).max()) < TOL32
    # FP64 values on the same mesh: 1e-12
    out64 = host(mesh.step(w.field, 0.2, w.dt, I.SCHEME_RK2, dev(v0.astype(np.float64))))
    assert rel_err(out64, ref, np.abs(v0).max()) < TOL64


def test_step_fp32_mesh_values(S, C, orc):
    """FP32 coordinates, feet and values: error against the FP64 pipeline."""
    w = I.swirl_500(alpha=5.0, order="morton", n=90)
    mesh = S.Mesh(C, w.xy, w.tri, S.COORDS_F32)
    v0 = w.v0.astype(np.float32)
    out, st = mesh.step(w.field, 0.1, w.dt, I.SCHEME_EULER, dev(v0), stats=True)
    ref, _, _, _ = orc.sl_step(w.xy, w.tri, v0.astype(np.float64), w.field, 0.1, w.dt, I.SCHEME_EULER)
    assert rel_err(host(out), ref, 1.0) < 1e-5
    assert st["feet"] == w.xy.shape[0]


def test_start_modes_and_step_cap_do_not_change_results(S, C, orc):
    w = I.swirl_500(alpha=20.0, order="random", n=64)
    mesh = S.Mesh(C, w.xy, w.tri)
    feet = orc.feet(w.xy, w.field, 0.5, w.dt, I.SCHEME_EULER)
    e_ref, _ = orc.locate(w.xy, w.tri, feet)
    base = mesh.locate_feet(feet=dev(feet), feet_in=True, want_steps=True, stats=True)
    assert (host(base["elem"]) == e_ref).all()
    rng = np.random.default_rng(3)
    given = rng.integers(0, w.tri.shape[0], w.xy.shape[0]).astype(np.int32)
    for mode, start in ((S.START_GIVEN, given), (S.START_FIXED, np.array([17], np.int32)),
                        (S.START_PREV, None), (S.START_PREV, None)):
        out = mesh.locate_feet(feet=dev(feet), feet_in=True, start_mode=mode,
                               start=None if start is None else dev(start), want_steps=True)
        assert (host(out["elem"]) == e_ref).all(), mode
    # strategy (b) from the exact previous element: no element change at all
    assert host(out["steps"]).max() == 0
    # a step cap of 1 sends nearly every walk through the randomised walk
    mesh.set_walk_limits(step_cap=1)
    out = mesh.locate_feet(feet=dev(feet), feet_in=True, start_mode=S.START_FIXED, start=dev(np.array([0], np.int32)),
                           stats=True)
    assert (host(out["elem"]) == e_ref).all()
    assert out["stats"]["fallback_walks"] > 0.9 * w.xy.shape[0]


def test_walk_steps_plateau_random_incident_start(S, C, orc):
    """Section 2.2 remark: a random incident start costs about 1.5 element
    changes even when the query is the start node; the start steered by the
    foot's direction (the incident triangle facing the diagonal of its
    quadrant) costs a fraction of one."""
    xy, tri = I.jittered_grid(300, 21)
    mesh = S.Mesh(C, xy, tri)
    rng = np.random.default_rng(8)
    # queries a tiny step away from every node in a random direction
    ang = rng.uniform(0, 2 * np.pi, xy.shape[0])
    q = xy + 1e-9 * np.stack([np.cos(ang), np.sin(ang)], axis=1)
    # a random incident triangle per node (from the triangle list)
    inc = [[] for _ in range(xy.shape[0])]
    for t, (a, b, c) in enumerate(tri):
        inc[a].append(t)
        inc[b].append(t)
        inc[c].append(t)
    start = np.array([l[rng.integers(0, len(l))] for l in inc], dtype=np.int32)
    out = mesh.locate_feet(feet=dev(q), feet_in=True, start_mode=S.START_GIVEN, start=dev(start), want_steps=True)
    e_ref, _ = orc.locate(xy, tri, q)
    e = host(out["elem"])
    ok = e_ref >= 0
    assert (e == e_ref).all()
    mean_random = host(out["steps"])[ok].mean()
    assert 1.2 < mean_random < 1.8, mean_random
    out = mesh.locate_feet(feet=dev(q), feet_in=True, want_steps=True)
    assert host(out["steps"])[ok].mean() < 0.4


def test_interpolate_entry_point(S, C, orc):
    w = I.swirl_500(alpha=5.0, order="random", n=50)
    p2 = orc.P2Dofs(w.xy, w.tri)
    mesh = S.Mesh(C, w.xy, w.tri, S.P2)
    q = I.random_points(3000, 9, -0.05, 1.05)
    elem, bary, _ = mesh.locate(dev(q))
    e_ref, b_ref = orc.locate(w.xy, w.tri, q)
    vals = I.quadratic_data(p2.xy)[:, None].repeat(3, axis=1) * np.array([1.0, -2.0, 0.5])
    for order in (1, 2):
        v = vals if order == 2 else vals[: w.xy.shape[0]]
        out = host(mesh.interpolate(order, elem, bary, dev(v), outside_value=-3.0))
        ref = orc.interp(order, w.tri, e_ref, b_ref, v, w.xy.shape[0], p2.tri_edges, -3.0)
        assert rel_err(out, ref, np.abs(v).max()) < TOL64
        out32 = host(mesh.interpolate(order, elem, bary, dev(v.astype(np.float32)), outside_value=-3.0))
        assert rel_err(out32, ref, np.abs(v).max()) < TOL32


def test_user_and_internal_order_agree(S, C):
    import torch
    w = I.swirl_500(alpha=5.0, order="random", n=40)
    m_user = S.Mesh(C, w.xy, w.tri)
    m_int = S.Mesh(C, w.xy, w.tri, S.INTERNAL_ORDER)
    perm = m_int.dof_order()
    v = w.v0
    a = host(m_user.step(w.field, 0.0, w.dt, I.SCHEME_EULER, dev(v)))
    v_int = m_int.permute_rows(dev(v), to_internal=True)
    assert (host(v_int) == v[perm]).all()
    b = m_int.step(w.field, 0.0, w.dt, I.SCHEME_EULER, v_int)
    back = host(m_int.permute_rows(b, to_internal=False))
    assert (back == a).all()


def test_api_errors(S, C):
    import torch
    xy, tri = I.jittered_grid(10, 1)
    mesh = S.Mesh(C, xy, tri)
    v = dev(np.zeros((xy.shape[0], 1)))
    with pytest.raises(S.SlwError) as ei:
        mesh.step(I.swirl(), 0.0, 0.1, 7, v)
    assert ei.value.name == "SLW_E_ARG"
    with pytest.raises(S.SlwError) as ei:
        mesh.step(I.swirl(), 0.0, 0.1, 0, v, order=2)
    assert ei.value.name == "SLW_E_UNSUPPORTED"
    with pytest.raises(S.SlwError):
        mesh.step(I.swirl(), 0.0, 0.1, 0, v, v_out=v)   # aliasing
