"""Lane repacking in the step kernel: every lane schedule gives the same bits,
the same walk statistics, and the oracle's values."""
import numpy as np
import pytest

from paper_2104_09189_amd import inputs as I
from gpu_util import ctx as _ctx, dev, host, rel_err

pytestmark = pytest.mark.gpu

SCHEDULES = (1, 2, 4, 8)
STAT_KEYS = ("feet", "outside", "walk_steps", "max_steps", "edge_ties", "vertex_ties", "fallback_walks")


@pytest.fixture(scope="module")
def S():
    from paper_2104_09189_amd import slwalk
    return slwalk


@pytest.fixture(scope="module")
def C(S):
    return _ctx()


def _run(S, mesh, fld, t_n, dt, scheme, v0, **kw):
    out = {}
    for rp in SCHEDULES:
        mesh.set_repack(rp)
        v, st = mesh.step(fld, t_n, dt, scheme, dev(v0), stats=True, **kw)
        out[rp] = (host(v).copy(), {k: st[k] for k in STAT_KEYS})
    mesh.set_repack(0)
    return out


def _same(out):
    v1, s1 = out[1]
    for rp, (v, s) in out.items():
        assert np.array_equal(v, v1), rp
        assert s == s1, (rp, s, s1)
    return v1, s1


def test_every_schedule_same_bits_and_oracle(S, C, orc):
    # 57 x 57 nodes: 3,249 DOFs, a ragged last chunk for every schedule
    xy, tri = I.permute_mesh(*I.jittered_grid(57, 611), 12)
    h = 1.0 / 56
    fld, dt = I.swirl(1.0), 5 * h
    mesh = S.Mesh(C, xy, tri)
    v0 = np.stack([I.gaussian_hill(xy), xy[:, 0], xy[:, 1] ** 2], axis=1).astype(np.float32)
    v, st = _same(_run(S, mesh, fld, 0.3, dt, S.SLW_RK2, v0))
    assert st["feet"] == xy.shape[0] and st["walk_steps"] > xy.shape[0]
    ref, _, _, _ = orc.sl_step(xy, tri, v0.astype(np.float64), fld, 0.3, dt, I.SCHEME_RK2)
    assert rel_err(v, ref, np.abs(v0).max()) < 1e-5


def test_p2_fp64_and_outside_feet(S, C, orc):
    xy, tri = I.jittered_grid(33, 612)
    p2 = orc.P2Dofs(xy, tri)
    mesh = S.Mesh(C, xy, tri, S.P2)
    fld = I.constant(0.3, -0.2)                   # pushes a band of feet out of the square
    v0 = I.gaussian_hill(p2.xy)[:, None]
    v, st = _same(_run(S, mesh, fld, 0.0, 0.1, S.SLW_EULER, v0, order=2, outside_value=-7.0))
    assert st["outside"] > 100
    ref, _, _, _ = orc.sl_step(xy, tri, v0, fld, 0.0, 0.1, I.SCHEME_EULER, order=2, p2=p2, outside_value=-7.0)
    assert rel_err(v, ref, 1.0) < 1e-12


def test_float_mesh_and_internal_order(S, C):
    xy, tri = I.jittered_grid(70, 613)
    mesh = S.Mesh(C, xy, tri, S.COORDS_F32 | S.INTERNAL_ORDER)
    v0 = I.gaussian_hill(xy)[mesh.dof_order()][:, None].astype(np.float32)
    _same(_run(S, mesh, I.swirl(0.7), 0.1, 20.0 / 69, S.SLW_RK2, v0))


def test_strategy_b_state_is_the_same(S, C):
    xy, tri = I.jittered_grid(45, 614)
    fld, dt = I.swirl(1.0), 3.0 / 44
    v0 = I.gaussian_hill(xy)[:, None]
    results = []
    for rp in SCHEDULES:
        mesh = S.Mesh(C, xy, tri)
        mesh.set_repack(rp)
        a = mesh.step(fld, 0.0, dt, S.SLW_EULER, dev(v0), start_mode=S.START_PREV)
        b, st = mesh.step(fld, dt, dt, S.SLW_EULER, a, start_mode=S.START_PREV, stats=True)
        results.append((host(b).copy(), {k: st[k] for k in STAT_KEYS}))
        mesh.free()
    for v, st in results[1:]:
        assert np.array_equal(v, results[0][0])
        assert st == results[0][1]


def test_given_starts_user_order(S, C, orc):
    xy, tri = I.permute_mesh(*I.jittered_grid(30, 615), 3)
    mesh = S.Mesh(C, xy, tri)
    rng = np.random.default_rng(616)
    start = dev(rng.integers(0, tri.shape[0], xy.shape[0]).astype(np.int32))
    v0 = I.gaussian_hill(xy)[:, None]
    v, _ = _same(_run(S, mesh, I.swirl(1.0), 0.0, 0.05, S.SLW_EULER, v0, start_mode=S.START_GIVEN, start=start))
    ref, _, _, _ = orc.sl_step(xy, tri, v0, I.swirl(1.0), 0.0, 0.05, I.SCHEME_EULER)
    assert rel_err(v, ref, 1.0) < 1e-12


def test_chart_starts_fused_in_every_schedule(S, C):
    """Chart and learned starts computed inside the repacking kernel (or by
    their own kernel with one foot per lane) give the steered start's bits."""
    xy, tri = I.permute_mesh(*I.jittered_grid(64, 617), 4)
    mesh = S.Mesh(C, xy, tri)
    mesh.chart_build(32)
    net = S.Mlp(C, seed=11)
    mesh.attach_mlp(net)
    fld, dt = I.swirl(1.0), 10.0 / 63
    v0 = np.stack([I.gaussian_hill(xy), xy[:, 1]], axis=1).astype(np.float32)
    mesh.set_repack(1)
    ref, st_ref = mesh.step(fld, 0.2, dt, S.SLW_RK2, dev(v0), stats=True)
    ref = host(ref).copy()
    for mode in (S.START_CHART, S.START_LEARNED, S.START_LEARNED_INDEX):
        v, _ = _same(_run(S, mesh, fld, 0.2, dt, S.SLW_RK2, v0, start_mode=mode))
        assert np.array_equal(v, ref), mode
