"""The hybrid start (a per-foot choice among the previous element, the chart
cell and the steered start, from how far the foot moved): results identical
to the steered start's, every element against the oracle, for any
threshold, with and without a chart, on the graded mesh across its Courant
range and on the first step (no previous elements)."""
import numpy as np
import pytest

from paper_2104_09189_amd import inputs as I
from gpu_util import check_elements_near, ctx as _ctx, dev, host, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    from paper_2104_09189_amd import slwalk
    return slwalk


@pytest.fixture(scope="module")
def C(S):
    return _ctx()


def _step(S, mesh, w, t_n, vin, mode):
    e = dev(np.zeros(mesh.n_nodes, np.int32))
    v, st = mesh.step(w.field, t_n, w.dt, w.scheme, vin, start_mode=mode, elem=e, stats=True)
    return host(v).copy(), host(e).copy(), st


@pytest.mark.parametrize("alpha", [5.0, 50.0])
def test_hybrid_graded_same_bits_and_oracle(S, C, orc, alpha):
    w = I.graded_swirl(alpha=alpha)
    mesh = S.Mesh(C, w.xy, w.tri, S.INTERNAL_ORDER)
    perm = mesh.dof_order()
    v0 = w.v0.astype(np.float32)
    vin = dev(v0[perm])
    mesh.chart_build(2048)
    for t_n in (6 * w.dt, 7 * w.dt):            # first step: no previous elements; second: from them
        ref_v, ref_e, st_a = _step(S, mesh, w, t_n, vin, S.START_STEERED)
        v, e, st = _step(S, mesh, w, t_n, vin, S.START_HYBRID)
        assert np.array_equal(v, ref_v) and np.array_equal(e, ref_e)
        assert st["walk_steps"] < st_a["walk_steps"]
        assert sum(st["step_hist"]) == st["feet"]
    q = orc.feet(w.xy, w.field, 8 * w.dt, w.dt, w.scheme)
    r, _ = orc.locate(w.xy, w.tri, q)
    e_user = np.empty_like(e)
    e_user[perm] = e
    check_elements_near(w.xy, w.tri, q, r, e_user, 64 * 2.0 ** -52)


def test_hybrid_threshold_and_no_chart_change_nothing(S, C, orc):
    w = I.swirl_500(alpha=20.0, order="random")
    mesh = S.Mesh(C, w.xy, w.tri)
    vin = dev(w.v0)
    ref_v, ref_e, _ = _step(S, mesh, w, 0.3, vin, S.START_STEERED)
    ref, _, r, _ = orc.sl_step(w.xy, w.tri, w.v0, w.field, 0.3, w.dt, w.scheme)
    for chart in (False, True):
        if chart:
            mesh.chart_build(512)
        for far in (0.25, 8.0, 1e30, 0.0):
            mesh.set_hybrid(far)
            _step(S, mesh, w, 0.2, vin, S.START_HYBRID)          # previous elements from another time
            v, e, st = _step(S, mesh, w, 0.3, vin, S.START_HYBRID)
            assert np.array_equal(v, ref_v) and np.array_equal(e, ref_e), (chart, far)
            assert rel_err(v, ref, np.abs(w.v0).max()) < 1e-12
    for bad in (-1.0, float("inf"), float("nan")):
        with pytest.raises(S.SlwError):
            mesh.set_hybrid(bad)
    with pytest.raises(S.SlwError):
        mesh.locate_feet(w.field, 0.3, w.dt, w.scheme, start_mode=S.START_HYBRID)
