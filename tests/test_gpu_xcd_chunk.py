"""The spread of tiles over the XCDs (slw_mesh_set_xcd_chunk) changes which
workgroup steps which tile, never a result: every chunk size gives the same
bits for the step (each start mode, P1 and P2, lane schedules, chains),
location, feet and interpolation, on grids smaller than one round of chunks
and with ragged tails; and the step matches the oracle."""
import numpy as np
import pytest

from paper_2104_09189_amd import inputs as I
from gpu_util import ctx as _ctx, dev, host, rel_err

pytestmark = pytest.mark.gpu

# 0: one range per XCD; 3: chunks that do not divide the tile count; 4096:
# larger than any tile count here (every tile on the tail path)
CHUNKS = (0, 1, 3, 16, 64, 4096)
STAT_KEYS = ("feet", "outside", "walk_steps", "max_steps", "edge_ties", "vertex_ties", "fallback_walks")


@pytest.fixture(scope="module")
def S():
    from paper_2104_09189_amd import slwalk
    return slwalk


@pytest.fixture(scope="module")
def C(S):
    return _ctx()


def _same_for_every_chunk(mesh, run):
    ref = None
    for c in CHUNKS:
        mesh.set_xcd_chunk(c)
        out = run()
        if ref is None:
            ref = out
            continue
        for a, b in zip(out, ref):
            if isinstance(a, dict):
                assert {k: a[k] for k in STAT_KEYS} == {k: b[k] for k in STAT_KEYS}, c
            else:
                assert np.array_equal(a, b, equal_nan=True), c
    mesh.set_xcd_chunk(64)
    return ref


@pytest.mark.parametrize("n", [9, 41, 130])
def test_step_modes_same_bits_for_every_chunk(S, C, orc, n):
    """Tile counts 1, 7 and 67: below one round of chunks, ragged, and over a round."""
    xy, tri = I.permute_mesh(*I.jittered_grid(n, 1100 + n), 5)
    fld = I.swirl(1.0)
    mesh = S.Mesh(C, xy, tri)
    mesh.chart_build(32)
    v0 = I.gaussian_hill(xy)[:, None] * np.array([1.0, -2.0, 0.5])
    t_n, dt = 0.2, 4.0 / (n - 1)
    for mode in (S.START_STEERED, S.START_PREV, S.START_NEIGHBOR, S.START_CHART, S.START_HYBRID):
        def run():
            e = dev(np.zeros(xy.shape[0], np.int32))
            if mode in (S.START_PREV, S.START_HYBRID):
                mesh.step(fld, t_n - dt, dt, S.SLW_RK2, dev(v0), start_mode=mode)
            v, st = mesh.step(fld, t_n, dt, S.SLW_RK2, dev(v0), start_mode=mode, elem=e, stats=True)
            return host(v).copy(), host(e).copy(), st
        v, e, _ = _same_for_every_chunk(mesh, run)
        if mode == S.START_STEERED:
            ref, q, elem, _ = orc.sl_step(xy, tri, v0, fld, t_n, dt, I.SCHEME_RK2)
            assert rel_err(v, ref, np.abs(v0).max()) < 1e-12


def test_p2_schedules_and_chains_same_bits(S, C):
    xy, tri = I.jittered_grid(57, 1201)
    fld = I.swirl(1.0)
    v0 = I.gaussian_hill(xy)[:, None]
    mesh2 = S.Mesh(C, xy, tri, S.P2)
    v2 = np.random.default_rng(3).normal(size=(mesh2.n_dofs, 2))
    _same_for_every_chunk(mesh2, lambda: (host(mesh2.step(fld, 0.1, 0.05, S.SLW_EULER, dev(v2), order=2)).copy(),))
    mesh = S.Mesh(C, xy, tri)
    for rp in (2, 4):
        mesh.set_repack(rp)
        _same_for_every_chunk(mesh, lambda: (host(mesh.step(fld, 0.1, 0.05, S.SLW_EULER, dev(v0))).copy(),))
    mesh.set_repack(0)
    mesh.set_chain(4)
    _same_for_every_chunk(mesh, lambda: (host(mesh.step(fld, 0.1, 0.05, S.SLW_EULER, dev(v0),
                                                        start_mode=S.START_NEIGHBOR)).copy(),))


def test_locate_feet_and_interpolate_same_bits(S, C):
    xy, tri = I.permute_mesh(*I.jittered_grid(73, 1301), 9)
    mesh = S.Mesh(C, xy, tri)
    rng = np.random.default_rng(13)
    q = dev(rng.uniform(-0.1, 1.1, (30001, 2)))
    v0 = dev(I.gaussian_hill(xy)[:, None] * np.ones((1, 4)))

    def run():
        e, b, s = mesh.locate(q, want_steps=True)
        out = mesh.locate_feet(I.swirl(1.0), 0.3, 0.05, S.SLW_RK2, want_feet=True, want_steps=True)
        vi = mesh.interpolate(1, e, b, v0)
        return (host(e).copy(), host(b).copy(), host(s).copy(), host(out["elem"]).copy(),
                host(out["feet"]).copy(), host(out["steps"]).copy(), host(vi).copy())
    _same_for_every_chunk(mesh, run)


def test_set_xcd_chunk_rejects_out_of_range(S, C):
    xy, tri = I.jittered_grid(9, 1401)
    mesh = S.Mesh(C, xy, tri)
    for bad in (-1, 4097):
        with pytest.raises(S.SlwError):
            mesh.set_xcd_chunk(bad)
    mesh.set_xcd_chunk(4096)
    mesh.set_xcd_chunk(0)
