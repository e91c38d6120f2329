"""Quadtree locator (non-walking comparator): the same elements as the
oracle and as the walk, bit-identical barycentric coordinates, for any leaf
size and depth."""
import numpy as np
import pytest

from paper_2104_09189_amd import inputs as I
from gpu_util import ctx as _ctx, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    from paper_2104_09189_amd import slwalk
    return slwalk


@pytest.fixture(scope="module")
def C(S):
    return _ctx()


def _queries(xy, tri, seed, m=3000):
    rng = np.random.default_rng(seed)
    a, b = xy[tri[:, 0]], xy[tri[:, 1]]
    q = [I.random_points(m, seed, -0.1, 1.1), xy, (a + b) * 0.5, a + 0.25 * (b - a),
         xy[tri].mean(axis=1)[rng.integers(0, tri.shape[0], 500)]]
    return np.concatenate(q)


@pytest.mark.parametrize("cap,depth", [(1, 24), (4, 24), (8, 3), (32, 0)])
def test_quadtree_equals_oracle_and_walk(S, C, orc, cap, depth):
    xy, tri = I.permute_mesh(*I.jittered_grid(30, 901), 6)
    tri = tri.copy()
    tri[::4] = tri[::4][:, [0, 2, 1]]              # clockwise input triangles
    mesh = S.Mesh(C, xy, tri)
    info = mesh.quadtree_build(cap, depth)
    assert info["depth"] <= depth and info["list_entries"] >= tri.shape[0]
    q = _queries(xy, tri, 5)
    e_qt, b_qt, st = mesh.locate_quadtree(dev(q), stats=True)
    e_ref, b_ref = orc.locate(xy, tri, q)
    e = host(e_qt)
    assert np.array_equal(e, e_ref)
    e_w, b_w, _ = mesh.locate(dev(q))
    assert np.array_equal(host(b_qt), host(b_w), equal_nan=True)
    inside = e_ref >= 0
    assert np.abs(host(b_qt)[inside] - b_ref[inside]).max() < 1e-12
    assert st["feet"] == q.shape[0] and st["outside"] == (~inside).sum()


def test_quadtree_graded_and_float_mesh(S, C, orc):
    xy, tri = I.graded_grid(101)
    q = np.concatenate([I.random_points(20000, 7, 0.0, 1.0), xy[::7]])
    mesh = S.Mesh(C, xy, tri)
    # the ring's thin triangles have long boxes: small leaves would list
    # them in too many cells
    with pytest.raises(S.SlwError):
        mesh.quadtree_build(2, 24)
    info = mesh.quadtree_build(32, 16)
    assert info["depth"] >= 4
    e_ref, _ = orc.locate(xy, tri, q)
    assert np.array_equal(host(mesh.locate_quadtree(dev(q))[0]), e_ref)
    mf = S.Mesh(C, xy, tri, S.COORDS_F32)
    mf.quadtree_build(32, 16)
    qf = q.astype(np.float32)
    ef, bf, _ = mf.locate_quadtree(dev(qf))
    ew, bw, _ = mf.locate(dev(qf))
    assert np.array_equal(host(ef), host(ew))
    assert np.array_equal(host(bf), host(bw), equal_nan=True)


def test_quadtree_errors_and_empty(S, C):
    xy, tri = I.jittered_grid(8, 902)
    mesh = S.Mesh(C, xy, tri)
    with pytest.raises(S.SlwError):
        mesh.locate_quadtree(dev(np.zeros((3, 2))))
    with pytest.raises(S.SlwError):
        mesh.quadtree_build(0, 10)
    mesh.quadtree_build(2, 10)
    e, b, _ = mesh.locate_quadtree(dev(np.zeros((0, 2))))
    assert e.shape[0] == 0
