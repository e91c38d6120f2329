"""The paper's walk on the host (oracle/walk.c): what the walk of Section 2.2
must return and how long it must take, checked against facts independent of
it -- the closed containment of the definition, the oracle's unique
containers, the 1.5-move mean of a random incident start on a regular star
(Remark in Section 2.2) and zero moves from the sector start, and walk lengths
growing with the Courant number (Section 3 (a))."""
import numpy as np
import pytest

from paper_2104_09189_amd import inputs as I


@pytest.fixture(scope="module")
def W():
    from oracle import walk
    return walk


def _containers_exact(orc, xy, tri, q, e):
    """Whether triangle e[i] is a closed container of q[i] (exact signs)."""
    ok = np.empty(len(e), bool)
    for i, (pt, t) in enumerate(zip(q, e)):
        a, b, c = (xy[v] for v in tri[t])
        s = [orc.orient_sign(a, b, pt), orc.orient_sign(b, c, pt), orc.orient_sign(c, a, pt)]
        ok[i] = min(s) >= 0 or max(s) <= 0
    return ok


@pytest.mark.parametrize("rule", [0, 1])
def test_walk_returns_a_closed_container_and_the_unique_one(W, orc, rule):
    xy, tri = I.permute_mesh(*I.jittered_grid(33, 71), 4)
    M = W.Mesh(xy, tri)
    q = orc.feet(xy, I.swirl(1.0), 0.3, 0.08, I.SCHEME_RK2)
    e, s = M.locate_nodes(q, rule, seed=9)
    r, _ = orc.locate(xy, tri, q)
    assert (e >= 0).all() and (r >= 0).all()
    assert _containers_exact(orc, xy, tri, q, e).all()
    unique = np.array([len(orc.containers(xy, tri, tuple(p))) == 1 for p in q])
    assert unique.sum() > 800
    assert np.array_equal(e[unique], r[unique])
    assert s.max() > 0


def test_walk_outside_and_given_starts(W, orc):
    xy, tri = I.jittered_grid(25, 72)
    M = W.Mesh(xy, tri)
    q = orc.feet(xy, I.constant(0.9, 0.3), 0.0, 0.2, I.SCHEME_EULER)
    e, s = M.locate_nodes(q, 1)
    r, _ = orc.locate(xy, tri, q)
    assert np.array_equal(e < 0, r < 0) and (e < 0).sum() > 50
    # the same walk from given starts (every foot from triangle 0)
    e2, s2 = M.walk(q, np.zeros(len(q), np.int32))
    assert np.array_equal(e2 < 0, r < 0)
    inside = e2 >= 0
    assert _containers_exact(orc, xy, tri, q[inside], e2[inside]).all()
    assert s2.mean() > s.mean()


def test_random_start_plateau_and_sector_start_zero(W):
    """Unjittered grid (every interior node has six incident triangles) and
    feet a tiny step from their node in a random direction: from a random
    incident triangle the walk turns around the node to the foot's triangle,
    0, 1, 1, 2, 2 or 3 moves, 1.5 on average; the sector start needs none."""
    n = 81
    xy, tri = I.grid_nodes(n), I.grid_triangles(n)
    M = W.Mesh(xy, tri)
    rng = np.random.default_rng(5)
    ang = rng.uniform(0, 2 * np.pi, xy.shape[0])
    q = xy + 1e-4 / (n - 1) * np.stack([np.cos(ang), np.sin(ang)], axis=1)
    interior = ((xy > 0) & (xy < 1)).all(axis=1)
    _, s_rand = M.locate_nodes(q, 0, seed=17)
    _, s_sec = M.locate_nodes(q, 1)
    assert abs(s_rand[interior].mean() - 1.5) < 0.06
    assert set(np.unique(s_rand[interior])) <= {0, 1, 2, 3}
    assert (s_sec[interior] == 0).all()


def test_walk_lengths_grow_linearly_with_courant(W, orc):
    xy, tri = I.jittered_grid(161, 73)
    M = W.Mesh(xy, tri)
    h = 1.0 / 160
    means = []
    for alpha in (4.0, 8.0, 16.0):
        q = orc.feet(xy, I.swirl(1.0), 0.2, alpha * h, I.SCHEME_RK2)
        e, s = M.locate_nodes(q, 1)
        means.append(s[e >= 0].mean())
    # linear with an offset (the start saves the first cells): doubling the
    # Courant number doubles the increase
    assert 1.7 < (means[2] - means[1]) / (means[1] - means[0]) < 2.5


def test_one_thread_equals_all_threads(W, orc):
    xy, tri = I.jittered_grid(65, 74)
    M = W.Mesh(xy, tri)
    q = orc.feet(xy, I.swirl(1.0), 0.1, 0.1, I.SCHEME_RK2)
    a = M.locate_nodes(q, 0, seed=3, threads=1)
    b = M.locate_nodes(q, 0, seed=3, threads=0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
