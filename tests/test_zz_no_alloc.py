"""slw_step_noalloc, the step entry point that allocates nothing (its
counters and permutation workspace live in a static device array), against
slw_step through the C-ABI: identical values, elements and statistics on two
calls in a row, the second with a smaller input, and the size limit."""
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


def _case(S, C, n, seed, k, dtype, order, scheme):
    import torch
    xy, tri = I.jittered_grid(n, seed)
    xy, tri = I.permute_mesh(xy, tri, seed + 1)       # user order differs from the internal one
    mesh = S.Mesh(C, xy, tri, S.P2 if order == 2 else 0)
    rows = mesh.n_nodes if order == 1 else mesh.n_dofs
    pts = xy if order == 1 else mesh.dof_coords()
    rng = np.random.default_rng(seed)
    v0 = np.concatenate([I.gaussian_hill(pts)[:, None], rng.uniform(-1, 1, (rows, k - 1))], axis=1)
    vin = dev(v0.astype(dtype))
    h = 1.0 / (n - 1)
    dt = 5.0 * h
    out = {}
    for noalloc in (True, False):
        e = torch.full((rows,), -7, dtype=torch.int32, device="cuda:0")
        v, st = mesh.step(I.swirl(1.0), 0.2, dt, scheme, vin, order=order, stats=True, elem=e, noalloc=noalloc)
        out[noalloc] = (host(v).copy(), host(e).copy(), st)
    return mesh, out


def test_noalloc_matches_step_on_two_calls_second_smaller(S, C):
    big = _case(S, C, 300, 11, 4, np.float64, 1, I.SCHEME_RK2)[1]
    small = _case(S, C, 60, 12, 2, np.float32, 2, I.SCHEME_EULER)[1]
    for res in (big, small):
        (va, ea, sa), (vb, eb, sb) = res[True], res[False]
        assert np.array_equal(va, vb)
        assert np.array_equal(ea, eb)
        assert (ea >= -1).all()
        assert sa == sb
        assert sum(sa["step_hist"]) == sa["feet"] > 0
    # the second call's counters started from zero (the first call's are not carried over)
    assert small[True][2]["feet"] == small[False][2]["feet"] < big[True][2]["feet"]


def test_noalloc_rejects_inputs_beyond_its_scratch(S, C):
    import torch
    xy, tri = I.jittered_grid(100, 13)
    xy, tri = I.permute_mesh(xy, tri, 14)
    mesh = S.Mesh(C, xy, tri)
    vin = torch.zeros((mesh.n_nodes, 1000), dtype=torch.float64, device="cuda:0")   # 80 MB > 64 MiB
    with pytest.raises(S.SlwError) as ei:
        mesh.step(I.swirl(1.0), 0.0, 0.01, I.SCHEME_EULER, vin, noalloc=True)
    assert ei.value.code == 1 and "scratch" in str(ei.value)
    # the library is still usable: a fitting call right after
    v1 = mesh.step(I.swirl(1.0), 0.0, 0.01, I.SCHEME_EULER, vin[:, :2].contiguous(), noalloc=True)
    v2 = mesh.step(I.swirl(1.0), 0.0, 0.01, I.SCHEME_EULER, vin[:, :2].contiguous())
    assert torch.equal(v1, v2)
