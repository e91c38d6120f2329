"""Variable step at the boundary on the GPU: feet that leave the domain stop
where their segment crosses the boundary and take the Dirichlet datum there
(against the oracle, and against the exact solution of constant advection)."""
import numpy as np
import pytest

from paper_2104_09189_amd import inputs as I
from gpu_util import ctx as _ctx, dev, host, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    from paper_2104_09189_amd import slwalk
    return slwalk


@pytest.fixture(scope="module")
def C(S):
    return _ctx()


AX, AY = 0.3, -0.2
C0, C1, C2 = 0.7, -1.3, 2.1
BC = (C0, C1, C2, -(C1 * AX + C2 * AY))


def _u(x, y, t):
    return C0 + C1 * (x - AX * t) + C2 * (y - AY * t)


@pytest.mark.parametrize("scheme", [0, 1])
def test_constant_advection_exact_with_inflow_data(S, C, scheme):
    xy, tri = I.permute_mesh(*I.jittered_grid(41, 801), 2)
    mesh = S.Mesh(C, xy, tri)
    mesh.set_boundary(S.BC_AFFINE, BC)
    t_n, dt = 0.4, 0.25
    v0 = np.stack([_u(xy[:, 0], xy[:, 1], t_n)] * 3, axis=1)
    v, st = mesh.step(I.constant(AX, AY), t_n, dt, scheme, dev(v0), stats=True)
    assert st["outside"] > 100
    ref = _u(xy[:, 0], xy[:, 1], t_n + dt)
    assert np.abs(host(v) - ref[:, None]).max() < 1e-12


@pytest.mark.parametrize("flags,order", [(0, 1), (0x8, 1), (0x2, 2)])
def test_boundary_values_match_oracle(S, C, orc, flags, order):
    xy, tri = I.permute_mesh(*I.jittered_grid(33, 802), 3)
    fld = I.Field(I.FIELD_AFFINE, (0.4, -1.1, 0.9, 0.2, 0.5, 0.5, 0.35, -0.3))
    mesh = S.Mesh(C, xy, tri, flags)
    p2 = orc.P2Dofs(xy, tri) if order == 2 else None
    pts = xy if order == 1 else p2.xy
    perm = mesh.dof_order() if flags & 0x8 else np.arange(mesh.n_dofs)
    v0 = I.gaussian_hill(pts)[:, None]
    bc = (2, (0.1, 0.5, -0.25, 0.75))
    mesh.set_boundary(S.BC_AFFINE, bc[1])
    v, st = mesh.step(fld, 0.3, 0.2, S.SLW_RK2, dev(v0[perm]), order=order, stats=True)
    ref, _, elem, _ = orc.sl_step(xy, tri, v0, fld, 0.3, 0.2, I.SCHEME_RK2, order=order, p2=p2, bc=bc)
    assert (elem < 0).sum() > 50
    assert st["outside"] == (elem < 0).sum()
    assert rel_err(host(v), ref[perm], 1.0) < 1e-12
    # constant data; and switching the data off restores outside_value
    mesh.set_boundary(S.BC_CONSTANT, (4.5,))
    v = host(mesh.step(fld, 0.3, 0.2, S.SLW_RK2, dev(v0[perm]), order=order))
    assert (v[(elem < 0)[perm]] == 4.5).all()
    mesh.set_boundary(S.BC_NONE)
    v = host(mesh.step(fld, 0.3, 0.2, S.SLW_RK2, dev(v0[perm]), order=order, outside_value=-2.0))
    assert (v[(elem < 0)[perm]] == -2.0).all()


def test_float_mesh_and_far_feet(S, C):
    """Feet far outside the bounding box are walked to the boundary too; a
    float mesh reproduces the exact solution to float accuracy."""
    xy, tri = I.jittered_grid(25, 803)
    mesh = S.Mesh(C, xy, tri, S.COORDS_F32)
    bx, by = 3.0, 1.0                               # most feet far outside
    mesh.set_boundary(S.BC_AFFINE, (C0, C1, C2, -(C1 * bx + C2 * by)))
    t_n, dt = 0.0, 0.5

    def g(x, y, t):
        return C0 + C1 * (x - bx * t) + C2 * (y - by * t)

    v0 = g(xy[:, 0], xy[:, 1], t_n)[:, None].astype(np.float32)
    v, st = mesh.step(I.constant(bx, by), t_n, dt, S.SLW_EULER, dev(v0), stats=True)
    assert st["outside"] > xy.shape[0] // 2
    xf = xy.astype(np.float32).astype(np.float64)
    ref = g(xf[:, 0], xf[:, 1], t_n + dt)
    assert np.abs(host(v)[:, 0] - ref).max() < 1e-4 * np.abs(ref).max()


def test_boundary_with_chart_start_and_rejections(S, C):
    xy, tri = I.jittered_grid(30, 804)
    mesh = S.Mesh(C, xy, tri)
    mesh.chart_build(16)
    mesh.set_boundary(S.BC_AFFINE, BC)
    t_n, dt = 0.4, 0.25
    v0 = _u(xy[:, 0], xy[:, 1], t_n)[:, None]
    mesh.set_repack(4)                              # ignored while boundary data are set
    v = host(mesh.step(I.constant(AX, AY), t_n, dt, S.SLW_EULER, dev(v0), start_mode=S.START_CHART))
    assert np.abs(v[:, 0] - _u(xy[:, 0], xy[:, 1], t_n + dt)).max() < 1e-12
    # strategy (c) on the mesh forest applies boundary data; on chains it refuses
    v = host(mesh.step(I.constant(AX, AY), t_n, dt, S.SLW_EULER, dev(v0), start_mode=S.START_NEIGHBOR))
    assert np.abs(v[:, 0] - _u(xy[:, 0], xy[:, 1], t_n + dt)).max() < 1e-12
    mesh.set_chain(4)
    with pytest.raises(S.SlwError):
        mesh.step(I.constant(AX, AY), t_n, dt, S.SLW_EULER, dev(v0), start_mode=S.START_NEIGHBOR)
    with pytest.raises(S.SlwError):
        mesh.set_boundary(7, BC)
