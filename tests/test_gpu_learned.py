"""Learned start proposal: the network's GPU kernels against the NumPy oracle
(gradient, bfloat16 forward, Adam), the chart, and the invariant that a
learned start never changes what is found (indices bit-exact against the
oracle's point location, values bit-identical to the steered start)."""
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


def _samples(m, seed, valid=True):
    rng = np.random.default_rng(seed)
    X = np.empty((m, 5), dtype=np.float32)
    X[:, :2] = rng.uniform(0, 1, (m, 2))
    X[:, 2:4] = rng.normal(0, 0.02, (m, 2))
    X[:, 4] = rng.uniform(0, 1, m)
    Y = rng.uniform(0, 1, (m, 2)).astype(np.float32)
    return X, Y


def _normalised(X, norm):
    """the library's input normalisation, in float32: (f - shift) * scale"""
    X = np.asarray(X, dtype=np.float32)
    return ((X - norm[:5].astype(np.float32)) * norm[5:].astype(np.float32)).astype(np.float32)


@pytest.mark.parametrize("m", [1, 1000, 65536 + 37])
def test_gradient_matches_oracle(S, C, m):
    from oracle import mlp
    net = S.Mlp(C, seed=3)
    p = mlp.he_uniform(11)
    net.set_params(p)
    X, Y = _samples(m, 20 + m)
    norm = np.array([0.5, 0.5, 0.0, 0.0, 0.5, 3.4, 3.4, 50.0, 50.0, 3.4], dtype=np.float32)
    net.set_normalization(norm)
    assert np.array_equal(net.get_params(), p)
    g, loss = net.grad(dev(X), dev(Y))
    Xn = _normalised(X, norm).astype(np.float64)
    g_ref = mlp.grad(p.astype(np.float64), Xn, Y.astype(np.float64))
    l_ref = mlp.loss(p.astype(np.float64), Xn, Y.astype(np.float64))
    scale = np.abs(g_ref).max()
    assert np.abs(g - g_ref).max() <= 2e-5 * scale, np.abs(g - g_ref).max() / scale
    assert np.linalg.norm(g - g_ref) <= 1e-5 * np.linalg.norm(g_ref)
    assert abs(loss - l_ref) <= 1e-5 * l_ref
    # fixed-order reduction: bit-reproducible
    g2, _ = net.grad(dev(X), dev(Y))
    assert np.array_equal(g, g2)


def test_gradient_ignores_samples_without_target(S, C):
    from oracle import mlp
    net = S.Mlp(C, seed=4)
    p = mlp.he_uniform(12)
    net.set_params(p)
    X, Y = _samples(3000, 77)
    Y[::3] = np.nan                                 # feet outside: no target
    g, loss = net.grad(dev(X), dev(Y))
    keep = ~np.isnan(Y[:, 0])
    Xk, Yk = X[keep].astype(np.float64), Y[keep].astype(np.float64)
    # mean over all 3000 samples of the error of the kept ones
    g_ref = mlp.grad(p.astype(np.float64), Xk, Yk) * keep.sum() / 3000.0
    assert np.abs(g - g_ref).max() <= 2e-5 * np.abs(g_ref).max()
    assert abs(loss - mlp.loss(p.astype(np.float64), Xk, Yk)) <= 1e-5 * loss


def test_forward_bf16_matches_emulating_oracle(S, C):
    from oracle import mlp
    net = S.Mlp(C, seed=5)
    p = mlp.he_uniform(13)
    rng = np.random.default_rng(14)
    p = (p + rng.normal(0, 0.05, p.size)).astype(np.float32)   # non-zero biases too
    net.set_params(p)
    norm = np.array([0.5, 0.5, 0.0, 0.0, 0.5, 3.4, 3.4, 50.0, 50.0, 3.4], dtype=np.float32)
    net.set_normalization(norm)
    X, _ = _samples(5000 + 17, 15)                  # ragged last wavefront
    out = host(net.forward(dev(X)))
    Xn = _normalised(X, norm)
    ref16, _ = mlp.forward(p.astype(np.float64), Xn.astype(np.float64), bf16_operands=True)
    ref64, _ = mlp.forward(p.astype(np.float64), Xn.astype(np.float64))
    scale = max(1.0, np.abs(ref64).max())
    # same roundings as the emulation; only the accumulation order differs
    assert np.abs(out - ref16).max() <= 1e-2 * scale, np.abs(out - ref16).max()
    # against full precision: bfloat16's 8-bit significand
    assert np.abs(out - ref64).max() <= 5e-2 * scale


def test_adam_three_steps_match_oracle(S, C):
    """Three Adam steps on three minibatches whose targets move up, down and
    up again, so the gradient changes sign between steps (a swap of the two
    moment rates or a wrong bias correction would show in the second and
    third steps).  The oracle takes its own FP64 gradient at its own
    parameters each step.  The GPU's FP32 gradient differs from it by up to
    2e-5 of the largest entry, which Adam's normalisation turns into a
    relative error of the update of about 2e-5 * max|g| / |g|: entries whose
    gradient stays above 1% of the largest at every step are compared to
    1% of the learning rate, every entry to the 3 lr that three steps can
    move it at most."""
    from oracle import mlp
    lr = 1e-3
    net = S.Mlp(C, seed=6)
    p0 = mlp.he_uniform(16)
    net.set_params(p0)
    p = p0.astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    strong = np.ones(p.size, dtype=bool)
    for t, shift in enumerate((1.0, -1.5, 2.0), start=1):
        X, Y = _samples(512, 40 + t)
        Y = (Y + shift).astype(np.float32)
        net.train(dev(X), dev(Y), epochs=1, batch=512, lr=lr, seed=t)    # one minibatch: one step
        g = mlp.grad(p, X.astype(np.float64), Y.astype(np.float64))
        strong &= np.abs(g) >= 1e-2 * np.abs(g).max()
        p, m, v = mlp.adam(p, g, m, v, t, lr=lr)
    p_gpu = net.get_params().astype(np.float64)
    assert strong.sum() > 100
    assert np.abs(p_gpu - p)[strong].max() <= 1e-2 * lr, np.abs(p_gpu - p)[strong].max()
    assert np.abs(p_gpu - p).max() <= 3 * lr


def test_training_reduces_loss(S, C):
    net = S.Mlp(C, seed=7)
    rng = np.random.default_rng(18)
    X = rng.uniform(0, 1, (50000, 5)).astype(np.float32)
    Y = np.stack([np.sqrt(X[:, 0]), 0.5 + 0.4 * np.sin(3 * X[:, 1])], axis=1).astype(np.float32)
    Xd, Yd = dev(X), dev(Y)
    net.fit_normalization(Xd)
    norm = net.get_normalization()
    assert np.allclose(norm[:5], X.mean(axis=0), atol=1e-5)
    assert np.allclose(norm[5:], 1.0 / X.std(axis=0), rtol=1e-4)
    _, l0 = net.grad(Xd, Yd)
    net.train(Xd, Yd, epochs=20, batch=1024, lr=3e-3, seed=2)
    _, l1 = net.grad(Xd, Yd)
    assert l1 < 0.02 * l0, (l0, l1)


def _swirl_case(n=120, alpha=20.0, seed=901):
    xy, tri = I.jittered_grid(n, seed)
    h = 1.0 / (n - 1)
    return xy, tri, I.swirl(10.0), alpha * h   # slowly varying: walks of about alpha / 2 steps


def test_chart_of_a_regular_grid(S, C):
    """On an unjittered grid the chart is (up to the rank offsets) the
    identity, and the DOFs' chart coordinates are their own ranks."""
    xy, tri = I.jittered_grid(17, 1, jitter=0.0)
    mesh = S.Mesh(C, xy, tri)
    mesh.chart_build(16)
    uv = mesh.chart_coords()
    c = xy[tri].mean(axis=1)
    assert np.abs(uv[:, 0] - c[:, 0]).max() < 0.04
    assert np.abs(uv[:, 1] - c[:, 1]).max() < 0.04


def test_chart_is_a_rank_transform(S, C):
    xy, tri = I.permute_mesh(*I.jittered_grid(60, 31), 8)
    mesh = S.Mesh(C, xy, tri)
    g = 16
    mesh.chart_build(g)
    uv = mesh.chart_coords()
    nt = tri.shape[0]
    # u: the ranks (r + 1/2) / nt of the centroids' x
    assert np.array_equal(np.sort(uv[:, 0]), ((np.arange(nt) + 0.5) / nt).astype(np.float32))
    c = xy[tri].mean(axis=1)
    o = np.argsort(uv[:, 0], kind="stable")
    dx = np.diff(c[o, 0])
    assert (dx > -1e-6).all()
    # v: ranks of y within each u slab
    slab = np.minimum((uv[:, 0].astype(np.float64) * g).astype(int), g - 1)
    for s in range(g):
        idx = np.nonzero(slab == s)[0]
        v = np.sort(uv[idx, 1])
        assert np.array_equal(v, ((np.arange(idx.size) + 0.5) / idx.size).astype(np.float32))
        oy = idx[np.argsort(uv[idx, 1])]
        assert (np.diff(c[oy, 1]) > -1e-6).all()


@pytest.mark.parametrize("flags", [0, 0x8, 0x1])   # user order, internal order, float mesh
def test_learned_start_finds_the_oracles_elements(S, C, orc, flags):
    xy, tri, fld, dt = _swirl_case()
    xy, tri = I.permute_mesh(xy, tri, 9)
    mesh = S.Mesh(C, xy, tri, flags)
    with pytest.raises(S.SlwError):
        mesh.step(fld, 0.0, dt, S.SLW_RK2, dev(I.gaussian_hill(xy)[:, None]), start_mode=S.START_LEARNED)
    mesh.chart_build(64)
    net = S.Mlp(C, seed=8)
    # training pairs from four steps of the plain walk
    import torch
    X = torch.empty((4 * mesh.n_dofs, 5), dtype=torch.float32, device="cuda:0")
    Y = torch.empty((4 * mesh.n_dofs, 2), dtype=torch.float32, device="cuda:0")
    ids = torch.arange(mesh.n_dofs, dtype=torch.int32, device="cuda:0")
    for s in range(4):
        sl = slice(s * mesh.n_dofs, (s + 1) * mesh.n_dofs)
        mesh.learned_gather(fld, (s + 1) * dt, dt, S.SLW_RK2, ids, X[sl], Y[sl])
    assert (~np.isnan(host(Y)[:, 0])).mean() > 0.9
    net.fit_normalization(X)
    net.train(X, Y, epochs=40, batch=256, lr=3e-3, seed=3)
    mesh.attach_mlp(net)
    t_np1 = 2.5 * dt
    f_ref = orc.feet(xy, fld, t_np1, dt, I.SCHEME_RK2)
    perm = mesh.dof_order() if flags & 0x8 else np.arange(mesh.n_dofs)
    cd = np.float32 if flags & 0x1 else np.float64
    feet = f_ref.astype(cd)
    e_ref, b_ref = orc.locate(xy.astype(cd).astype(np.float64), tri, feet.astype(np.float64))
    # the network's time input is t_{n+1}
    out_l = mesh.locate_feet(t_np1=t_np1, dt=dt, feet=dev(feet[perm]), feet_in=True, start_mode=S.START_LEARNED,
                             want_steps=True, stats=True)
    out_s = mesh.locate_feet(feet=dev(feet[perm]), feet_in=True, want_steps=True, stats=True)
    out_c = mesh.locate_feet(feet=dev(feet[perm]), feet_in=True, start_mode=S.START_CHART, want_steps=True,
                             stats=True)
    out_i = mesh.locate_feet(t_np1=t_np1, dt=dt, feet=dev(feet[perm]), feet_in=True,
                             start_mode=S.START_LEARNED_INDEX, want_steps=True, stats=True)
    assert np.array_equal(host(out_l["elem"]), e_ref[perm])
    assert np.array_equal(host(out_s["elem"]), e_ref[perm])
    assert np.array_equal(host(out_c["elem"]), e_ref[perm])
    assert np.array_equal(host(out_i["elem"]), e_ref[perm])
    # the learned index's searches end in the exact chart cell: the same starts, the same walks
    assert np.array_equal(host(out_i["steps"]), host(out_c["steps"]))
    # the exact chart cell starts within a few steps of the foot
    assert out_c["stats"]["walk_steps"] < 0.2 * out_s["stats"]["walk_steps"], (out_c["stats"], out_s["stats"])
    if not flags & 0x1:
        inside = e_ref[perm] >= 0
        assert np.abs(host(out_l["bary"])[inside] - b_ref[perm][inside]).max() < 1e-12
    # fewer steps than the steered start at Courant 20
    assert out_l["stats"]["walk_steps"] < 0.5 * out_s["stats"]["walk_steps"], (out_l["stats"], out_s["stats"])
    # fused step: learned and steered starts give identical bits
    v0 = I.gaussian_hill(xy)[perm][:, None]
    a = host(mesh.step(fld, 1.5 * dt, dt, S.SLW_RK2, dev(v0), start_mode=S.START_LEARNED))
    b = host(mesh.step(fld, 1.5 * dt, dt, S.SLW_RK2, dev(v0)))
    c = host(mesh.step(fld, 1.5 * dt, dt, S.SLW_RK2, dev(v0), start_mode=S.START_CHART))
    i = host(mesh.step(fld, 1.5 * dt, dt, S.SLW_RK2, dev(v0), start_mode=S.START_LEARNED_INDEX))
    assert np.array_equal(a, b)
    assert np.array_equal(c, b)
    assert np.array_equal(i, b)


def test_untrained_network_is_still_exact(S, C, orc):
    xy, tri, fld, dt = _swirl_case(n=50, alpha=5.0, seed=902)
    p2 = orc.P2Dofs(xy, tri)
    mesh = S.Mesh(C, xy, tri, S.P2)
    mesh.chart_build(8)
    net = S.Mlp(C, seed=9)                        # random weights, identity normalisation
    mesh.attach_mlp(net)
    v0 = I.gaussian_hill(p2.xy)[:, None]
    v = host(mesh.step(fld, 0.0, dt, S.SLW_EULER, dev(v0), order=2, start_mode=S.START_LEARNED))
    ref, _, _, _ = orc.sl_step(xy, tri, v0, fld, 0.0, dt, I.SCHEME_EULER, order=2, p2=p2)
    assert np.abs(v - ref).max() <= 1e-12 * np.abs(v0).max()
    v = host(mesh.step(fld, 0.0, dt, S.SLW_EULER, dev(v0), order=2, start_mode=S.START_CHART))
    assert np.abs(v - ref).max() <= 1e-12 * np.abs(v0).max()
    # an untrained network as the guess of the learned index: still the exact cell
    v = host(mesh.step(fld, 0.0, dt, S.SLW_EULER, dev(v0), order=2, start_mode=S.START_LEARNED_INDEX))
    assert np.abs(v - ref).max() <= 1e-12 * np.abs(v0).max()
    mesh.attach_mlp(None)
    with pytest.raises(S.SlwError):
        mesh.step(fld, 0.0, dt, S.SLW_EULER, dev(v0), order=2, start_mode=S.START_LEARNED)
