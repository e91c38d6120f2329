"""Helpers shared by the GPU tests: device setup and tolerances."""
import numpy as np


def rel_err(v, ref, scale=None):
    """max |v - ref| / max(|ref|, scale) over all entries (the value metric:
    per value |v - v_ref| <= tol * max(|v_ref|, |V^n|_inf))."""
    v = np.asarray(v, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if scale is None:
        scale = np.abs(ref).max() if ref.size else 1.0
    den = np.maximum(np.abs(ref), scale)
    den = np.where(den == 0, 1.0, den)
    return float((np.abs(v - ref) / den).max()) if ref.size else 0.0


def ctx():
    import torch
    from paper_2104_09189_amd import slwalk as S
    torch.cuda.init()
    return S.Context(0)


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _seg_dist(p, a, b):
    """distance from points p to segments a-b (rows), FP64"""
    ab = b - a
    t = np.einsum("ij,ij->i", p - a, ab) / np.maximum(np.einsum("ij,ij->i", ab, ab), 1e-300)
    t = np.clip(t, 0.0, 1.0)
    c = a + t[:, None] * ab
    return np.hypot(*(p - c).T)


def tri_distance(xy, tri, e, q):
    """distance from q[i] to the closed triangle tri[e[i]] (0 inside), FP64"""
    A, B, C = xy[tri[e, 0]], xy[tri[e, 1]], xy[tri[e, 2]]

    def o(a, b, c):
        return (a[:, 0] - c[:, 0]) * (b[:, 1] - c[:, 1]) - (a[:, 1] - c[:, 1]) * (b[:, 0] - c[:, 0])
    s = np.sign(o(A, B, C))
    inside = (o(B, C, q) * s >= 0) & (o(C, A, q) * s >= 0) & (o(A, B, q) * s >= 0)
    d = np.minimum(np.minimum(_seg_dist(q, A, B), _seg_dist(q, B, C)), _seg_dist(q, C, A))
    return np.where(inside, 0.0, d)


def check_elements_near(xy, tri, q_ref, e_ref, e_gpu, r, max_share=1e-3):
    """Index parity for feet the GPU computes itself (its feet agree with the
    oracle's feet q_ref to within r, so the query points may differ by a
    rounding).  Where the oracle's foot lies farther than r from every edge
    of its element (or, outside, farther than r from the mesh), the GPU's
    element must be the oracle's, bit for bit.  Where it lies within r of an
    edge, the GPU's element must be a triangle within r of the oracle's foot
    (-1 only if the foot is within r of the domain's outside).  At most
    max_share of the feet may pass by the second rule alone (near an edge
    and a different element from the oracle's).  Returns how many did."""
    xy = np.asarray(xy, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.int64)
    q = np.asarray(q_ref, dtype=np.float64)
    e_ref = np.asarray(e_ref, dtype=np.int64)
    e_gpu = np.asarray(e_gpu, dtype=np.int64)
    amb = np.zeros(e_ref.shape[0], dtype=bool)
    inn = e_ref >= 0
    if inn.any():
        # distance of the oracle's foot to each edge line of its element
        t = tri[e_ref[inn]]
        P = [xy[t[:, k]] for k in range(3)]
        qi = q[inn]
        dmin = np.full(qi.shape[0], np.inf)
        for k in range(3):
            a, b = P[(k + 1) % 3], P[(k + 2) % 3]
            ln = np.hypot(*(b - a).T)
            o = (a[:, 0] - qi[:, 0]) * (b[:, 1] - qi[:, 1]) - (a[:, 1] - qi[:, 1]) * (b[:, 0] - qi[:, 0])
            dmin = np.minimum(dmin, np.abs(o) / ln)
        amb[inn] = dmin <= r
    out = ~inn & np.isfinite(q).all(axis=1)
    if out.any():
        # outside: ambiguous if some triangle is within r (nearest by the GPU's answer, checked below)
        amb[out] = e_gpu[out] >= 0
    sure = ~amb
    bad = sure & (e_gpu != e_ref)
    assert not bad.any(), f"{int(bad.sum())} elements differ from the oracle (first at {np.nonzero(bad)[0][:5]})"
    ai = np.nonzero(amb & (e_gpu != e_ref))[0]
    if ai.size:
        g = e_gpu[ai]
        ok = np.zeros(ai.size, dtype=bool)
        has = g >= 0
        if has.any():
            ok[has] = tri_distance(xy, tri, g[has], q[ai[has]]) <= r
        # the GPU says outside: the oracle's foot must lie within r of the
        # domain's boundary (the tests' domains are their meshes' bounding boxes)
        lo, hi = xy.min(axis=0), xy.max(axis=0)
        qn = q[ai[~has]]
        gap = np.minimum(np.minimum(qn[:, 0] - lo[0], hi[0] - qn[:, 0]), np.minimum(qn[:, 1] - lo[1], hi[1] - qn[:, 1]))
        ok[~has] = gap <= r
        assert ok.all(), f"{int((~ok).sum())} near-edge feet got an element farther than {r} from the oracle foot"
    assert ai.size <= max_share * max(e_ref.shape[0], 1), (
        f"{ai.size} of {e_ref.shape[0]} feet near an edge got another element than the oracle's: "
        f"feet {q[ai[:4]].tolist()} oracle {e_ref[ai[:4]].tolist()} gpu {e_gpu[ai[:4]].tolist()}")
    return int(ai.size)
