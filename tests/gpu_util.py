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
