"""The paper's walk on the host (Section 2.2, Algorithm 1; strategy (a)'s
start of Section 3), in plain FP64: `walk.c`.

TEST AND BENCHMARK INFRASTRUCTURE ONLY (walk lengths of the method as the
paper states it, and its speed on the host cores); the GPU library never
calls it.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import oracle as _orc

RULE_RANDOM = 0   # a random incident triangle (the paper's start)
RULE_SECTOR = 1   # the incident triangle whose angle at the node contains the foot direction


def _lib():
    L = _orc.lib()
    if not getattr(L, "_o3_ready", False):
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        L.o3_locate_nodes.restype = ctypes.c_int64
        L.o3_locate_nodes.argtypes = [dp, ctypes.c_int64, ip, ip, ip, ip, dp, ctypes.c_int, ctypes.c_uint64,
                                      ctypes.c_int64, ip, ip, ctypes.c_int]
        L.o3_walk.restype = ctypes.c_int64
        L.o3_walk.argtypes = [dp, ip, ip, ctypes.c_int64, dp, ip, ctypes.c_int64, ip, ip, ctypes.c_int]
        L.o3_max_threads.restype = ctypes.c_int
        L._o3_ready = True
    return L


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


class Mesh:
    """Neighbour and incidence arrays of a triangle mesh (nodes n x 2,
    triangles nt x 3, any orientation): nbr[t, k] is the triangle across the
    edge opposite vertex k (-1 on the boundary); inc[inc_ptr[i]:inc_ptr[i+1]]
    are the triangles incident to node i, in increasing id."""

    def __init__(self, xy, tri):
        self.xy = np.ascontiguousarray(xy, dtype=np.float64)
        self.tri = np.ascontiguousarray(tri, dtype=np.int32)
        n, nt = self.xy.shape[0], self.tri.shape[0]
        t = self.tri.astype(np.int64)
        a = np.concatenate([t[:, 1], t[:, 2], t[:, 0]])       # edge opposite vertex 0, 1, 2
        b = np.concatenate([t[:, 2], t[:, 0], t[:, 1]])
        key = np.minimum(a, b) * n + np.maximum(a, b)
        owner = np.concatenate([np.arange(nt)] * 3)
        k = np.repeat(np.arange(3), nt)
        order = np.argsort(key, kind="stable")
        ks, os_, kk = key[order], owner[order], k[order]
        same = np.nonzero(ks[1:] == ks[:-1])[0]
        nbr = np.full((nt, 3), -1, dtype=np.int32)
        nbr[os_[same], kk[same]] = os_[same + 1]
        nbr[os_[same + 1], kk[same + 1]] = os_[same]
        self.nbr = nbr
        flat = t.ravel()
        self.inc_ptr = np.zeros(n + 1, dtype=np.int32)
        np.add.at(self.inc_ptr, flat + 1, 1)
        self.inc_ptr = np.cumsum(self.inc_ptr).astype(np.int32)
        self.inc = (np.argsort(flat, kind="stable") // 3).astype(np.int32)

    def locate_nodes(self, q, rule=RULE_SECTOR, seed=0, threads=0, cap=1 << 22):
        """Feet q (n x 2) of every node: start by rule, walk; returns
        (elem, steps); elem -1 outside, -2 when the cap ended the walk."""
        q = np.ascontiguousarray(q, dtype=np.float64)
        n = self.xy.shape[0]
        elem = np.empty(n, np.int32)
        steps = np.empty(n, np.int32)
        _lib().o3_locate_nodes(_d(self.xy), n, _i(self.tri), _i(self.nbr), _i(self.inc_ptr), _i(self.inc), _d(q),
                               int(rule), int(seed) & (2 ** 64 - 1), int(cap), _i(elem), _i(steps), int(threads))
        return elem, steps

    def walk(self, q, start, threads=0, cap=1 << 22):
        """The walk from given start triangles; returns (elem, steps)."""
        q = np.ascontiguousarray(q, dtype=np.float64)
        start = np.ascontiguousarray(start, dtype=np.int32)
        m = q.shape[0]
        elem = np.empty(m, np.int32)
        steps = np.empty(m, np.int32)
        _lib().o3_walk(_d(self.xy), _i(self.tri), _i(self.nbr), m, _d(q), _i(start), int(cap), _i(elem), _i(steps),
                       int(threads))
        return elem, steps


def max_threads() -> int:
    return int(_lib().o3_max_threads())
