"""slw_step_autotune: the knob of each start mode (lane schedule, hybrid
threshold, strategy (c) forest or chain) and then the XCD chunk chosen among
bit-identical candidates, applied to the mesh, cached; the caller's values
and previous elements untouched."""
import json

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


def test_step_autotune_modes_cache_and_state(S, C, tmp_path):
    w = I.swirl_500(alpha=20.0, order="random", n=200)
    cache = tmp_path / "step_tune.json"
    twin = S.Mesh(C, w.xy, w.tri)
    mesh = S.Mesh(C, w.xy, w.tri)
    mesh.chart_build(256)
    twin.chart_build(256)
    v0 = w.v0.astype(np.float32)
    vin = dev(v0)
    before = host(vin).copy()
    ref = host(mesh.step(w.field, 0.3, w.dt, w.scheme, vin)).copy()
    choices = {}
    for mode, allowed in ((S.START_STEERED, (1, 2, 4, 8)), (S.START_NEIGHBOR, (0, 2, 4, 8, 16)),
                          (S.START_HYBRID, (0.5, 1, 2, 4, 8, 16, 32, 64))):
        if mode == S.START_HYBRID:
            # previous elements from an earlier step, on both meshes
            mesh.step(w.field, 0.1, w.dt, w.scheme, vin, start_mode=mode)
            twin.step(w.field, 0.1, w.dt, w.scheme, vin, start_mode=mode)
        val, chunk, ms = mesh.autotune_step(w.field, 0.3, w.dt, w.scheme, vin, start_mode=mode, cache_path=cache,
                                            with_chunk=True)
        assert val in allowed and chunk in (0, 16, 32, 64, 128) and ms > 0
        choices[mode] = (val, chunk)
        v, st = mesh.step(w.field, 0.3, w.dt, w.scheme, vin, start_mode=mode, stats=True)
        assert np.array_equal(host(v), ref), mode
        if mode == S.START_HYBRID:
            # the previous elements were restored: the twin (same history, same threshold) walks the same
            twin.set_hybrid(val)
            twin.set_xcd_chunk(chunk)
            _, st2 = twin.step(w.field, 0.3, w.dt, w.scheme, vin, start_mode=mode, stats=True)
            assert st == st2
    assert np.array_equal(host(vin), before)
    data = json.loads(cache.read_text())
    assert len(data) == 3
    assert all("xcd_chunk" in e and "lds_window" in e for e in data.values())
    assert all(e["lds_window"] in (0, 256, 512, 768) for e in data.values())
    # a second call answers from the cache, with the same choice, on a
    # mesh whose XCD chunk was changed meanwhile
    for mode, (val, chunk) in choices.items():
        if mode == S.START_HYBRID:
            mesh.step(w.field, 0.1, w.dt, w.scheme, vin, start_mode=mode)
        mesh.set_xcd_chunk(3)
        got = mesh.autotune_step(w.field, 0.3, w.dt, w.scheme, vin, start_mode=mode, cache_path=cache, with_chunk=True)
        assert got[:2] == (val, chunk)
    assert len(json.loads(cache.read_text())) == 3
