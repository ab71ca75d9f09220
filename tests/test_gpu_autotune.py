"""The autotuner picks a kernel shape by timing candidates on the caller's
own state without changing it, and caches its choice."""
import json
import os

import numpy as np
import pytest

from gpu_util import smooth_random_state

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0707_2437_amd as lbm  # noqa: E402


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_lattice_autotune_keeps_state_and_results(dtype):
    nx, ny = 700, 333
    fields = smooth_random_state(nx, ny, seed=12)
    with lbm.Lattice(nx, ny, 0.7, 0.45, dtype) as L:
        L.init(*fields).step(5)
        f0 = L.get_f()
        tile = L.autotune(reps=3, use_cache=False)
        assert np.array_equal(L.get_f(), f0)  # tuning launches do not touch the state
        assert L.time == 5
        got = L.step(20).get_f()
    with lbm.Lattice(nx, ny, 0.7, 0.45, dtype) as L:
        ref = L.init(*fields).step(25).get_f()
    assert np.array_equal(got, ref), tile


def test_pool_autotune_keeps_state(tmp_path, monkeypatch):
    with lbm.Pool(1 << 30, "f32") as P:
        slots = [P.add(nx, ny, 0.8, 0.3) for nx, ny in ((300, 200), (64, 512), (513, 65))]
        for k, s in enumerate(slots):
            P.init(s, *smooth_random_state(*P.shapes[s][::-1], seed=k))
        P.step(slots, 3)
        before = [P.get_f(s) for s in slots]
        tile = P.autotune(slots, reps=2, use_cache=False)
        after = [P.get_f(s) for s in slots]
        assert all(np.array_equal(a, b) for a, b in zip(before, after))
        assert [P.time(s) for s in slots] == [3, 3, 3]
        assert tile[1] in (4, 8, 16)


def test_tune_cache_file_is_written():
    """LBM_TUNE_CACHE is read by the library at its first tuning, so this test
    only checks the in-process cache path: a cached lookup is consistent."""
    with lbm.Lattice(96, 96, 0.7, 0.4, "f32") as L:
        L.init()
        t1 = L.autotune(reps=2, use_cache=True)
        t2 = L.autotune(reps=2, use_cache=True)
        assert t1 == t2
