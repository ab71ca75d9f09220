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
        assert tile[1] in (4, 8, 12, 16)


_TUNE_CHILD = """
import json, sys
import numpy as np
import paper_0707_2437_amd as lbm
from paper_0707_2437_amd import workloads
with lbm.Lattice(96, 96, 0.7, 0.4, "f32") as L:
    L.init(*workloads.plane_wave_fields(96, 96, 0.4, seed=1))
    tile = L.autotune(reps=2, use_cache=True)
    np.save(sys.argv[1], L.step(5).get_f())
print(json.dumps(list(tile)))
"""


def _tune_child(cache, out):
    import subprocess
    import sys
    env = dict(os.environ, LBM_TUNE_CACHE=str(cache))
    r = subprocess.run([sys.executable, "-c", _TUNE_CHILD, str(out)], env=env, capture_output=True, text=True,
                       timeout=300, cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert r.returncode == 0, r.stderr
    return tuple(json.loads(r.stdout.strip().splitlines()[-1]))


def test_tune_cache_file_round_trip(tmp_path):
    """LBM_TUNE_CACHE names a file of tuned shapes, one JSON object per line,
    read at a process's first tuning, later lines overriding earlier ones.
    A fresh process tunes a 96² FP32 lattice and appends its pick; a second
    fresh process, given the file with a later line naming another shape for
    the same key, applies that shape without timing anything (no line is
    added), and its state after 5 steps is bitwise the first process's."""
    cache = tmp_path / "tune.jsonl"
    t1 = _tune_child(cache, tmp_path / "f1.npy")
    lines = cache.read_text().splitlines()
    assert len(lines) == 1
    rec = json.loads(lines[0])
    assert rec["key"].split("|")[1:] == ["lattice", "1", "96x96"] and rec["key"].startswith("gfx")
    assert (rec["vx"], rec["nw"], rec["h"], rec["flags"]) == t1 and rec["us"] > 0
    other = (4, 16, 8, 16) if t1[:2] != (4, 16) else (1, 4, 8, 16)  # vertical stack, plain stores
    with open(cache, "a") as fh:
        fh.write(json.dumps({"key": rec["key"], "vx": other[0], "nw": other[1], "h": other[2], "flags": other[3],
                             "ch": 0, "us": 1.0}) + "\n")
    t2 = _tune_child(cache, tmp_path / "f2.npy")
    assert t2 == other
    assert len(cache.read_text().splitlines()) == 2
    assert np.array_equal(np.load(tmp_path / "f1.npy"), np.load(tmp_path / "f2.npy"))
