"""lbm_pool_step_noalloc (no device allocation in the call, batch
descriptors in a fixed device array) against lbm_pool_step: bitwise the
same populations, on two calls in a row, the second with a smaller batch,
in each pool mode (graph mode launches grouped); a batch beyond the array's limits is
refused and leaves the slots unstepped."""
import ctypes

import numpy as np
import pytest

from gpu_util import smooth_random_state

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0707_2437_amd as lbm  # noqa: E402

FIRST = [(130, 77, 0.6, 0.81, 40), (64, 300, 1.2, 0.04, 17), (257, 129, 0.55, 0.3, 33), (5, 200, 0.8, 0.2, 40),
         (600, 64, 0.9, 0.5, 25)]
SECOND = [(40, 30, 0.7, 0.4, 12), (3, 3, 0.7, 0.5, 9)]  # fewer and smaller lattices


def run(step_name, mode, cases_list):
    out = []
    with lbm.Pool(1 << 30, "f32") as P:
        P.set_mode(mode)
        for cases in cases_list:
            fields = [smooth_random_state(nx, ny, seed=7 * k + nx) for k, (nx, ny, *_) in enumerate(cases)]
            slots = [P.add(nx, ny, tau, c2) for (nx, ny, tau, c2, _) in cases]
            for s, f in zip(slots, fields):
                P.init(s, *f)
            getattr(P, step_name)(slots, [c[4] for c in cases])
            out.append([P.get_f(s) for s in slots])
            for s in slots:
                P.remove(s)
    return out


@pytest.mark.parametrize("mode", [lbm.GROUPED, lbm.GRAPH, lbm.PERSISTENT])
def test_step_noalloc_equals_step(mode):
    ref = run("step", mode, [FIRST, SECOND])
    got = run("step_noalloc", mode, [FIRST, SECOND])
    for call in range(2):
        assert len(ref[call]) == len(got[call])
        for a, b in zip(ref[call], got[call]):
            assert np.array_equal(a, b), (mode, call)


def test_step_noalloc_refuses_too_many_lattices():
    with lbm.Pool(1 << 30, "f32") as P:
        slots = [P.add(3, 3, 0.7, 0.5) for _ in range(4097)]
        rho = torch.ones(9, dtype=torch.float64, device="cuda")
        for s in slots:
            P.init_device(s, rho, None, None)
        with pytest.raises(lbm.LBMError) as ei:
            P.step_noalloc(slots, 1)
        assert ei.value.status == lbm.EINVAL
        assert all(P.time(s) == 0 for s in slots)
        P.step_noalloc(slots[:4096], 1)  # at the limit
        assert P.time(slots[0]) == 1 and P.time(slots[4096]) == 0
