"""Batched form: a pool of lattices of uneven size, tau and c^2 stepped by
batched launches (grouped, captured hipGraph, persistent) gives
every lattice bitwise the result of stepping it alone; the pool enforces its
memory budget; errors are reported."""
import numpy as np
import pytest

import oracle
from gpu_util import max_rel_err, smooth_random_state

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0707_2437_amd as lbm  # noqa: E402

# (nx, ny, tau, c2, steps): tiny, ragged, tall, wide, several tiles
CASES = [(3, 3, 0.7, 0.5, 40), (130, 77, 0.6, 0.81, 40), (64, 300, 1.2, 0.04, 17), (333, 41, 0.9, 1.0 / 3.0, 0),
         (257, 129, 0.55, 0.3, 33), (5, 200, 0.8, 0.2, 40)]


def run_alone(nx, ny, tau, c2, steps, dtype, fields):
    with lbm.Lattice(nx, ny, tau, c2, dtype) as L:
        return L.init(*fields).step(steps).get_f()


@pytest.mark.parametrize("mode", [lbm.GROUPED, lbm.GRAPH, lbm.PERSISTENT])
@pytest.mark.parametrize("dtype", ["f64", "f32", "f16s"])
def test_batched_equals_alone_bitwise(dtype, mode):
    fields = [smooth_random_state(nx, ny, seed=17 * k + 1) for k, (nx, ny, *_) in enumerate(CASES)]
    with lbm.Pool(4 << 30, dtype) as P:
        P.set_mode(mode)
        slots = [P.add(nx, ny, tau, c2) for (nx, ny, tau, c2, _) in CASES]
        for s, f in zip(slots, fields):
            P.init(s, *f)
        P.step(slots, [c[4] for c in CASES])
        # a second call with the same shape replays the captured graph
        P.step(slots, [c[4] for c in CASES])
        got = [P.get_f(s) for s in slots]
        times = [P.time(s) for s in slots]
    for (nx, ny, tau, c2, n), f, g, t in zip(CASES, fields, got, times):
        assert t == 2 * n
        assert np.array_equal(g, run_alone(nx, ny, tau, c2, 2 * n, dtype, f)), (nx, ny)


def test_persistent_with_few_workgroups_bitwise():
    """Persistent mode with 4 workgroups: each strides over many tiles and
    waits at the grid barrier every step."""
    fields = [smooth_random_state(nx, ny, seed=k) for k, (nx, ny, *_) in enumerate(CASES)]
    with lbm.Pool(1 << 30, "f32") as P:
        P.set_mode(lbm.PERSISTENT, max_grid=4)
        slots = [P.add(nx, ny, tau, c2) for (nx, ny, tau, c2, _) in CASES]
        for s, f in zip(slots, fields):
            P.init(s, *f)
        P.step(slots, [c[4] for c in CASES])
        assert 1 <= P.persistent_members() <= 4
        got = [P.get_f(s) for s in slots]
    for (nx, ny, tau, c2, n), f, g in zip(CASES, fields, got):
        assert np.array_equal(g, run_alone(nx, ny, tau, c2, n, "f32", f))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("vx,nw", [(1, 4), (1, 8), (2, 4), (2, 16), (4, 16)])
def test_persistent_every_shape_bitwise(dtype, vx, nw):
    """A persistent launch in every tile shape. The runtime's report of how
    many workgroups a CU holds at once can be too high (the FP32 (1, 4)
    kernel's scalar registers allow 7 waves per SIMD, and a launch sized by
    the report timed out at its first grid barrier); the workgroups that are
    not resident when the launch starts take no part, and every lattice is
    still bitwise the plain kernel's."""
    fields = [smooth_random_state(nx, ny, seed=5 * k + 2) for k, (nx, ny, *_) in enumerate(CASES)]
    with lbm.Pool(1 << 30, dtype) as P:
        P.set_tile(vx, nw, 2)
        P.set_mode(lbm.PERSISTENT)
        slots = [P.add(nx, ny, tau, c2) for (nx, ny, tau, c2, _) in CASES]
        for s, f in zip(slots, fields):
            P.init(s, *f)
        P.step(slots, [c[4] for c in CASES])
        P.sync()
        # every CU holds at least one workgroup of these shapes, and the
        # resident workgroups all join before membership closes
        assert P.persistent_members() >= torch.cuda.get_device_properties(0).multi_processor_count
        got = [P.get_f(s) for s in slots]
    for (nx, ny, tau, c2, n), f, g in zip(CASES, fields, got):
        assert np.array_equal(g, run_alone(nx, ny, tau, c2, n, dtype, f)), (nx, ny)


def test_persistent_beside_a_running_kernel_bitwise():
    """A persistent launch made while another stream's kernels hold part of
    the GPU (a 4096^2 lattice stepping on a second stream): the workgroups
    that are resident when it starts take part, the others end, and every
    lattice is still bitwise the plain kernel's."""
    fields = [smooth_random_state(nx, ny, seed=3 * k + 4) for k, (nx, ny, *_) in enumerate(CASES)]
    other = torch.cuda.Stream()
    mine = torch.cuda.Stream()
    with lbm.Lattice(4096, 4096, 0.6, 0.2, "f32") as big, lbm.Pool(1 << 30, "f32") as P:
        big.set_stream(other)
        big.init()
        P.set_stream(mine)
        P.set_mode(lbm.PERSISTENT)
        slots = [P.add(nx, ny, tau, c2) for (nx, ny, tau, c2, _) in CASES]
        for s, f in zip(slots, fields):
            P.init(s, *f)
        torch.cuda.synchronize()
        big.step(200)  # about 40 ms of work queued on the other stream
        P.step(slots, [c[4] for c in CASES])
        P.sync()
        members = P.persistent_members()
        got = [P.get_f(s) for s in slots]
        torch.cuda.synchronize()
    assert members >= 1
    for (nx, ny, tau, c2, n), f, g in zip(CASES, fields, got):
        assert np.array_equal(g, run_alone(nx, ny, tau, c2, n, "f32", f)), (nx, ny)


@pytest.mark.parametrize("tile,per_item", [((1, 4, 0), 1), ((2, 16, 2), 3), ((4, 8, 0), 8), ((2, 8, 2), 64)])
def test_pool_tile_does_not_change_results(tile, per_item):
    fields = [smooth_random_state(nx, ny, seed=k) for k, (nx, ny, *_) in enumerate(CASES)]
    with lbm.Pool(1 << 30, "f64") as P:
        P.set_tile(*tile)
        P.set_items(per_item)
        slots = [P.add(nx, ny, tau, c2) for (nx, ny, tau, c2, _) in CASES]
        for s, f in zip(slots, fields):
            P.init(s, *f)
        P.step(slots, 25)
        got = [P.get_f(s) for s in slots]
    for (nx, ny, tau, c2, _), f, g in zip(CASES, fields, got):
        assert np.array_equal(g, run_alone(nx, ny, tau, c2, 25, "f64", f))


def test_pool_members_match_oracle():
    cases = [(48, 36, 0.7, 0.5), (31, 64, 0.6, 0.9)]
    with lbm.Pool(1 << 30, "f64") as P:
        slots, refs = [], []
        for k, (nx, ny, tau, c2) in enumerate(cases):
            f = smooth_random_state(nx, ny, seed=40 + k)
            s = P.add(nx, ny, tau, c2)
            P.init(s, *f)
            slots.append(s)
            refs.append(oracle.Oracle(nx, ny, tau, c2).init(*f).step(200).get_f())
        P.step(slots, 200)
        for s, r in zip(slots, refs):
            assert max_rel_err(P.get_f(s), r) <= 1e-12


def test_budget_admission_and_slot_reuse():
    b = lbm.Pool.slot_bytes(256, 256, "f32")
    with lbm.Pool(3 * b, "f32") as P:
        s = [P.add(256, 256, 0.8, 0.3) for _ in range(3)]
        assert P.used_bytes == 3 * b
        assert P.try_add(256, 256, 0.8, 0.3) is None  # over budget
        with pytest.raises(lbm.LBMError) as ei:
            P.add(256, 256, 0.8, 0.3)
        assert ei.value.status == lbm.ENOMEM
        P.remove(s[1])
        assert P.used_bytes == 2 * b
        assert P.add(256, 256, 0.8, 0.3) == s[1]  # id reused


def test_freed_ranges_reused_without_crosstalk():
    """Slots are ranges of a few large device allocations: removing two
    adjacent slots and admitting larger and smaller lattices reuses (and
    merges) their ranges; every lattice then steps bitwise as it does alone,
    and initialising a new slot leaves its neighbours' state untouched."""
    shapes = [(100, 90), (64, 64), (130, 77), (257, 129), (40, 300)]
    with lbm.Pool(1 << 28, "f32") as P:
        live = {}
        for k, (nx, ny) in enumerate(shapes):
            f = smooth_random_state(nx, ny, seed=60 + k)
            s = P.add(nx, ny, 0.7, 0.3)
            P.init(s, *f)
            live[s] = (nx, ny, f, 0)
        P.step(list(live), 7)
        live = {s: (nx, ny, f, 7) for s, (nx, ny, f, _) in live.items()}
        before = {s: P.get_f(s) for s in live}
        for s in list(live)[1:3]:
            P.remove(s)
            del live[s]
        for k, (nx, ny) in enumerate([(200, 110), (33, 47), (64, 64)]):
            f = smooth_random_state(nx, ny, seed=80 + k)
            s = P.add(nx, ny, 0.9, 0.25)
            P.init(s, *f)
            live[s] = (nx, ny, f, 0)
        for s in (0, 3, 4):
            assert np.array_equal(P.get_f(s), before[s])
        P.step(list(live), 11)
        got = {s: P.get_f(s) for s in live}
    for s, (nx, ny, f, t0) in live.items():
        tau, c2 = (0.7, 0.3) if t0 else (0.9, 0.25)
        assert np.array_equal(got[s], run_alone(nx, ny, tau, c2, t0 + 11, "f32", f)), (s, nx, ny)


def test_pool_errors():
    with lbm.Pool(1 << 28, "f32") as P:
        s = P.add(32, 32, 0.8, 0.3)
        with pytest.raises(lbm.LBMError) as ei:
            P.step([s], [1])
        assert ei.value.status == lbm.ESTATE
        P.init(s)
        with pytest.raises(lbm.LBMError) as ei:
            P.step([s, s], [1, 1])
        assert ei.value.status == lbm.EINVAL
        with pytest.raises(lbm.LBMError) as ei:
            P.step([s + 7], [1])
        assert ei.value.status == lbm.EINVAL
        with pytest.raises(lbm.LBMError) as ei:
            P.add(2, 32, 0.8, 0.3)
        assert ei.value.status == lbm.EINVAL
        out = torch.zeros(3, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()  # the fill (torch's stream) before the pool's stream writes
        with pytest.raises(lbm.LBMError) as ei:
            P.totals_device(s + 7, out)  # no such slot
        assert ei.value.status == lbm.EINVAL
        with pytest.raises(lbm.LBMError) as ei:
            P.step_noalloc([s, s], [1, 1])  # a slot listed twice
        assert ei.value.status == lbm.EINVAL
        assert P.persistent_members() == 0  # no persistent launch yet
        P.totals_device(s, out)
        P.sync()
        assert np.array_equal(out.cpu().numpy(), P.totals(s)[0])


def test_nonfinite_job_detected_and_isolated():
    """A lattice with a NaN is reported by its totals and does not disturb
    the other slots stepped in the same launches."""
    with lbm.Pool(1 << 28, "f32") as P:
        good, bad = P.add(40, 30, 0.7, 0.4), P.add(40, 30, 0.7, 0.4)
        f = smooth_random_state(40, 30, seed=2)
        rho_bad = f[0].copy()
        rho_bad[5, 5] = np.nan
        P.init(good, *f)
        P.init(bad, rho_bad, f[1], f[2])
        P.step([good, bad], 30)
        assert P.totals(bad)[1] == lbm.ENONFINITE
        assert P.totals(good)[1] == 0
        ref = run_alone(40, 30, 0.7, 0.4, 30, "f32", f)
        assert np.array_equal(P.get_f(good), ref)


def test_persistent_barrier_timeout_reported(monkeypatch):
    """The grid barrier's wait is bounded in time. With the bound forced to
    zero from the host (LBM_BARRIER_WAIT_US=0), a workgroup that has to wait
    gives up at once, raises the error flag and ends; every workgroup then
    ends the launch. The next read of the pool reports LBM_EDEVICE (the
    steps are incomplete), a launch made before that read does nothing, and
    after the flag has been read the pool steps correctly again."""
    nx, ny = 200, 150
    f = smooth_random_state(nx, ny, seed=5)
    with lbm.Pool(1 << 28, "f32") as P:
        P.set_mode(lbm.PERSISTENT)
        s = P.add(nx, ny, 0.7, 0.3)
        P.init(s, *f)
        monkeypatch.setenv("LBM_BARRIER_WAIT_US", "0")
        P.step([s], [20])
        P.step([s], [5])  # finds the flag set: returns at once
        monkeypatch.delenv("LBM_BARRIER_WAIT_US")
        _, _, _, _, st = P.moments(s, fields=False, check=False)
        assert st == lbm.EDEVICE
        P.sync()  # the flag was read and cleared by the moments call
        P.init(s, *f)
        P.step([s], [20])
        P.sync()
        got = P.get_f(s)
    assert np.array_equal(got, run_alone(nx, ny, 0.7, 0.3, 20, "f32", f))
