"""Pools in two-step tiles (LBM_TILE_TWO_STEP: each batched launch takes two
steps of every listed lattice, the first held in LDS). Their results are
bitwise those of the single-step batched kernels: uneven lattices (sub-tile
and ragged), per-slot step counts (an odd count takes its last step alone),
several calls in a row (each slot's buffer phase), grouped, graph and
persistent modes,
the no-allocation entry point, reads after two-step calls, switching tiles
and modes between calls, and the shape errors."""
import numpy as np
import pytest

from gpu_util import smooth_random_state

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0707_2437_amd as lbm  # noqa: E402

TWO, NT = 32, 2
SPECS = [(3, 3), (5, 4), (64, 64), (130, 77), (300, 41), (257, 129), (700, 333)]
CALLS = [[2, 3, 1, 0, 4, 5, 7], [1, 1, 1, 1, 1, 1, 1], [6, 2, 3, 4, 0, 1, 2]]
SINGLE = (2, 8, NT)


def make_pool(dtype, tile, mode=lbm.GROUPED):
    P = lbm.Pool(1 << 30, dtype)
    P.set_mode(mode)
    if tile:
        P.set_tile(*tile)
    slots = []
    for k, (nx, ny) in enumerate(SPECS):
        s = P.add(nx, ny, 0.6 + 0.05 * k, 0.1 + 0.05 * k)
        P.init(s, *smooth_random_state(nx, ny, seed=k))
        slots.append(s)
    return P, slots


def run(dtype, tile, mode=lbm.GROUPED, calls=CALLS, noalloc=False):
    P, slots = make_pool(dtype, tile, mode)
    with P:
        for n in calls:
            (P.step_noalloc if noalloc else P.step)(slots, np.array(n, dtype=np.int32))
        return ([P.get_f(s) for s in slots], [P.totals(s)[0] for s in slots], [P.time(s) for s in slots],
                P.get_tile())


@pytest.mark.parametrize("dtype", ["f64", "f32", "f32s", "f16s"])
def test_pool_two_step_bitwise(dtype):
    ref_f, ref_tot, ref_t, _ = run(dtype, (4, 8, NT) if dtype == "f16s" else SINGLE)
    assert ref_t == [sum(c[k] for c in CALLS) for k in range(len(SPECS))]
    shapes = [(1, 12, TWO | NT), (1, 16, TWO | NT), (2, 12, TWO | NT), (2, 16, TWO | NT)]
    for vx, nw, fl in shapes:
        for mode in (lbm.GROUPED, lbm.GRAPH):
            f, tot, t, tile = run(dtype, (vx, nw, fl), mode)
            assert tile == (vx, nw, fl)
            assert t == ref_t
            for k in range(len(SPECS)):
                assert np.array_equal(f[k], ref_f[k]), (dtype, vx, nw, mode, SPECS[k])
                assert np.array_equal(tot[k], ref_tot[k])


def test_pool_two_step_noalloc_bitwise():
    ref_f, _, _, _ = run("f32", SINGLE)
    f, _, _, _ = run("f32", (2, 16, TWO | NT), noalloc=True)
    assert all(np.array_equal(a, b) for a, b in zip(f, ref_f))


def test_pool_switching_tiles_and_modes_between_calls():
    """Two-step and single-step calls in any order, and a switch to the
    persistent mode (which takes single steps), keep every slot's state
    where the next call looks for it."""
    ref_f, _, _, _ = run("f32", SINGLE)
    P, slots = make_pool("f32", (2, 16, TWO | NT))
    with P:
        P.step(slots, np.array(CALLS[0], dtype=np.int32))
        P.set_tile(*SINGLE)
        P.step(slots, np.array(CALLS[1], dtype=np.int32))
        P.set_tile(1, 16, TWO)
        P.set_mode(lbm.PERSISTENT)  # two-step passes between grid barriers
        assert P.get_tile() == (1, 16, TWO)
        P.step(slots, np.array(CALLS[2], dtype=np.int32))
        got = [P.get_f(s) for s in slots]
    assert all(np.array_equal(a, b) for a, b in zip(got, ref_f))


@pytest.mark.parametrize("dtype,tile", [("f64", (2, 16, TWO | NT)), ("f32", (2, 16, TWO | NT)),
                                        ("f32", (1, 12, TWO))])
@pytest.mark.parametrize("max_grid", [0, 3])
def test_pool_two_step_persistent_bitwise(dtype, tile, max_grid):
    """One persistent launch per call in two-step tiles (all members, or 3
    workgroups taking every item), across consecutive calls with per-slot
    odd and even counts, equals the single-step grouped pool."""
    ref_f, ref_tot, ref_t, _ = run(dtype, SINGLE)
    P, slots = make_pool(dtype, tile, lbm.PERSISTENT)
    with P:
        P.set_mode(lbm.PERSISTENT, max_grid)
        for n in CALLS:
            P.step(slots, np.array(n, dtype=np.int32))
        P.sync()
        got = [P.get_f(s) for s in slots]
        members = P.persistent_members()
        assert [P.time(s) for s in slots] == ref_t
    assert (members == 3) if max_grid == 3 else (members >= 8)
    assert all(np.array_equal(a, b) for a, b in zip(got, ref_f))


def test_pool_two_step_reinit_and_readd():
    """init resets a slot's buffer phase; a slot removed and added again
    starts from its own init."""
    P, slots = make_pool("f32", (2, 16, TWO | NT))
    with P:
        P.step(slots, 3)
        nx, ny = SPECS[3]
        P.init(slots[3], *smooth_random_state(nx, ny, seed=3))
        P.remove(slots[4])
        s4 = P.add(*SPECS[4], 0.8, 0.3)
        P.init(s4, *smooth_random_state(*SPECS[4], seed=44))
        P.step([slots[3], s4], 5)
        a, b = P.get_f(slots[3]), P.get_f(s4)
    Q, qs = make_pool("f32", SINGLE)
    with Q:
        Q.step([qs[3]], 5)
        ra = Q.get_f(qs[3])
        Q.remove(qs[4])
        q4 = Q.add(*SPECS[4], 0.8, 0.3)
        Q.init(q4, *smooth_random_state(*SPECS[4], seed=44))
        Q.step([q4], 5)
        rb = Q.get_f(q4)
    assert np.array_equal(a, ra) and np.array_equal(b, rb)


def test_pool_two_step_shape_errors():
    with lbm.Pool(1 << 26, "f32") as P:
        for bad in ((4, 16, TWO), (2, 8, TWO), (2, 16, TWO | 1), (2, 16, 64), (1, 32, TWO)):
            with pytest.raises(lbm.LBMError):
                P.set_tile(*bad)
        P.set_tile(2, 16, TWO | 16 | NT)  # the vertical-stack bit is accepted
        assert P.get_tile() == (2, 16, TWO | NT)
    with lbm.Pool(1 << 26, "f16s") as P:  # FP16 storage has the two-step form too
        assert P.get_tile() == (4, 8, NT)  # its default stays single-step
        P.set_tile(2, 16, TWO)
        P.set_mode(lbm.PERSISTENT)
        assert P.get_tile() == (2, 16, TWO)
