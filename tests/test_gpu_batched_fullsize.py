"""Parity of the batching workload at its full size, in the configuration the
benchmark times: 256 seeded periodic lattices (nx, ny ~ U{64..1024}, tau,
c^2 and a Gaussian density pulse of amplitude up to 0.1 each), FP32, one
pool in graph mode with the autotuned tile, 2000 steps in one call.

- Every lattice against the plain single-lattice kernel stepping it alone:
  every population of the final state is bitwise equal, and so are the
  FP64 totals (a fixed-order reduction of the state).
- A seeded subset against the FP64 oracle (Eq. 5 stepped in full): the 16
  smallest lattices and 4 drawn at random among those of at most 512^2
  sites (the bound keeps the oracle's share of the test to seconds). FP32
  bound: 1e-5 max relative error in f per 1000 steps (the FP32 error of the
  plain kernel grows linearly with the step count), so 2e-5 here.
- Every lattice: finite totals, and mass conserved within the worst case of
  one FP32 rounding (2^-24 relative) of every stored population per step.
"""
import numpy as np
import pytest

import oracle
from gpu_util import max_rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0707_2437_amd as lbm  # noqa: E402
from paper_0707_2437_amd import workloads  # noqa: E402

STEPS = 2000
TOL_F32 = 1e-5 * STEPS / 1000


def oracle_subset(specs, seed=7):
    order = sorted(range(len(specs)), key=lambda k: specs[k]["nx"] * specs[k]["ny"])
    small = order[:16]
    rest = [k for k in order[16:] if specs[k]["nx"] * specs[k]["ny"] <= 512 * 512]
    rng = np.random.default_rng(seed)
    return small + [int(k) for k in rng.choice(rest, 4, replace=False)]


def test_batched_full_size_against_plain_kernel_and_oracle():
    specs = workloads.batch_specs(256, seed=0)
    stream = torch.cuda.Stream()
    budget = sum(lbm.Pool.slot_bytes(s["nx"], s["ny"], "f32") for s in specs)
    subset = oracle_subset(specs)
    with lbm.Pool(budget, "f32") as P:
        P.set_stream(stream)
        P.set_mode(lbm.GRAPH)
        slots = []
        for sp in specs:
            s = P.add(sp["nx"], sp["ny"], sp["tau"], sp["c2"])
            P.init(s, *workloads.batch_fields(sp))
            slots.append(s)
        tot0 = [P.totals(s)[0] for s in slots]
        tile = P.autotune(slots, reps=5)
        print(f"tile {tile}", flush=True)
        P.step(slots, STEPS)
        P.sync()
        tot = [P.totals(s) for s in slots]
        assert all(st == 0 for _, st in tot), "non-finite totals"

        # mass: at most one FP32 rounding of each stored population per step
        drift = max(abs(t[0][0] - m0[0]) / m0[0] for t, m0 in zip(tot, tot0))
        print(f"max relative mass drift over 256 lattices: {drift:.2e}", flush=True)
        assert drift <= STEPS * 2.0 ** -24

        # every lattice, bitwise, against the plain kernel stepping it alone
        got = {}
        for k, sp in enumerate(specs):
            with lbm.Lattice(sp["nx"], sp["ny"], sp["tau"], sp["c2"], "f32") as L:
                L.set_stream(stream)
                L.init(*workloads.batch_fields(sp)).step(STEPS)
                alone_tot = L.totals()
                alone_f = L.get_f()
            f = P.get_f(slots[k])
            assert np.array_equal(alone_f, f), (k, sp)
            assert np.array_equal(np.asarray(alone_tot), np.asarray(tot[k][0])), (k, sp)
            if k in subset:
                got[k] = f
        print("all 256 lattices bitwise equal to the plain kernel", flush=True)

    # the seeded subset against the FP64 oracle
    oracle.set_threads(0)
    worst = 0.0
    for k in subset:
        sp = specs[k]
        ref = oracle.Oracle(sp["nx"], sp["ny"], sp["tau"], sp["c2"]).init(*workloads.batch_fields(sp)) \
            .step(STEPS).get_f()
        err = max_rel_err(got[k], ref)
        worst = max(worst, err)
        print(f"lattice {k} {sp['nx']}x{sp['ny']} tau {sp['tau']:.3f} c2 {sp['c2']:.3f} amp {sp['amp']:.3f}: "
              f"max rel err {err:.2e}", flush=True)
        assert err <= TOL_F32, (k, sp, err)
    print(f"worst over {len(subset)} lattices: {worst:.2e}")


def test_batched_full_size_one_persistent_launch():
    """The same workload as one persistent launch of 2000 steps (its own
    autotuned shape): every lattice's populations bitwise equal to the graph
    mode's, which the test above ties to the plain kernel and the oracle."""
    specs = workloads.batch_specs(256, seed=0)
    stream = torch.cuda.Stream()
    budget = sum(lbm.Pool.slot_bytes(s["nx"], s["ny"], "f32") for s in specs)
    states = {}
    for mode in (lbm.GRAPH, lbm.PERSISTENT):
        with lbm.Pool(budget, "f32") as P:
            P.set_stream(stream)
            P.set_mode(mode)
            slots = []
            for sp in specs:
                s = P.add(sp["nx"], sp["ny"], sp["tau"], sp["c2"])
                P.init(s, *workloads.batch_fields(sp))
                slots.append(s)
            tile = P.autotune(slots, reps=3)
            P.step(slots, STEPS)
            P.sync()
            if mode == lbm.PERSISTENT:
                print(f"persistent tile {tile}, {P.persistent_members()} workgroups", flush=True)
            states[mode] = [P.get_f(s) for s in slots]
    for k, (a, b) in enumerate(zip(states[lbm.GRAPH], states[lbm.PERSISTENT])):
        assert np.array_equal(a, b), (k, specs[k])
    print("all 256 lattices bitwise equal in graph and persistent modes", flush=True)
