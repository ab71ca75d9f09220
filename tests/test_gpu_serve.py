"""Served form: jobs arriving over time are admitted as memory frees up,
stepped together in ticks with per-job step counts, and each job's result is
bitwise the one it gets when run alone and, for a seeded sample, matches the
FP64 oracle; a job that blows up is reported as failed without disturbing
the others."""
import numpy as np
import pytest

import oracle
from gpu_util import max_rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0707_2437_amd as lbm  # noqa: E402
from paper_0707_2437_amd import serve, workloads  # noqa: E402


def alone(job):
    rho = serve.pulse_field_device(torch, job.nx, job.ny, job.amp)
    with lbm.Lattice(job.nx, job.ny, job.tau, job.c2, "f32") as L:
        L.init_device(rho, None, None)
        return L.step(job.steps).get_f()


def test_each_job_same_alone_and_in_the_mix():
    jobs = serve.job_stream(rate=40.0, duration=0.4, seed=3, side_log2=(6, 8), steps=(30, 300))
    assert len(jobs) >= 8
    budget = 3 * lbm.Pool.slot_bytes(256, 256, "f32")  # not all jobs fit at once
    srv = serve.Server(budget, "f32", tick_steps=37, keep_f=True)
    st = srv.run(jobs, duration=0.0, drain=True)
    srv.close()
    assert st["jobs_completed"] == len(jobs) and st["jobs_failed"] == 0
    assert st["ticks"] > 1
    done = {j.id: j for j in srv.finished}
    waited = sum(1 for j in done.values() if j.t_admit > j.arrival + 1e-3)
    assert waited > 0  # some jobs were admitted only after others freed memory
    for j in done.values():
        assert np.array_equal(j.f, alone(j)), j.id
        assert j.t_done >= j.t_admit >= j.arrival


def test_totals_ring_wraps_and_grows():
    """The totals of finishing jobs go through a ring of device rows copied to
    pinned host rows and read one tick later. With a ring of 4 rows and many
    short jobs, the ring wraps (after reading back the queued ticks) and
    grows (when one tick finishes more jobs than half of it); every job's
    FP64 totals are still bitwise those of the job stepped alone."""
    # all jobs arrive at once; their step counts end in six different ticks,
    # each finishing 6-7 jobs (more than half of the ring: it grows), and
    # the later ticks reuse the ring's rows (it wraps)
    rng = np.random.default_rng(11)
    jobs = [serve.Job(id=k, nx=int(rng.choice([32, 48, 64])), ny=int(rng.choice([32, 48, 64])),
                      tau=float(rng.uniform(0.6, 1.2)), c2=float(rng.uniform(0.1, 0.5)),
                      amp=float(rng.uniform(0.01, 0.05)), steps=7 * (1 + k % 6) - (k % 2), arrival=0.0)
            for k in range(40)]
    srv = serve.Server(1 << 28, "f32", tick_steps=7, ring_rows=4)
    st = srv.run(jobs, duration=0.0, drain=True)
    srv.close()
    assert st["jobs_completed"] == len(jobs)
    assert srv._ring_dev.shape[0] > 4  # it grew at least once
    for j in srv.finished:
        rho = serve.pulse_field_device(torch, j.nx, j.ny, j.amp)
        with lbm.Lattice(j.nx, j.ny, j.tau, j.c2, "f32") as L:
            L.init_device(rho, None, None)
            tot = L.step(j.steps).totals()
        assert np.array_equal(np.asarray(tot), np.asarray(j.totals)), j.id


def test_unstable_job_fails_alone():
    jobs = [serve.Job(id=0, nx=64, ny=64, tau=0.6, c2=0.3, amp=0.05, steps=200, arrival=0.0),
            serve.Job(id=1, nx=48, ny=48, tau=0.505, c2=3.0, amp=0.3, steps=2000, arrival=0.0),
            serve.Job(id=2, nx=80, ny=40, tau=0.9, c2=0.1, amp=0.02, steps=150, arrival=0.05)]
    srv = serve.Server(1 << 28, "f32", tick_steps=64, keep_f=True)
    srv.run(jobs, duration=0.0, drain=True)
    srv.close()
    by_id = {j.id: j for j in srv.finished}
    assert by_id[1].status == "failed"
    for i in (0, 2):
        assert by_id[i].status == "done"
        assert np.array_equal(by_id[i].f, alone(by_id[i]))


def test_served_jobs_match_oracle():
    """A seeded sample of jobs served in the mix (admitted as memory frees up,
    stepped in shared ticks) against the FP64 oracle stepping each job's
    lattice (Eq. 5) from the same pulse field for the same number of steps:
    FP32 bar 1e-5 max relative error in f per 1000 steps (the FP32 error of
    the plain kernel grows linearly with the step count)."""
    jobs = serve.job_stream(rate=30.0, duration=0.5, seed=5, side_log2=(6, 7), steps=(200, 1000))
    assert len(jobs) >= 8
    budget = 3 * lbm.Pool.slot_bytes(128, 128, "f32")  # not all jobs fit at once
    srv = serve.Server(budget, "f32", tick_steps=64, keep_f=True)
    st = srv.run(jobs, duration=0.0, drain=True)
    srv.close()
    assert st["jobs_completed"] == len(jobs)
    done = sorted(srv.finished, key=lambda j: j.id)
    sample = np.random.default_rng(0).choice(len(done), 6, replace=False)
    oracle.set_threads(0)
    for k in sample:
        j = done[k]
        rho, _, _ = workloads.gaussian_pulse_fields(j.nx, j.ny, j.amp)
        ref = oracle.Oracle(j.nx, j.ny, j.tau, j.c2).init(rho).step(j.steps).get_f()
        err = max_rel_err(j.f, ref)
        tol = 1e-5 * max(1.0, j.steps / 1000.0)
        print(f"job {j.id} {j.nx}x{j.ny} tau {j.tau:.3f} c2 {j.c2:.3f} amp {j.amp:.3f} {j.steps} steps: "
              f"max rel err {err:.2e}", flush=True)
        assert err <= tol, (j.id, err)
