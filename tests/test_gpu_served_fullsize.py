"""Parity of the serving workload at its full size, as the benchmark runs it:
the first 3 s of its seeded Poisson stream (50 jobs/s; square sides 2^U[7,11],
500 to 20000 steps log-uniform, random tau, c^2 and pulse amplitude; FP32)
into a server with a 200 GB budget stepping 100-step ticks, stopped when the
window ends (jobs still resident, others finished and retired, their slot
memory reused by later arrivals).

Every job that ran, finished or not, is then stepped alone by the plain
single-lattice kernel for the same number of steps: the FP64 totals (a
fixed-order reduction of the state) are bitwise equal, so continuous
batching changed no job's arithmetic.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0707_2437_amd as lbm  # noqa: E402
from paper_0707_2437_amd import serve  # noqa: E402

WINDOW = 3.0


def alone_totals(job, steps):
    rho = serve.pulse_field_device(torch, job.nx, job.ny, job.amp)
    with lbm.Lattice(job.nx, job.ny, job.tau, job.c2, "f32") as L:
        L.init_device(rho, None, None)
        return np.asarray(L.step(steps).totals())


def test_served_full_size_jobs_match_alone():
    jobs = serve.job_stream(50.0, WINDOW, seed=0)
    srv = serve.Server(int(200e9), "f32", tick_steps=100)
    st = srv.run(jobs, WINDOW)
    resident = [(j, j.steps - j.remaining, np.asarray(srv.pool.totals(s)[0])) for s, j in srv.running.items()]
    srv.close()
    finished = [j for j in srv.finished if j.status == "done"]
    print(f"{st['jobs_arrived']} arrived, {len(finished)} finished, {len(resident)} resident, "
          f"{st['ticks']} ticks", flush=True)
    assert st["jobs_failed"] == 0
    assert len(finished) >= 5 and len(resident) >= 20  # churn: retirements and resident jobs
    for j in finished:
        assert np.array_equal(np.asarray(j.totals), alone_totals(j, j.steps)), ("finished", j.id)
    for j, done, tot in resident:
        assert done > 0 and done % 100 == 0  # whole ticks only: a shorter last tick retires the job
        assert np.all(np.isfinite(tot))
        assert np.array_equal(tot, alone_totals(j, done)), ("resident", j.id, done)
