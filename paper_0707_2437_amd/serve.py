"""Served form: a continuous-batching request loop over an lbm_pool.

Jobs (one periodic lattice each: nx, ny, tau, c2, an initial Gaussian density
pulse, a number of steps) arrive over time. The server admits queued jobs as
slots whenever the pool's device-memory budget has room, keeps their
lattices resident, and in every tick advances all resident jobs together by
up to `tick_steps` steps each in one batched pool call (each job by exactly
what it still needs), so jobs that arrive while others run join the next
tick and their work overlaps on the device. The host does not wait for a
tick before queueing the next: the jobs a tick finishes have their
conservation totals queued on the device behind it and their slots released
at once (all pool work runs in order on one stream), and the totals are read
back one tick later, while the next tick runs. A non-finite total marks a
job failed; completion time is when the host reads its totals.

    python -m paper_0707_2437_amd.serve --rate 50 --duration 600 --budget-gb 200

prints one JSON line of statistics: jobs offered / admitted / completed /
failed / left waiting, throughput (lattice-site updates per second), latency
p50 / p99 of completed jobs, and queueing time vs service time.
"""
import argparse
import json
import math
import sys
import time
from dataclasses import dataclass, field

import numpy as np

from . import lattice as _lattice
from .pool import GROUPED, Pool


@dataclass
class Job:
    id: int
    nx: int
    ny: int
    tau: float
    c2: float
    amp: float
    steps: int
    arrival: float = 0.0  # seconds after the start of the run
    slot: int = -1
    remaining: int = 0
    t_admit: float = math.nan
    t_done: float = math.nan
    status: str = "queued"  # queued | running | retiring (totals in flight) | done | failed
    totals: list = field(default_factory=list)

    @property
    def sites(self):
        return self.nx * self.ny


def job_stream(rate, duration, seed=0, side_log2=(7, 11), steps=(500, 20000), max_jobs=None):
    """Seeded Poisson arrivals at `rate` per second over `duration` seconds:
    square lattices of side 2^U[side_log2] (log-uniform), steps log-U[steps],
    tau ~ U[0.55, 1.5], c^2 ~ U[0.04, 0.6], pulse amplitude ~ U[0.01, 0.1]."""
    rng = np.random.default_rng(seed)
    jobs, t = [], 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration or (max_jobs is not None and len(jobs) >= max_jobs):
            break
        side = int(round(2 ** rng.uniform(*side_log2)))
        jobs.append(Job(id=len(jobs), nx=side, ny=side, tau=float(rng.uniform(0.55, 1.5)),
                        c2=float(rng.uniform(0.04, 0.6)), amp=float(rng.uniform(0.01, 0.1)),
                        steps=int(round(math.exp(rng.uniform(math.log(steps[0]), math.log(steps[1]))))),
                        arrival=t))
    return jobs


def pulse_field_device(torch, nx, ny, amp, device="cuda"):
    """rho = 1 + amp exp(-r^2 / (2 sigma^2)), sigma = min(nx, ny)/16, centred,
    as a float64 device tensor (the initial velocity is zero)."""
    y = torch.arange(ny, dtype=torch.float64, device=device)[:, None]
    x = torch.arange(nx, dtype=torch.float64, device=device)[None, :]
    sigma = min(nx, ny) / 16.0
    r2 = (x - nx / 2.0) ** 2 + (y - ny / 2.0) ** 2
    return (1.0 + amp * torch.exp(-r2 / (2.0 * sigma * sigma))).contiguous()


class Server:
    def __init__(self, budget_bytes, dtype="f32", tick_steps=100, stream=None, keep_f=False, progress_every=0.0,
                 ring_rows=1024):
        import torch

        self.torch = torch
        self.pool = Pool(budget_bytes, dtype)
        self.pool.set_mode(GROUPED)
        self.dtype = dtype
        self.tick_steps = int(tick_steps)
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.pool.set_stream(self.stream)
        self.keep_f = keep_f
        self.progress_every = float(progress_every)
        self.queue = []       # admitted order: FIFO
        self.running = {}     # slot -> job
        self.finished = []
        self.pending = []     # queued ticks not yet read back
        self.site_updates = 0
        self.gpu_seconds = 0.0
        self.ticks = 0
        # ring of rows for the totals of finishing jobs: device rows written
        # by lbm_pool_totals_device, copied to pinned host rows
        self._ring = 0
        self._ring_dev = None
        self._ring_host = None
        self._ensure_ring(int(ring_rows))

    def _ensure_ring(self, rows):
        if self._ring_dev is not None and self._ring_dev.shape[0] >= rows:
            return
        torch = self.torch
        self.drain(keep=0)  # no queued tick still writes the old ring
        with torch.cuda.stream(self.stream):
            self._ring_dev = torch.empty((rows, 3), dtype=torch.float64, device="cuda")
        self._ring_host = torch.empty((rows, 3), dtype=torch.float64, pin_memory=True)
        self._ring = 0

    def close(self):
        self.drain(keep=0)
        self.pool.close()

    def submit(self, job):
        job.status = "queued"
        self.queue.append(job)

    def _admit(self, now):
        """Admit queued jobs in arrival order while the budget has room."""
        while self.queue:
            job = self.queue[0]
            slot = self.pool.try_add(job.nx, job.ny, job.tau, job.c2)
            if slot is None:
                if not self.running:  # a job larger than the whole budget can never run
                    self.queue.pop(0)
                    job.status, job.t_done = "failed", now
                    self.finished.append(job)
                    continue
                break
            self.queue.pop(0)
            # The field is made on the pool's stream and the init kernel reads
            # it on the same stream, so torch may recycle its memory for later
            # work on that stream once the Python reference is gone.
            with self.torch.cuda.stream(self.stream):
                rho = pulse_field_device(self.torch, job.nx, job.ny, job.amp)
            self.pool.init_device(slot, rho, None, None)
            job.slot, job.remaining, job.t_admit, job.status = slot, job.steps, now, "running"
            self.running[slot] = job

    def tick(self, now):
        """Admit, queue the next steps of every resident job (one batched pool
        call), and queue the totals of the jobs these steps finish, releasing
        their slots. Nothing here waits for the device (keep_f aside)."""
        torch = self.torch
        self._admit(now)
        if not self.running:
            return
        slots = list(self.running)
        nsteps = [min(self.tick_steps, self.running[s].remaining) for s in slots]
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(self.stream)
        self.pool.step(slots, nsteps)
        ev1.record(self.stream)
        self.ticks += 1
        done = []
        for s, n in zip(slots, nsteps):
            job = self.running[s]
            job.remaining -= n
            self.site_updates += n * job.sites
            if job.remaining == 0:
                done.append(job)
        entry = {"ev0": ev0, "ev1": ev1, "jobs": done}
        if done:
            if self._ring + len(done) > self._ring_dev.shape[0]:
                # wrap: read back every queued tick first (their rows are
                # reused); grow when one tick's jobs fill half the ring
                if 2 * len(done) > self._ring_dev.shape[0]:
                    self._ensure_ring(2 * len(done))
                else:
                    self.drain(keep=0)
                    self._ring = 0
            r0 = self._ring
            for k, job in enumerate(done):
                self.pool.totals_device(job.slot, self._ring_dev[r0 + k])
                if self.keep_f:
                    job.f = self.pool.get_f(job.slot)
                self.pool.remove(job.slot)
                del self.running[job.slot]
                job.status = "retiring"
            rows = slice(r0, r0 + len(done))
            with torch.cuda.stream(self.stream):
                self._ring_host[rows].copy_(self._ring_dev[rows], non_blocking=True)
            evd = torch.cuda.Event()
            evd.record(self.stream)
            entry.update({"rows": rows, "done_ev": evd})
            self._ring = r0 + len(done)
        self.pending.append(entry)

    def drain(self, keep=1):
        """Read back every queued tick but the last `keep`: GPU time, and the
        totals of the jobs they finished (which completes those jobs)."""
        while len(self.pending) > keep:
            e = self.pending.pop(0)
            (e.get("done_ev") or e["ev1"]).synchronize()
            now = time.perf_counter() - self._t0
            self.gpu_seconds += e["ev0"].elapsed_time(e["ev1"]) / 1e3
            if e["jobs"]:
                tot = self._ring_host[e["rows"]].tolist()
                for job, t in zip(e["jobs"], tot):
                    job.totals = [float(v) for v in t]
                    job.status = "done" if all(math.isfinite(v) for v in t) else "failed"
                    job.t_done = now
                    self.finished.append(job)

    def run(self, jobs, duration, drain=False):
        """Serve `jobs` (arrival times in seconds from now, honoured in real
        time) for `duration` seconds of wall time, then stop; with `drain`,
        keep going until every job has arrived and finished."""
        pending = sorted(jobs, key=lambda j: j.arrival)
        k = 0
        self._t0 = t0 = time.perf_counter()
        next_report = self.progress_every if self.progress_every > 0 else math.inf
        while True:
            now = time.perf_counter() - t0
            while k < len(pending) and pending[k].arrival <= now:
                self.submit(pending[k])
                k += 1
            if now >= next_report:
                print(f"# served t={now:.0f}s arrived {k} completed {len(self.finished)} running "
                      f"{len(self.running)} waiting {len(self.queue)} MLUPS {self.site_updates / now / 1e6:.0f}",
                      file=sys.stderr, flush=True)
                next_report += self.progress_every
            if now >= duration and not drain:
                break
            if not self.running and not self.queue:
                if self.pending:
                    self.drain(keep=0)
                    continue
                if k >= len(pending):
                    break
                time.sleep(min(0.01, max(0.0, pending[k].arrival - now)))
                continue
            self.tick(now)
            self.drain(keep=1)  # the tick before this one, while this one runs
        self.drain(keep=0)
        elapsed = time.perf_counter() - t0
        return self.stats(len(pending), k, elapsed)

    def stats(self, offered_total, arrived, elapsed):
        done = [j for j in self.finished if j.status == "done"]
        lat = np.array([j.t_done - j.arrival for j in done]) if done else np.array([])
        wait = np.array([j.t_admit - j.arrival for j in done]) if done else np.array([])
        serv = np.array([j.t_done - j.t_admit for j in done]) if done else np.array([])
        pct = lambda a, q: float(np.percentile(a, q)) if len(a) else None
        return {
            "jobs_offered": offered_total, "jobs_arrived": arrived, "jobs_completed": len(done),
            "jobs_failed": sum(1 for j in self.finished if j.status == "failed"),
            "jobs_running": len(self.running), "jobs_waiting": len(self.queue),
            "elapsed_s": elapsed, "ticks": self.ticks, "gpu_busy_s": self.gpu_seconds,
            "gpu_busy_frac": self.gpu_seconds / elapsed if elapsed > 0 else None,
            "site_updates": self.site_updates, "mlups": self.site_updates / elapsed / 1e6 if elapsed > 0 else None,
            "mlups_while_busy": self.site_updates / self.gpu_seconds / 1e6 if self.gpu_seconds > 0 else None,
            "latency_p50_s": pct(lat, 50), "latency_p99_s": pct(lat, 99),
            "queue_wait_p50_s": pct(wait, 50), "queue_wait_p99_s": pct(wait, 99),
            "service_p50_s": pct(serv, 50), "service_p99_s": pct(serv, 99),
            "pool_used_bytes": self.pool.used_bytes,
            "pool_device_bytes": self.pool.device_bytes,
        }


def offered_mlups(jobs, duration):
    return sum(j.sites * j.steps for j in jobs) / duration / 1e6


def main(argv=None):
    p = argparse.ArgumentParser()
    p.add_argument("--rate", type=float, default=50.0, help="mean job arrivals per second (Poisson)")
    p.add_argument("--duration", type=float, default=600.0, help="seconds of serving")
    p.add_argument("--budget-gb", type=float, default=200.0)
    p.add_argument("--dtype", default="f32", choices=list(_lattice.DTYPES))
    p.add_argument("--tick-steps", type=int, default=100)
    p.add_argument("--seed", type=int, default=0)
    p.add_argument("--progress-every", type=float, default=30.0, help="seconds between progress lines (stderr)")
    p.add_argument("--out", default=None, help="also write the JSON statistics to this file")
    a = p.parse_args(argv)
    import torch

    torch.cuda.set_device(0)
    jobs = job_stream(a.rate, a.duration, seed=a.seed)
    srv = Server(int(a.budget_gb * 1e9), a.dtype, a.tick_steps, progress_every=a.progress_every)
    st = srv.run(jobs, a.duration)
    st.update({"rate_per_s": a.rate, "duration_s": a.duration, "budget_gb": a.budget_gb, "dtype": a.dtype,
               "tick_steps": a.tick_steps, "offered_mlups": offered_mlups(jobs, a.duration),
               "command": "python -m paper_0707_2437_amd.serve " + " ".join(argv if argv is not None else sys.argv[1:])})
    srv.close()
    print(json.dumps(st), flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(st, fh, indent=1)


if __name__ == "__main__":
    sys.exit(main())
