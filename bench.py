"""Benchmark: MLUPS and HBM-roofline fraction of the variable-speed-of-sound
D2Q9 step (Buick & Cosgrove, Sec. 3 Eq. 5) on one MI355X.

Workload (one "step"): one time step of each of five periodic 4096 x 4096
lattices, tau = 0.6, c^2 in {0.04, 0.2, 1/3, 0.5, 0.81} (c_e = 0.2 ... 0.9),
each initialised with a plane sound wave of amplitude 1e-3 plus seeded
uniform density noise +-1e-4. Headline: FP32 storage and arithmetic. The
same sweep in FP64, and the altered-equilibrium model (the other route to
a free c^2, Sec. 3 opening) over c^2 in {0.04, 0.2, 1/3, 0.5, 0.56}, are
reported under "forms", beside the batched form (256
seeded lattices of uneven size, tau and c^2 in one pool) and the served form
(a continuous-batching server fed Poisson job arrivals for a short window).

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line. Inputs are initialised on the device before the timed
region; the timed region holds exactly K steps, bracketed by
torch.cuda.synchronize() and HIP events recorded on the stream the kernels
run on.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E
# rocprofv3 counter records of the FP32 4096^2 launches: the two-step and single-step kernels
TRAFFIC_RECORDS = {"step2": os.path.join(ROOT, "profiles", "step2_f32_4096_traffic.json"),
                   "step": os.path.join(ROOT, "profiles", "step_f32_4096_traffic.json")}
TWO_STEP = 32  # LBM_TILE_TWO_STEP
BYTES_PER_SITE = {"f64": 144, "f32": 72, "f32s": 72, "f16s": 36}  # 9 reads + 9 writes
FIELD_BYTES = {"f64": 8, "f32": 4, "f32s": 4, "f16s": 4}  # one read of a c^2 field's coefficient


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1000)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--n", type=int, default=4096, help="lattice side")
    p.add_argument("--forms", default="f32_1step,f64,f32_eq,f32_field",
                   help="extra forms to time, comma separated ('' for none); a '_eq' suffix selects the "
                        "altered-equilibrium model over its own c^2 sweep, '_field' a c^2 field per lattice, "
                        "'_1step' the single-step kernel")
    p.add_argument("--form-steps", type=int, default=300)
    p.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    p.add_argument("--cpu-steps", type=int, default=100, help="oracle steps on all host cores")
    p.add_argument("--cpu-steps-one-core", type=int, default=10, help="oracle steps on one core")
    p.add_argument("--batch", type=int, default=256, help="lattices of the batched form (0: skip it)")
    p.add_argument("--batch-steps", type=int, default=2000)
    p.add_argument("--batch-mode", default="graph", choices=["grouped", "graph", "persistent"])
    p.add_argument("--batch-persistent-steps", type=int, default=200,
                   help="also time the persistent form for this many steps (0: skip)")
    p.add_argument("--pcie-steps", type=int, default=1000,
                   help="steps of the host-array run (fields in, populations out; 0: skip)")
    p.add_argument("--precision-steps", type=int, default=300,
                   help="steps of the precision workload (8192^2 shear wave, shifted FP32 / FP16; 0: skip)")
    p.add_argument("--serve-seconds", type=float, default=30.0,
                   help="window of the served form (Poisson jobs at --serve-rate; 0: skip it)")
    p.add_argument("--serve-rate", type=float, default=50.0)
    p.add_argument("--serve-budget-gb", type=float, default=200.0)
    p.add_argument("--copy-probe", action="store_true",
                   help="only run a device copy of known size (reference for HBM byte counters)")
    return p.parse_args()


def form_parts(form):
    """'<dtype>[_eq|_field]' -> (dtype, variant)."""
    for v in ("_eq", "_field"):
        if form.endswith(v):
            return form[:-len(v)], v[1:]
    return form, ""


def form_bytes_per_site(form):
    dtype, variant = form_parts(form)
    return BYTES_PER_SITE[dtype] + (FIELD_BYTES[dtype] if variant == "field" else 0)


def make_sweep(lbm, workloads, torch, n, form, stream):
    # "<dtype>_eq": the altered-equilibrium model over its own c^2 sweep;
    # "<dtype>_field": each lattice of the sweep with a lens-shaped c^2 field
    dtype, variant = form_parts(form)
    model, sweep = lbm.MODEL_FORCING, workloads.C2_SWEEP
    if variant == "eq":
        model, sweep = lbm.MODEL_EQUILIBRIUM, workloads.C2_SWEEP_EQ
    lattices = []
    for k, c2 in enumerate(sweep):
        rho, ux, uy = workloads.plane_wave_fields(n, n, c2, seed=k)
        L = lbm.Lattice(n, n, 0.6, c2, dtype, model=model)
        if variant == "field":
            L.set_c2_field(workloads.lens_c2_field(n, n, c2, depth=0.5))
        L.set_stream(stream)
        L.init(rho, ux, uy)
        lattices.append(L)
    return lattices


def launches_of(tile, steps):
    """Kernel launches lbm_step makes for `steps` steps in this shape: two
    steps per launch for a two-step shape (a lone last step takes one more)."""
    return (steps + 1) // 2 if tile[3] & TWO_STEP else steps


def time_sweep(torch, lattices, steps, warmup, stream):
    # Steps are taken two at a time per lattice (one two-step launch, or two
    # single-step launches), lattice after lattice.
    def run(k):
        for s in range(0, k, 2):
            for L in lattices:
                L.step(min(2, k - s))
    run(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    run(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1e3, wall


def kernel_name(tile, form):
    vx, nw, h, flags = tile
    dtype, variant = form_parts(form)
    t = {"f64": "double,false", "f32": "float,false", "f32s": "float,true", "f16s": "_Float16,true"}[dtype]
    if flags & TWO_STEP:
        return (f"lbm::step2_vstack_kernel<{t},{vx},{nw},{'true' if flags & 2 else 'false'},"
                f"{'true' if variant == 'field' else 'false'}>")
    if flags & 16:
        return (f"lbm::step_vstack_kernel<{t},{vx},{nw},{'true' if flags & 2 else 'false'},"
                f"{'true' if variant == 'field' else 'false'}>")
    pf = 2 if flags & 8 else (flags & 1)
    return f"lbm::step_kernel<{t},{vx},{nw},{pf},{'true' if flags & 2 else 'false'}> (h={h})"


def measured_traffic(kernel, n):
    """HBM bytes per launch from the committed rocprofv3 counter record of
    this kernel (two-step or single-step), if it was taken on the current
    kernel source and kernel; else None."""
    which = "step2" if kernel.startswith("lbm::step2_") else "step"
    try:
        from paper_0707_2437_amd import profiling
        rec = json.load(open(TRAFFIC_RECORDS[which]))
    except (OSError, ValueError, ImportError):
        return None
    if rec.get("kernel_source_sha256") != profiling.kernel_source_sha(which) or rec.get("kernel") != kernel \
            or rec.get("algorithmic_bytes_per_launch") != BYTES_PER_SITE["f32"] * n * n:
        return None
    return rec["traffic_bytes_per_launch"]


def measure_form(lbm, workloads, torch, n, dtype, steps, warmup, tile=None):
    # all launches go to one dedicated stream; the HIP events are recorded on it
    stream = torch.cuda.Stream()
    lats = make_sweep(lbm, workloads, torch, n, dtype, stream)
    if tile is not None:
        for L in lats:
            L.set_tile(*tile)
    tile = lats[0].get_tile()
    sec, wall = time_sweep(torch, lats, steps, warmup, stream)
    tot = [L.totals() for L in lats]
    for L in lats:
        L.close()
    sites = n * n * len(lats)
    # every launch reads and writes each site's nine populations once
    launches = launches_of(tile, steps) * len(lats)
    mlups = sites * steps / sec / 1e6
    gbs = form_bytes_per_site(dtype) * n * n / (sec / launches) / 1e9
    return {"mlups": mlups, "ms_per_step": 1e3 * sec / steps, "kernel_us": 1e6 * sec / launches,
            "achieved_GBs": gbs, "frac": gbs / PEAK_HBM_GBS, "wall_s": wall,
            "mass_total_first": tot[0][0], "kernel": kernel_name(tile, dtype), "tile": list(tile)}


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or the machine type."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(workloads, n, steps, steps_one_core):
    """The FP64 oracle on a bounded sample of the same workload: one of the
    five lattices (c^2 = 0.2), stepped on all host cores for `steps` steps and
    on one core for `steps_one_core` steps (the per-site arithmetic is the same,
    so are the results)."""
    import oracle

    rho, ux, uy = workloads.plane_wave_fields(n, n, 0.2, seed=1)

    def leg(threads, k, keep=False):
        oracle.set_threads(threads)
        o = oracle.Oracle(n, n, 0.6, 0.2).init(rho, ux, uy)
        o.step(1)  # page in
        t0 = time.perf_counter()
        o.step(k)
        sec = time.perf_counter() - t0
        if keep:
            return n * n * k / sec / 1e6, sec, oracle.get_threads(), o
        o.close()
        return n * n * k / sec / 1e6, sec, oracle.get_threads(), None

    all_mlups, all_sec, cores, ref = leg(0, steps, keep=True)
    parity = parity_against(ref, rho, ux, uy, n, steps + 1)
    ref.close()
    one_mlups, one_sec, _, _ = leg(1, steps_one_core)
    oracle.set_threads(0)
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    model = cpu_model()
    return {"value": round(all_mlups, 2), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"FP64 oracle, one {n}x{n} lattice of the sweep (c^2 = 0.2, tau = 0.6): {steps} steps on "
                      f"{cores} threads in {all_sec:.1f} s, {steps_one_core} steps on one thread in {one_sec:.1f} s",
            "one_core": {"value": round(one_mlups, 2), "unit": "MLUPS", "steps": steps_one_core,
                         "seconds": round(one_sec, 2)},
            "all_cores": {"value": round(all_mlups, 2), "unit": "MLUPS", "threads": cores, "steps": steps,
                          "seconds": round(all_sec, 2)},
            "cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable, "parity": parity}


def parity_against(ref, rho, ux, uy, n, steps, amp=1e-3):
    """The GPU's FP32 and FP64 forms against the oracle state `ref` (the same
    lattice, fields and step count): max relative error in f, and the errors
    of delta rho and u normalised by the wave's amplitude."""
    import numpy as np
    import paper_0707_2437_amd as lbm

    f_ref = ref.get_f()
    r_ref, ux_ref, uy_ref, _ = ref.moments()
    out = {"steps": steps, "lattice": [n, n], "c2": 0.2, "tau": 0.6}
    for dtype in ("f32", "f64"):
        with lbm.Lattice(n, n, 0.6, 0.2, dtype) as L:
            L.init(rho, ux, uy).step(steps)
            f = L.get_f()
            r, u, v, _ = L.moments()
        out[dtype] = {"max_rel_err_f": float(np.max(np.abs(f - f_ref) / np.abs(f_ref))),
                      "drho_err_over_amp": float(np.max(np.abs(r - r_ref)) / amp),
                      "u_err_over_amp": float(max(np.max(np.abs(u - ux_ref)), np.max(np.abs(v - uy_ref))) / amp)}
        del f
    return out


def measure_batched(lbm, workloads, torch, nlat, steps, mode, warmup=5, persistent_steps=0):
    """The batching workload: nlat seeded lattices of uneven size, tau and c^2
    (FP32) in one pool, stepped `steps` times by one call (in persistent mode
    one persistent launch); compared with the plain single-lattice kernel
    stepping the same lattices one launch each."""
    specs = workloads.batch_specs(nlat, seed=0)
    sites = sum(s["nx"] * s["ny"] for s in specs)
    stream = torch.cuda.Stream()
    budget = sum(lbm.Pool.slot_bytes(s["nx"], s["ny"], "f32") for s in specs)
    P = lbm.Pool(budget, "f32")
    P.set_stream(stream)
    P.set_mode({"grouped": lbm.GROUPED, "graph": lbm.GRAPH, "persistent": lbm.PERSISTENT}[mode])
    slots = []
    for sp in specs:
        s = P.add(sp["nx"], sp["ny"], sp["tau"], sp["c2"])
        P.init(s, *workloads.batch_fields(sp))
        slots.append(s)
    tile = P.autotune(slots, reps=5)
    P.step(slots, warmup)
    torch.cuda.synchronize()
    capture = None
    if mode == "graph":
        # The first call of a shape captures and instantiates its graph (host
        # work, once per shape); the timed call below replays it. The first
        # call's wall time less one replay's is reported as the capture cost.
        t = time.perf_counter()
        P.step(slots, steps)
        torch.cuda.synchronize()
        capture = time.perf_counter() - t
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    P.step(slots, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    P.sync()
    sec = e0.elapsed_time(e1) / 1e3
    nonfinite = sum(1 for s in slots if P.totals(s)[1] != 0)
    pers = None
    pers_tile = pers_members = None
    if persistent_steps > 0 and mode != "persistent":
        P.set_mode(lbm.PERSISTENT)
        pers_tile = P.autotune(slots, reps=5)  # the persistent kernel's own best shape
        P.step(slots, 2)
        torch.cuda.synchronize()
        e0.record(stream)
        P.step(slots, persistent_steps)
        e1.record(stream)
        torch.cuda.synchronize()
        P.sync()
        pers = sites * persistent_steps / (e0.elapsed_time(e1) / 1e3) / 1e6  # single steps (72 B per update)
        pers_members = P.persistent_members()
    P.close()
    # plain kernel, the lattices one at a time, two steps per call (the
    # single-lattice default shape: one two-step launch per lattice per two
    # steps; same lattices, fewer steps)
    psteps = max(2, steps // 10) // 2 * 2
    lats = []
    for sp in specs:
        L = lbm.Lattice(sp["nx"], sp["ny"], sp["tau"], sp["c2"], "f32")
        L.set_stream(stream)
        L.init(*workloads.batch_fields(sp))
        lats.append(L)
    for L in lats:
        L.step(warmup)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(psteps // 2):
        for L in lats:
            L.step(2)
    e1.record(stream)
    torch.cuda.synchronize()
    psec = e0.elapsed_time(e1) / 1e3
    for L in lats:
        L.close()
    mlups = sites * steps / sec / 1e6
    plain = sites * psteps / psec / 1e6
    # algorithmic bytes per site update: one load and one store per launch,
    # a two-step launch covering two updates
    per_update = BYTES_PER_SITE["f32"] / (2 if tile[2] & TWO_STEP else 1)
    return {"mlups": mlups, "frac": mlups * 1e6 * per_update / 1e9 / PEAK_HBM_GBS,
            "lattices": nlat, "sites": sites, "steps": steps, "mode": mode, "tile": list(tile),
            "seconds": sec, "plain_mlups": plain, "vs_plain": mlups / plain, "nonfinite_lattices": nonfinite,
            "persistent_mlups": pers, "persistent_tile": None if pers_tile is None else list(pers_tile),
            "persistent_members": pers_members,
            "graph_capture_s": None if capture is None else max(0.0, capture - sec)}


def measure_host_transfers(lbm, workloads, torch, n, steps):
    """One lattice of the sweep as a caller with host arrays runs it: FP64
    fields in through lbm_init (host to device, then the equilibrium set-up
    kernel), `steps` steps, the populations back through lbm_get_f (device to
    host, FP64). Not the headline (which starts with the state resident in
    HBM); the rate that includes PCIe."""
    rho, ux, uy = workloads.plane_wave_fields(n, n, 0.2, seed=1)
    with lbm.Lattice(n, n, 0.6, 0.2, "f32") as L:
        L.init(rho, ux, uy).step(2)
        L.get_f()  # warm: buffers, staging memory, code
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L.init(rho, ux, uy)  # synchronous
        t1 = time.perf_counter()
        L.step(steps)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        L.get_f()  # synchronous
        t3 = time.perf_counter()
    return {"mlups": n * n * steps / (t3 - t0) / 1e6, "steps": steps, "lattice": [n, n],
            "init_s": t1 - t0, "steps_s": t2 - t1, "get_f_s": t3 - t2,
            "bytes_in": 3 * n * n * 8, "bytes_out": 9 * n * n * 8}


def measure_precision(lbm, workloads, torch, steps, warmup=5, n=8192):
    """The precision workload: a periodic 8192^2 shear wave (tau = 0.7,
    c^2 = 0.25) in the shifted FP32 and FP16 storage forms."""
    out = {}
    stream = torch.cuda.Stream()
    for dtype in ("f32s", "f16s"):
        _, ux, _ = workloads.shear_wave_fields(n, n, amp=0.01)
        L = lbm.Lattice(n, n, 0.7, 0.25, dtype)
        L.set_stream(stream)
        L.init(None, ux, None)
        del ux
        sec, _ = time_sweep(torch, [L], steps, warmup, stream)
        tile = L.get_tile()
        L.close()
        mlups = n * n * steps / sec / 1e6
        gbs = form_bytes_per_site(dtype) * n * n * launches_of(tile, steps) / sec / 1e9
        out[dtype] = {"mlups": mlups, "achieved_GBs": gbs, "frac": gbs / PEAK_HBM_GBS, "steps": steps,
                      "kernel": kernel_name(tile, dtype), "lattice": [n, n]}
    return out


def measure_served(serve, seconds, rate, budget_gb):
    """The serving workload: Poisson job arrivals (sides 128..2048, 500..20000
    steps, FP32) into a continuous-batching server with a device-memory
    budget, for `seconds` of wall time."""
    jobs = serve.job_stream(rate, seconds, seed=0)
    srv = serve.Server(int(budget_gb * 1e9), "f32", tick_steps=100)
    st = srv.run(jobs, seconds)
    srv.close()
    st["offered_mlups"] = serve.offered_mlups(jobs, seconds)
    st["rate_per_s"] = rate
    st["budget_gb"] = budget_gb
    return st


def copy_probe(torch):
    """Device-to-device copy of 1 GiB, 20 times (reference kernel for the HBM
    byte counters: 1 GiB read + 1 GiB written per dispatch)."""
    nbytes = 1 << 30
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / 20
    print(json.dumps({"copy_probe_bytes": 2 * nbytes, "copy_GBs": 2 * nbytes / sec / 1e9}), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); "
              "the lattices of this workload are independent and would shard whole, "
              "so N GPUs would report N times the one-GPU rate.", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_0707_2437_amd as lbm
    from paper_0707_2437_amd import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if a.copy_probe:
        copy_probe(torch)
        return

    n = a.n
    head = measure_form(lbm, workloads, torch, n, "f32", a.steps, a.warmup)
    forms = {"f32": head}
    for f in [s for s in a.forms.split(",") if s]:
        if f.endswith("_1step"):  # the single-step vertical-stack kernel (the default shape before two-step)
            forms[f] = measure_form(lbm, workloads, torch, n, f[:-len("_1step")], a.form_steps, a.warmup,
                                    tile=(2, 8, 8, 18))
        else:
            forms[f] = measure_form(lbm, workloads, torch, n, f, a.form_steps, a.warmup)
        print(f"# form {f}: {forms[f]['mlups']:.0f} MLUPS, {100 * forms[f]['frac']:.1f}% of HBM peak",
              file=sys.stderr, flush=True)

    if a.precision_steps > 0:
        for k, v in measure_precision(lbm, workloads, torch, a.precision_steps).items():
            forms[f"precision_{k}"] = v
            print(f"# precision {k}: {v['mlups']:.0f} MLUPS, {100 * v['frac']:.1f}% of HBM peak",
                  file=sys.stderr, flush=True)

    if a.batch > 0:
        forms["batched_f32"] = measure_batched(lbm, workloads, torch, a.batch, a.batch_steps, a.batch_mode,
                                               persistent_steps=a.batch_persistent_steps)
        print(f"# batched: {forms['batched_f32']['mlups']:.0f} MLUPS over {a.batch} lattices "
              f"({forms['batched_f32']['vs_plain']:.2f}x the plain kernel one lattice at a time)",
              file=sys.stderr, flush=True)

    if a.serve_seconds > 0:
        from paper_0707_2437_amd import serve
        forms["served_f32"] = measure_served(serve, a.serve_seconds, a.serve_rate, a.serve_budget_gb)
        sv = forms["served_f32"]
        print(f"# served: {sv['mlups']:.0f} MLUPS, {sv['jobs_completed']} jobs done, latency p50 "
              f"{sv['latency_p50_s']} s p99 {sv['latency_p99_s']} s", file=sys.stderr, flush=True)

    if a.pcie_steps > 0:
        forms["f32_with_host_transfers"] = measure_host_transfers(lbm, workloads, torch, n, a.pcie_steps)

    cpu = None if a.no_cpu else cpu_baseline(workloads, n, a.cpu_steps, a.cpu_steps_one_core)
    if cpu is not None:
        cpu["gpu_over_all_cores"] = round(head["mlups"] / cpu["all_cores"]["value"], 1)
        cpu["gpu_over_one_core"] = round(head["mlups"] / cpu["one_core"]["value"], 1)
    sweep = list(workloads.C2_SWEEP)
    out = {
        "metric": "MLUPS (lattice-site updates per second / 1e6), one MI355X",
        "value": round(head["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"c2 sweep: 5 periodic {n}x{n} D2Q9 lattices, variable-speed-of-sound step",
                   "lattice": [n, n], "lattices_per_step": len(sweep), "tau": 0.6,
                   "c2": [round(c, 6) for c in sweep],
                   "init": "plane sound wave amp 1e-3 + uniform density noise 1e-4 (seeded)"},
        "roofline": {"bound": "hbm", "achieved": round(head["achieved_GBs"], 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(head["frac"], 4),
                     "traffic": measured_traffic(head["kernel"], n),
                     "kernel": head["kernel"],
                     "bytes_per_launch": BYTES_PER_SITE["f32"] * n * n,
                     "avg_launch_us": round(head["kernel_us"], 2)},
        "cpu_baseline": cpu,
        "forms": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                  for k, v in forms.items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
