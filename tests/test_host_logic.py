"""Host-side logic that needs no GPU: the benchmark's command line and form
names, the seeded input generators (which hold none of the method's
arithmetic), and the served form's job stream."""
import math
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_0707_2437_amd import serve, workloads  # noqa: E402


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_bench_form_names_and_bytes():
    assert bench.form_parts("f32") == ("f32", "")
    assert bench.form_parts("f32_eq") == ("f32", "eq")
    assert bench.form_parts("f64_field") == ("f64", "field")
    # 9 loads + 9 stores of the storage type, plus the field's coefficient
    assert bench.form_bytes_per_site("f32") == 72 and bench.form_bytes_per_site("f64") == 144
    assert bench.form_bytes_per_site("f16s") == 36 and bench.form_bytes_per_site("f32_eq") == 72
    assert bench.form_bytes_per_site("f32_field") == 76 and bench.form_bytes_per_site("f64_field") == 152
    assert bench.kernel_name((2, 16, 8, 50), "f32") == "lbm::step2_vstack_kernel<float,false,2,16,true,false>"
    assert bench.kernel_name((1, 16, 8, 50), "f64") == "lbm::step2_vstack_kernel<double,false,1,16,true,false>"
    assert bench.kernel_name((2, 16, 8, 50), "f32_field") == "lbm::step2_vstack_kernel<float,false,2,16,true,true>"
    assert bench.launches_of((2, 16, 8, 50), 1000) == 500 and bench.launches_of((2, 16, 8, 50), 7) == 4
    assert bench.launches_of((2, 8, 8, 18), 1000) == 1000
    assert bench.kernel_name((2, 8, 8, 18), "f32_field") == "lbm::step_vstack_kernel<float,false,2,8,true,true>"
    assert bench.kernel_name((2, 8, 8, 18), "f32_eq") == "lbm::step_vstack_kernel<float,false,2,8,true,false>"


def test_c2_sweeps():
    assert max(workloads.C2_SWEEP) == 0.81 and min(workloads.C2_SWEEP) == 0.04
    assert max(workloads.C2_SWEEP_EQ) < 0.6  # the altered-equilibrium model's range


def test_plane_wave_is_right_going():
    rho, ux, uy = workloads.plane_wave_fields(64, 8, 0.25, amp=1e-3, noise=0.0)
    assert uy is None and np.allclose(ux, 0.5 * (rho - 1.0), rtol=0, atol=1e-16)  # rounding of 1 + x
    r1, _, _ = workloads.plane_wave_fields(64, 8, 0.25, seed=3)
    r2, _, _ = workloads.plane_wave_fields(64, 8, 0.25, seed=3)
    assert np.array_equal(r1, r2)


def test_simple_wave_riemann_invariant_is_zero():
    rho, ux, _ = workloads.simple_wave_fields(400, 3, 0.04, 0.002)
    assert np.max(np.abs(ux - 0.2 * np.log(rho))) < 1e-16  # rounding of exp and log
    assert abs(np.max(ux) - 0.002) < 1e-9


def test_lens_field():
    f = workloads.lens_c2_field(96, 64, 0.5, depth=0.6)
    assert f.shape == (64, 96)
    assert abs(f.min() - 0.5 * 0.4) < 1e-12 and f.max() <= 0.5
    g = workloads.lens_c2_field(96, 64, 0.5, depth=0.6, noise=0.05, seed=4)
    assert np.all(np.abs(g / f - 1) <= 0.05) and len(np.unique(g)) > 0.9 * g.size


def test_batch_specs():
    a = workloads.batch_specs(256, seed=0)
    assert a == workloads.batch_specs(256, seed=0)
    assert all(64 <= s["nx"] <= 1024 and 64 <= s["ny"] <= 1024 for s in a)
    assert all(0.55 <= s["tau"] <= 1.5 and 0.04 <= s["c2"] <= 0.6 for s in a)
    assert sum(s["nx"] * s["ny"] for s in a) == 84833258  # the batched benchmark's sites


def test_job_stream():
    jobs = serve.job_stream(50.0, 30.0, seed=0)
    assert jobs == serve.job_stream(50.0, 30.0, seed=0)
    t = [j.arrival for j in jobs]
    assert t == sorted(t) and 0 < t[0] and t[-1] <= 30.0
    assert abs(len(jobs) - 1500) < 5 * math.sqrt(1500)  # Poisson count at 50 per second
    assert all(j.nx == j.ny and 128 <= j.nx <= 2048 for j in jobs)
    assert all(500 <= j.steps <= 20000 and 0.55 <= j.tau <= 1.5 and 0.04 <= j.c2 <= 0.6 for j in jobs)
    assert serve.offered_mlups(jobs, 30.0) == pytest.approx(sum(j.sites * j.steps for j in jobs) / 30e6)
    assert len(serve.job_stream(50.0, 30.0, seed=0, max_jobs=10)) == 10


def _pmc_csv(path, rows):
    import csv
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, c, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def test_traffic_record_from_counters_of_known_units(tmp_path):
    """HBM bytes from the counters: reads are 32, 64 and 128 bytes per request
    of each size (DRAM reads in 32-byte units beside them), writes 64 bytes per
    64-byte request and 32 per other request; the same counters on a copy of
    known size give the units check."""
    from paper_0707_2437_amd import profiling
    k = "void lbm::step_vstack_kernel<float, false, 2, 8, true, false>(lbm::StepTile, int)"
    rd = [(k, "TCC_EA0_RDREQ_32B_sum", 10.0), (k, "TCC_EA0_RDREQ_64B_sum", 20.0),
          (k, "TCC_EA0_RDREQ_128B_sum", 100.0), (k, "TCC_EA0_RDREQ_DRAM_32B_sum", 460.0),
          (k, "TCC_EA0_RDREQ_128B_sum", 300.0), (k, "TCC_EA0_RDREQ_32B_sum", 10.0),
          (k, "TCC_EA0_RDREQ_64B_sum", 20.0), (k, "TCC_EA0_RDREQ_DRAM_32B_sum", 460.0),
          ("other", "TCC_EA0_RDREQ_128B_sum", 1e9)]
    _pmc_csv(tmp_path / "r.csv", rd)
    _pmc_csv(tmp_path / "w.csv", [(k, "TCC_EA0_WRREQ_sum", 100.0), (k, "TCC_EA0_WRREQ_64B_sum", 90.0)])
    c = "__amd_rocclr_copyBuffer"
    _pmc_csv(tmp_path / "cr.csv", [(c, "TCC_EA0_RDREQ_32B_sum", 0.0), (c, "TCC_EA0_RDREQ_64B_sum", 0.0),
                                   (c, "TCC_EA0_RDREQ_128B_sum", 8192.0), (c, "TCC_EA0_RDREQ_DRAM_32B_sum", 32768.0)])
    _pmc_csv(tmp_path / "cw.csv", [(c, "TCC_EA0_WRREQ_sum", 16384.0), (c, "TCC_EA0_WRREQ_64B_sum", 16384.0)])
    alg = 2.0 * 40000.0
    rec = profiling.traffic_record("float, false, 2, 8, true, false", str(tmp_path / "r.csv"),
                                   str(tmp_path / "w.csv"), str(tmp_path / "cr.csv"), str(tmp_path / "cw.csv"),
                                   1024.0 * 1024.0, alg)
    reads = 32 * 10.0 + 64 * 20.0 + 128 * 200.0  # the 128-byte count is the mean of two dispatches
    writes = 64 * 90.0 + 32 * 10.0
    assert rec["reads_per_dispatch"]["dispatches"] == 2 and rec["writes_per_dispatch"]["dispatches"] == 1
    assert rec["read_bytes_per_launch"] == reads and rec["reads_per_dispatch"]["dram_bytes"] == 32 * 460.0
    assert rec["write_bytes_per_launch"] == writes
    assert rec["copy_check"] == {"bytes_each_way": 1024.0 * 1024.0, "read_ratio": 1.0, "dram_read_ratio": 1.0,
                                 "write_ratio": 1.0}
    assert rec["traffic_over_algorithmic"] == (reads + writes) / alg
    assert rec["read_over_algorithmic"] == reads / (alg / 2)
    assert rec["kernel_source_sha256"] == profiling.kernel_source_sha()
    with pytest.raises(ValueError):
        profiling.pmc_mean(str(tmp_path / "r.csv"), "no such kernel", "TCC_EA0_RDREQ_32B_sum")


def test_committed_traffic_record_matches_the_kernel_sources():
    """The benchmark reports roofline.traffic only from a counter record taken
    on the current kernel sources; the committed one must be current."""
    import json
    from paper_0707_2437_amd import profiling
    rec = json.load(open(os.path.join(ROOT, "profiles", "step_f32_4096_traffic.json")))
    assert rec["kernel_source_sha256"] == profiling.kernel_source_sha()
    assert bench.measured_traffic(rec["kernel"], 4096) == rec["traffic_bytes_per_launch"]
    # the two-step kernel (the benchmark's headline shape) has its own record
    rec2 = json.load(open(os.path.join(ROOT, "profiles", "step2_f32_4096_traffic.json")))
    assert rec2["kernel_sources"] == "step2" and rec2["kernel_source_sha256"] == profiling.kernel_source_sha("step2")
    assert rec2["kernel"] == "lbm::step2_vstack_kernel<float,false,2,16,true,false>"
    assert bench.measured_traffic(rec2["kernel"], 4096) == rec2["traffic_bytes_per_launch"]
    assert 1.0 < rec2["traffic_over_algorithmic"] < 1.5


def test_slot_arena_ranges(tmp_path):
    """The pool's range allocator (csrc/arena.h), built with g++ against a
    fake allocator: first-fit reuse, merging with free neighbours on both
    sides, chunk sizes bounded by the budget and by 2 GiB, a range larger than
    a chunk, a failed chunk allocation, alignment, and release."""
    import shutil

    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    exe = str(tmp_path / "arena_check")
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-I", os.path.join(root, "paper_0707_2437_amd", "csrc"),
                    os.path.join(root, "tests", "arena_check.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.strip() == "arena ok", r.stdout + r.stderr
