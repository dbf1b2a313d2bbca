#!/usr/bin/env python3
"""Benchmark: RK4 steps of the P_7 / 128^3 / FP32 inclusion workload.

One "step" is one full RK4 step (four stages, each: forward plane FFT pass,
z-derivative pass, moment-coupling pass, inverse plane pass with the fused
pointwise epilogue, plus the per-step readings/residual kernel) over the
whole device-resident state. The metric counts voxel x harmonic x RK-stage
updates per second. Prints one JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
                       [--workload p7_spheres] [--no-cpu-baseline]
                       [--copy-probe]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, 8 TB/s
METRIC = "voxel·harmonic RK-stage updates/s"

DESCR = {
    "p7_spheres": "P_7 (64 real moments), 128^3 grid, dx=0.25 mm, 16-voxel half-cosine "
                  "absorbing layer, background mu_a=0.01 mu_s=10 g=0.9 with 5 seeded "
                  "spherical inclusions, isotropic point pulse, 32 detectors, "
                  "RK4 dt=0.2 dx/c (c=0.3 mm/ps)",
    "p5_steady": "P_5 (36 moments), 256^3 log-normal medium, collimated slab source",
    "p3_adjoint": "P_3 (16 moments), 96^3 inclusion phantom, Gaussian pulse",
    "p1_gauss": "P_1 (4 moments), 32^3 homogeneous, Gaussian pulse",
}


def source_sha() -> str:
    h = hashlib.sha256()
    cs = os.path.join(ROOT, "paper_1801_06364_amd", "csrc")
    for f in sorted(os.listdir(cs)):
        with open(os.path.join(cs, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()


def algorithmic_bytes(kind: str, n: int, M: int, N: int, s: int) -> float:
    """Compulsory HBM bytes of one launch of each kernel class.

    The packed xy spectrum of one moment field holds n^2 (n/2) complex
    values, the same bytes as the real field (M n^3 s for all moments).
    fwd_plane: read the stage input, write the spectrum.
    zderiv: read the spectrum, write its z derivative.
    couple: read the spectrum and the derivative, write the coupled spectrum.
    inv_plane: read the coupled spectrum, the stage input, u and the
    per-degree loss maps ((N+1) n^3), write the stage output; averaged over
    the four RK stages (the first stage reads u once, the last one also
    updates the FP64 integrated fluence, 16 bytes per voxel).
    """
    F = M * n ** 3 * s
    if kind == "fwd_plane":
        return 2 * F
    if kind == "zderiv":
        return 2 * F
    if kind == "couple":
        return 3 * F
    if kind in ("inv_plane", "inv_rows"):
        return 3.75 * F + (N + 1) * n ** 3 * s + 16 * n ** 3 / 4
    if kind in ("fwd_rows", "y_fwd", "y_inv"):
        return 2 * F
    return 0.0


def cpu_baseline(wl, workers: int):
    """Time the FP64 oracle on a bounded sample: one RK stage (one full
    operator evaluation plus the stage update) of the same workload."""
    import numpy as np
    from oracle import pn
    pn.WORKERS = workers
    B = pn.coupling_matrices(wl.N)
    U = pn.real_basis_transform(wl.N)
    k = pn.wavenumbers(wl.n, wl.dx)
    Sig, _ = pn.potentials(wl.mu_a, wl.mu_s, wl.g, wl.N, wl.W, wl.mu0, wl.mu1)
    psi = pn.to_complex_basis(pn.full_moments(wl.psi0, wl.M), U).astype(complex)
    t0 = time.perf_counter()
    f = pn.operator(psi, Sig, None, B, k, wl.c, workers)
    psi = psi + (0.5 * wl.dt) * f
    el = time.perf_counter() - t0
    del f, psi
    upd = wl.n ** 3 * wl.M
    return {"value": upd / el, "unit": "updates/s", "cores": workers, "kind": "oracle",
            "sample": f"one RK stage (operator + stage update) of the full {wl.n}^3 P_{wl.N} "
                      f"workload in FP64, complex SH basis; {upd} updates in {el:.1f} s; "
                      f"scipy.fft workers={workers}, NumPy elementwise single-threaded"}


def traffic_for(kind: str, workload: str):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    rec = t.get(workload, {}).get(kind)
    if not rec or t.get("source_sha") != source_sha():
        return None
    return rec["bytes_per_launch"]


def serving_bench(a):
    """Continuous batching vs one-at-a-time on the seeded request trace:
    Poisson arrivals at 1.5 / (mean one-at-a-time service time)."""
    # one hardware queue per request stream (HIP's default is 4 per process),
    # set before the runtime initialises
    os.environ.setdefault("GPU_MAX_HW_QUEUES", str(max(4, min(16, a.slots))))
    import numpy as np
    import torch

    import rte_inputs as ri
    from paper_1801_06364_amd import serving

    torch.cuda.set_device(0)
    specs = ri.serving_requests(count=a.requests, seed=4)
    srv = serving.Server(budget_bytes=int(a.budget_gib * 2 ** 30), max_slots=a.slots,
                         large_slots=a.large_slots)
    # warm-up: one small request (library load, first launches), not reported
    srv.service_times([ri.RequestSpec(-1, 32, 1, 5, 0, 0, 1.0)])
    print(f"[serving] {len(specs)} requests; measuring one-at-a-time service times",
          file=sys.stderr, flush=True)
    alone = srv.service_times(specs)
    svc = np.array([r.finished - r.admitted for r in alone.values()])
    rate = 1.5 / svc.mean()
    arr = serving.poisson_arrivals(specs, rate)
    fifo = serving.fifo_replay(specs, arr, alone)
    print(f"[serving] mean service {svc.mean():.3f} s, rate {rate:.3f}/s; serving batched",
          file=sys.stderr, flush=True)
    bat = srv.serve(specs, arr)
    same = sum(1 for s in specs if bat.results[s.rid].ok and
               bat.results[s.rid].checksum == alone[s.rid].checksum)
    fs, bs = fifo.summary(), bat.summary()
    out = {"metric": "p50/p99 solve latency and aggregate updates/s (serving)",
           "value": bs["updates_per_s"], "unit": "updates/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{len(specs)} seeded requests (seed 4): grids {{32,48,64,96,128}}^3, "
                                  "P_N in {1,3,5,7}, 200-1000 RK4 steps, half homogeneous / half 1-5 "
                                  "inclusions, Gaussian pulse; Poisson arrivals at 1.5 / mean "
                                  "one-at-a-time service time",
                      "budget_GiB": a.budget_gib, "slots": a.slots, "large_slots": a.large_slots,
                      "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES"), "rate_per_s": rate,
                      "mean_service_s": float(svc.mean())},
           "batched": bs, "one_at_a_time": fs,
           "speedup_p50": fs["p50_latency_s"] / bs["p50_latency_s"],
           "speedup_p99": fs["p99_latency_s"] / bs["p99_latency_s"],
           "speedup_throughput": bs["updates_per_s"] / fs["updates_per_s"],
           "results_identical_alone_vs_mix": f"{same}/{len(specs)}"}
    print(json.dumps(out), flush=True)


def accuracy_report():
    """FP32 and FP64 GPU results against the FP64 oracle on the bench recipe
    at a reduced size (p7_spheres, 32^3, 12 steps): relative L2 per result
    (readings relative to the fluence peak of each step)."""
    import numpy as np

    import rte_inputs as ri
    from oracle import pn
    from paper_1801_06364_amd.rte import Solver

    n, steps = 32, 12
    wl = ri.workload("p7_spheres", n=n, steps=steps)
    ref = pn.solve(wl.n, wl.N, wl.dx, wl.c, wl.dt, wl.mu_a, wl.mu_s, wl.g, wl.psi0, None, wl.W,
                   wl.mu0, wl.mu1, steps, det_index=wl.det_index)

    def rel(x, y):
        return float(np.linalg.norm(np.ravel(x) - np.ravel(y)) / np.linalg.norm(np.ravel(y)))

    out = {"workload": f"p7_spheres recipe at {n}^3, {steps} RK4 steps"}
    for prec in ("f32", "f64"):
        s = Solver.from_workload(ri.workload("p7_spheres", n=n, steps=steps, precision=prec))
        s.step(steps)
        r = s.readings()
        out[prec] = {"fluence": rel(s.fluence(), ref["fluence"]),
                     "state": rel(s.get_state(), ref["state"]),
                     "integrated_fluence": rel(s.fluence(1), ref["phi_int"]),
                     "readings_max_err_over_peak": float(np.max(np.abs(r - ref["readings"]) /
                                                                ref["peak"][:, None]))}
        s.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="p7_spheres")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--serving", action="store_true",
                    help="serve the seeded Poisson request trace instead (separate JSON line)")
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--budget-gib", type=float, default=12.0)
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--large-slots", type=int, default=2)
    ap.add_argument("--no-accuracy", action="store_true")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the hot path is a single-GPU solve; "
              "multi-GPU runs are not part of this build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import rte_inputs as ri
    from paper_1801_06364_amd.rte import Solver

    if a.serving:
        return serving_bench(a)

    wl = ri.workload(a.workload, steps=a.steps + a.warmup)
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    s = Solver.from_workload(wl, stream=stream)
    print(f"[bench] {a.workload} n={wl.n} N={wl.N} {wl.precision} created", file=sys.stderr,
          flush=True)
    s.step(a.warmup)
    stream.synchronize()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    s.step(a.steps)
    ev1.record(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    done = s.steps_done()
    assert done == a.steps + a.warmup, (done, a.steps + a.warmup)
    fl = s.fluence()
    assert np.all(np.isfinite(fl))
    print(f"[bench] timed {a.steps} steps: {ms:.2f} ms (wall {wall:.3f} s)", file=sys.stderr,
          flush=True)

    upd_step = wl.n ** 3 * wl.M * 4
    value = upd_step * a.steps / (ms / 1e3)
    sbytes = 8 if wl.precision == "f64" else 4

    prof = s.profile_kernels(a.profile_steps)
    per = {k: (t / c if c else 0.0) for k, (t, c) in prof.items()}
    dom = max((k for k in prof if k != "end_step"), key=lambda k: prof[k][0])
    alg = algorithmic_bytes(dom, wl.n, wl.M, wl.N, sbytes)
    achieved = alg / (per[dom] / 1e3) / 1e9
    tb = traffic_for(dom, a.workload)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": tb, "algorithmic_bytes": alg,
                "avg_launch_ms": per[dom]}
    s.close()

    # device-to-device copy of 1 GiB: the practical streaming bandwidth of this
    # GPU, reported beside the published peak (it is not used as the peak)
    x = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1.0)
    y.copy_(x)
    torch.cuda.synchronize()
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    reps = 3 if a.copy_probe else 5
    c0.record()
    for _ in range(reps):
        y.copy_(x)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * x.numel() * 4 * reps / (c0.elapsed_time(c1) / 1e3) / 1e9
    roofline["copy_kernel_GBs"] = copy_gbs
    del x, y

    out = {
        "metric": METRIC, "value": value, "unit": "updates/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms / a.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": wl.precision, "data": "synthetic",
        "config": {"workload": f"{a.workload}: {DESCR.get(a.workload, '')}", "n": wl.n,
                   "order_N": wl.N, "moments": wl.M, "precision": wl.precision,
                   "updates_per_step": upd_step, "parallelism": "single GPU"},
        "kernel_ms_per_launch": per,
        "roofline": roofline,
    }
    if not a.no_accuracy:
        out["accuracy"] = accuracy_report()
    if not a.no_cpu_baseline:
        workers = int(os.environ.get("OMP_NUM_THREADS", "0")) or min(16, os.cpu_count() or 1)
        wlc = ri.workload(a.workload, steps=1)
        out["cpu_baseline"] = cpu_baseline(wlc, workers)
        print(f"[bench] cpu baseline: {out['cpu_baseline']['value']:.3e} updates/s",
              file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
