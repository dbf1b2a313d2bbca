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


def stages_per_step(scheme: str) -> int:
    """Operator evaluations (stages) per time step: four for RK4, one for
    the forward-Euler step of eq. (11)."""
    return 1 if scheme == "euler" else 4


def algorithmic_bytes(kind: str, n: int, M: int, N: int, s: int) -> float:
    """Compulsory HBM bytes of one launch of each kernel class.

    The packed xy spectrum of one moment field holds n^2 (n/2) complex
    values, the same bytes as the real field (M n^3 s for all moments).
    fwd_plane: read the stage input, write the spectrum.
    zderiv: read the spectrum, write its z derivative.
    couple: read the spectrum and the derivative, write the coupled spectrum.
    inv_plane (grids up to 128, fused with the next stage's forward
    transform): read the coupled spectrum, the stage input, u and the
    per-degree loss maps ((N+1) n^3), write the stage output and its xy
    spectrum; averaged over the four RK stages (the first stage reads u
    once, the last one also updates the FP64 integrated fluence, 16 bytes
    per voxel).
    inv_rows (larger grids: x transforms only, fused with the next
    stage's forward row transform): the same bytes as inv_plane.
    """
    F = M * n ** 3 * s
    if kind == "fwd_plane":
        return 2 * F
    if kind == "zderiv":
        return 2 * F
    if kind == "couple":
        return 3 * F
    if kind == "inv_plane":
        return 4.75 * F + (N + 1) * n ** 3 * s + 16 * n ** 3 / 4
    if kind == "inv_rows":
        return 4.75 * F + (N + 1) * n ** 3 * s + 16 * n ** 3 / 4
    if kind in ("fwd_rows", "y_fwd", "y_inv"):
        return 2 * F
    return 0.0


def cpu_baseline(wl, workers: int):
    """Time the FP64 oracle on a bounded sample: one full RK4 step (four
    operator evaluations and the stage combinations) of the same workload."""
    import numpy as np
    from oracle import pn
    pn.WORKERS = workers
    B = pn.coupling_matrices(wl.N)
    U = pn.real_basis_transform(wl.N)
    k = pn.wavenumbers(wl.n, wl.dx)
    Sig, _ = pn.potentials(wl.mu_a, wl.mu_s, wl.g, wl.N, wl.W, wl.mu0, wl.mu1)
    psi = pn.to_complex_basis(pn.full_moments(wl.psi0, wl.M), U).astype(complex)

    def f(y):
        return pn.operator(y, Sig, None, B, k, wl.c, workers)

    t0 = time.perf_counter()
    psi = pn.rk4_step(psi, f, wl.dt)
    el = time.perf_counter() - t0
    del psi
    upd = wl.n ** 3 * wl.M * 4
    return {"value": upd / el, "unit": "updates/s", "cores": workers, "kind": "oracle",
            "sample": f"one RK4 step (four operator evaluations and the stage combinations) of the full "
                      f"{wl.n}^3 P_{wl.N} workload in FP64, complex SH basis; {upd} updates in {el:.1f} s; "
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
    os.environ["GPU_MAX_HW_QUEUES"] = str(max(4, min(16, a.slots)))
    import numpy as np
    import torch

    import rte_inputs as ri
    from paper_1801_06364_amd import serving

    torch.cuda.set_device(0)
    specs = ri.serving_requests(count=a.requests, seed=4)
    srv = serving.Server(budget_bytes=int(a.budget_gib * 2 ** 30), max_slots=a.slots,
                         chunk=a.chunk, big_slots=a.big_slots)
    # warm-up: one small request (library load, first launches), not reported
    srv.service_times([ri.RequestSpec(-1, 32, 1, 5, 0, 0, 1.0)])
    print(f"[serving] {len(specs)} requests; measuring one-at-a-time service times",
          file=sys.stderr, flush=True)
    alone = {}
    for i in range(0, len(specs), 32):   # in groups, with a progress line after each
        alone.update(srv.service_times(specs[i:i + 32]))
        print(f"[serving] {len(alone)}/{len(specs)} measured alone", file=sys.stderr, flush=True)
    svc = np.array([r.finished - r.admitted for r in alone.values()])
    rate = 1.5 / svc.mean()
    arr = serving.poisson_arrivals(specs, rate)
    fifo = serving.fifo_replay(specs, arr, alone)
    print(f"[serving] mean service {svc.mean():.3f} s, rate {rate:.3f}/s; serving batched",
          file=sys.stderr, flush=True)
    bat = srv.serve(specs, arr)
    # bitwise comparison of every fluence field (SHA-256 of its bytes)
    same = sum(1 for s in specs if bat.results[s.rid].ok and bat.results[s.rid].digest and
               bat.results[s.rid].digest == alone[s.rid].digest)
    fs, bs = fifo.summary(), bat.summary()
    out = {"metric": "p50/p99 solve latency and aggregate updates/s (serving)",
           "value": bs["updates_per_s"], "unit": "updates/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{len(specs)} seeded requests (seed 4): grids {{32,48,64,96,128}}^3, "
                                  "P_N in {1,3,5,7}, 200-1000 RK4 steps, half homogeneous / half 1-5 "
                                  "inclusions, Gaussian pulse; Poisson arrivals at 1.5 / mean "
                                  "one-at-a-time service time",
                      "budget_GiB": a.budget_gib, "max_slots_per_batch": a.slots,
                      "slots_above_512MiB": a.big_slots,
                      "chunk_steps": a.chunk,
                      "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES"), "rate_per_s": rate,
                      "mean_service_s": float(svc.mean())},
           "batched": bs, "one_at_a_time": fs,
           "speedup_p50": fs["p50_latency_s"] / bs["p50_latency_s"],
           "speedup_p99": fs["p99_latency_s"] / bs["p99_latency_s"],
           "speedup_throughput": bs["updates_per_s"] / fs["updates_per_s"],
           "results_identical_alone_vs_mix": f"{same}/{len(specs)}",
           "identity_check": "SHA-256 of each final fluence field, alone vs served"}
    print(json.dumps(out), flush=True)


FP32_VALU_PEAK = 157.3   # TFLOP/s, MI355X vector FP32 (published; counts packed FP32)
FP64_VALU_PEAK = 78.6    # TFLOP/s, MI355X vector FP64 (published)


def taylor_plan(kk, ct, sigmax, prec):
    """Substeps s and Taylor terms J per spectral point of the exact
    propagation (the kernel's rule: s = ceil(nu / theta), J the fewest terms
    with (nu/s)^(J+1) / (J+1)! exp(nu/s) <= eps, nu = c T (|k| + max Sigma))."""
    import math

    import numpy as np
    m, eps = (24, 2.0 ** -53) if prec == "f64" else (14, 2.0 ** -24)
    lo, hi = 0.0, 64.0
    for _ in range(200):
        t = 0.5 * (lo + hi)
        if (m + 1) * math.log(t) - math.lgamma(m + 2) + t <= math.log(eps):
            lo = t
        else:
            hi = t
    theta = lo
    nu = ct * (kk + sigmax)
    s = np.where(nu > theta, np.ceil(nu / theta), 1.0)
    nus = nu / s
    J = np.ones_like(nus)
    bound = 0.5 * nus * nus * np.exp(nus)
    for _ in range(m):
        more = (bound > eps) & (J < m)
        J = np.where(more, J + 1, J)
        bound = np.where(more, bound * nus / (J + 1), bound)
    return s, J, theta


def expo_term_flops(N: int):
    """Floating-point operations of one Taylor term at one spectral point:
    per non-zero entry of k.B (each belongs to one axis) its value (1 flop)
    and the complex-by-real multiply-add (4); per moment the loss (4), the
    step scale (2) and the accumulation (2)."""
    from paper_1801_06364_amd.rte import rte_coupling_dense
    bx, by, bz = rte_coupling_dense(N)
    nz = int(((bx != 0) | (by != 0) | (bz != 0)).sum())
    M = (N + 1) ** 2
    return nz * 5 + 8 * M


def expo_bench(a):
    """Exact propagation (homogeneous medium, periodic grid) over the time
    of 100 RK4 steps against marching those steps, both on the GPU."""
    import numpy as np
    import torch

    import rte_inputs as ri
    from paper_1801_06364_amd.rte import Solver

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    n, N, dx, c, prec = 128, 7, 0.25, 0.3, "f32"
    mua, mus, g = 0.01, 10.0, 0.9
    dt = 0.2 * dx / c
    K = 100
    T = K * dt
    ma, ms_, gg = ri.homogeneous_maps(n, mua, mus, g)
    psi0 = ri.gaussian_ic(n, 0, sigma=2.0)
    M = (N + 1) ** 2

    def solver(step_dt):
        return Solver(n, N, dx, c, step_dt, ma, ms_, gg, psi0=psi0, W=0, precision=prec,
                      stream=stream)

    s = solver(dt)
    s.expo_advance(T)                   # warm-up
    s.set_state(np.concatenate([psi0, np.zeros((M - 1, n, n, n))]))
    reps = max(1, a.expo_reps)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(reps):
        s.expo_advance(T)
    ev1.record(stream)
    stream.synchronize()
    ms_expo = ev0.elapsed_time(ev1) / reps
    print(f"[expo] {reps} advances of {T:.3f} ps: {ms_expo:.2f} ms each", file=sys.stderr, flush=True)
    s.set_state(np.concatenate([psi0, np.zeros((M - 1, n, n, n))]))
    s.expo_advance(T)
    ex = s.fluence()
    prof = s.profile_expo(T)
    s.close()

    r = solver(dt)
    r.step(5)
    stream.synchronize()
    r.set_state(np.concatenate([psi0, np.zeros((M - 1, n, n, n))]))
    ev0.record(stream)
    r.step(K)
    ev1.record(stream)
    stream.synchronize()
    ms_rk4 = ev0.elapsed_time(ev1)
    rk = r.fluence()
    r.close()
    print(f"[expo] {K} RK4 steps: {ms_rk4:.2f} ms", file=sys.stderr, flush=True)

    k = 2 * np.pi * np.fft.fftfreq(n, d=dx)
    k[n // 2] = 0.0
    kz, ky, kx = np.meshgrid(k, k, k[: n // 2], indexing="ij")
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    sigmax = max(mua + mus * (1 - g ** l) for l in range(N + 1))
    sub, J, theta = taylor_plan(kk, c * T, sigmax, prec)
    terms = float((sub * J).sum())
    per = {k_: t / cnt for k_, (t, cnt) in prof.items()}
    F = M * n ** 3 * 4
    if "expo_table" in prof:
        # block exponentials by scaling and squaring (FP64), per f^2 = fx^2 +
        # fy^2 + fz^2 and order m >= 0 (m and -m share their blocks), d x d
        # blocks: 14 Taylor terms of the tridiagonal generator (per entry and
        # term 8 flops for the two couplings, 4 for |k| and the loss, 2 for
        # the step, 6 for the E and P sums), then q doublings P <- P + E P,
        # E <- E E (two complex d^3 products, 8 flops per multiply-add, and
        # the P sum)
        nf2 = (n // 2 - 1) ** 2 * 3 + 1
        ks = 2 * np.pi / (n * dx) * np.sqrt(np.arange(nf2, dtype=float))
        nu = c * T * (ks + sigmax)
        q = np.where(nu > 0.5, np.ceil(np.log2(np.maximum(nu, 0.5) / 0.5)), 0.0)
        table_flops = 0.0
        for m in range(0, N + 1):
            d = N + 1 - m
            table_flops += nf2 * 14 * 20 * d * d + float(q.sum()) * (16 * d ** 3 + 2 * d * d)
        t_tab = per["expo_table"]
        t_app = per["expo"]
        # rotations to and from the k = z frame (read and write the
        # spectrum twice) and the block products (read and write it once)
        apply_bytes = 6 * F
        if t_tab >= t_app:
            achieved = table_flops / (t_tab / 1e3) / 1e12
            roof = {"bound": "alu", "kernel": "expo_table (FP64)", "achieved": achieved, "peak": FP64_VALU_PEAK,
                    "unit": "TFLOP/s", "frac": achieved / FP64_VALU_PEAK,
                    "traffic": traffic_for("expo_table", "expo_homogeneous_128"),
                    "algorithmic_flops": table_flops, "avg_launch_ms": t_tab}
        else:
            achieved = apply_bytes / (t_app / 1e3) / 1e9
            roof = {"bound": "hbm", "kernel": "expo (frame rotations + block products)", "achieved": achieved,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                    "traffic": traffic_for("expo", "expo_homogeneous_128"),
                    "algorithmic_bytes": apply_bytes, "avg_launch_ms": t_app}
        roof["table_ms"] = t_tab
        roof["apply_ms"] = t_app
    else:
        flops = terms * expo_term_flops(N)
        t_expo = per["expo"]
        achieved = flops / (t_expo / 1e3) / 1e12
        roof = {"bound": "alu", "kernel": "expo (per-point series)", "achieved": achieved,
                "peak": FP32_VALU_PEAK, "unit": "TFLOP/s", "frac": achieved / FP32_VALU_PEAK,
                "traffic": traffic_for("expo", "expo_homogeneous_128"), "compulsory_bytes": 2 * F,
                "algorithmic_flops": flops, "avg_launch_ms": t_expo,
                "peak_without_packed_fp32": FP32_VALU_PEAK / 2}
    out = {"metric": "simulated time per second, exact propagation in a homogeneous medium",
           "value": T / (ms_expo / 1e3), "unit": "ps/s", "n_gpus": 1, "steps": reps,
           "warmup": 1, "ms_per_step": ms_expo, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": prec, "data": "synthetic",
           "config": {"workload": f"homogeneous {n}^3 P_{N} (mu_a {mua}, mu_s {mus}, g {g}), "
                                  f"dx {dx} mm, periodic grid, Gaussian pulse (sigma 2 voxels); "
                                  f"one advance = {T:.4f} ps = {K} RK4 steps of dt 0.2 dx/c",
                      "n": n, "order_N": N},
           "rk4_ms_same_interval": ms_rk4, "speedup_vs_rk4": ms_rk4 / ms_expo,
           "rk4_vs_exact_fluence_rel_l2": float(np.linalg.norm(rk - ex) / np.linalg.norm(ex)),
           "kernel_ms_per_launch": per,
           "taylor": {"theta": theta, "mean_substeps": float(sub.mean()), "max_substeps": float(sub.max()),
                      "mean_terms_per_point_of_the_series": terms / sub.size},
           "roofline": roof}
    print(json.dumps(out), flush=True)


def gmres_iteration_bytes(n, M, N, s, m, K):
    """Compulsory HBM bytes of one Arnoldi step averaged over a restart
    cycle of m steps. The operator: with K = 0 one application of S + Sigma
    (forward plane pass 2F, z derivative 2F, coupling 3F, inverse pass
    reading the spectrum, input and loss maps and writing the output
    3F + maps); with K > 0 a copy (2F), K RK4 steps without bookkeeping (per
    stage 2F + 2F + 3F and an inverse pass reading spectrum, stage input, u
    and maps and writing 1: 4F + maps, the first stage reading u once: one F
    less) and the difference (3F). Then two classical Gram-Schmidt passes
    against j + 1 basis vectors (inner products read j + 2 vectors, the
    update reads j + 2 and writes 1), the norm (F) and the normalisation
    (2F)."""
    F = M * n ** 3 * s
    maps = (N + 1) * n ** 3 * s
    if K == 0:
        op = 10 * F + maps
    else:
        op = 2 * F + K * (4 * (11 * F + maps) - F) + 3 * F
    tot = 0.0
    for j in range(m):
        tot += op + 2 * ((j + 2) * F + (j + 3) * F) + 3 * F
    return tot / m


def steady_bench(a):
    """Steady state of the absorbing-layer recipe (log-normal medium,
    collimated slab source) at n^3 / P_5 (n = 128 by default: at 64^3 a
    state of 38 MB sits in the caches, so an HBM roofline means little
    there) by device GMRES against time marching, both in FP32, each
    measured to the same distance from an FP64 GMRES reference."""
    import numpy as np
    import torch

    import rte_inputs as ri
    from paper_1801_06364_amd.rte import Solver

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    n = a.steady_n
    ref_wl = ri.workload("p5_steady", n=n, steps=0, precision="f64")
    r = Solver.from_workload(ref_wl, stream=stream)
    it_ref, res_ref = r.steady_gmres(tol=1e-10, restart=30, max_iters=4000, steps_per_apply=a.steady_k)
    ref = r.fluence()
    r.close()
    print(f"[steady] FP64 reference: {it_ref} Arnoldi steps, residual {res_ref:.1e}", file=sys.stderr,
          flush=True)

    def err(x):
        return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))

    wl = ri.workload("p5_steady", n=n, steps=0, precision="f32")
    g = Solver.from_workload(wl, stream=stream)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    it, res = g.steady_gmres(tol=a.steady_tol, restart=30, max_iters=4000, steps_per_apply=a.steady_k)
    t_gmres = time.perf_counter() - t0
    e_gmres = err(g.fluence())
    g.close()
    print(f"[steady] GMRES FP32: {it} Arnoldi steps, {t_gmres:.2f} s, fluence error {e_gmres:.2e}",
          file=sys.stderr, flush=True)
    # the same solve on the steady-state operator itself (no time steps)
    g = Solver.from_workload(wl, stream=stream)
    t0 = time.perf_counter()
    it_a, res_a = g.steady_gmres(tol=a.steady_tol, restart=30, max_iters=4000, steps_per_apply=0)
    t_a = time.perf_counter() - t0
    e_a = err(g.fluence())
    g.close()
    print(f"[steady] GMRES on S + Sigma FP32: {it_a} Arnoldi steps, {t_a:.2f} s, fluence error {e_a:.2e}",
          file=sys.stderr, flush=True)

    m = Solver.from_workload(wl, stream=stream, record_steps=0)
    steps, t_march, e_march = 0, 0.0, 1.0
    chunk = 100
    while e_march > e_gmres and t_march < a.steady_march_limit:
        ev0.record(stream)
        m.step(chunk)
        ev1.record(stream)
        stream.synchronize()
        t_march += ev0.elapsed_time(ev1) / 1e3
        steps += chunk
        e_march = err(m.fluence())
    m.close()
    print(f"[steady] marching FP32: {steps} steps, {t_march:.2f} s, fluence error {e_march:.2e}",
          file=sys.stderr, flush=True)
    bytes_it = gmres_iteration_bytes(n, wl.M, wl.N, 4, 30, a.steady_k)
    gbs = bytes_it * it / t_gmres / 1e9
    out = {"metric": "time to steady state (device GMRES vs time marching)",
           "value": t_gmres, "unit": "s", "n_gpus": 1, "steps": it, "warmup": 0,
           "ms_per_step": 1e3 * t_gmres / max(it, 1), "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"p5_steady recipe at {n}^3 (P_5, log-normal medium, absorbing "
                                  "layer, collimated slab source); target: the "
                                  f"fluence error GMRES reaches at relative residual {a.steady_tol:g} "
                                  f"(operator I - P^{a.steady_k}, P one RK4 step), against an FP64 "
                                  "GMRES solve at 1e-10",
                      "n": n, "order_N": wl.N, "restart": 30, "steps_per_apply": a.steady_k},
           "gmres": {"arnoldi_steps": it, "residual": res, "seconds": t_gmres,
                     "fluence_error": e_gmres},
           "gmres_on_S_plus_Sigma": {"arnoldi_steps": it_a, "residual": res_a, "seconds": t_a,
                                     "fluence_error": e_a},
           "marching": {"steps": steps, "seconds": t_march, "fluence_error": e_march,
                        "reached_target": e_march <= e_gmres},
           "speedup_vs_marching": t_march / t_gmres,
           "roofline": {"bound": "hbm", "kernel": "arnoldi step (operator + CGS2)",
                        "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                        "algorithmic_bytes": bytes_it}}
    print(json.dumps(out), flush=True)


def cfg3_bench(a):
    """The 256^3 / P_5 steady-state workload (log-normal medium, collimated
    slab source): FP32 time marching until the relative fluence change of a
    step drops below 1e-6 (steady state by marching, Sec. II.A / III.B),
    then the FP64 GPU march over the same number of steps n* (the same
    trajectory: the error of FP32 alone, at the full horizon), both timed.
    Fluence and FP64 integrated fluence compared by relative L2. Optionally
    (--cfg3-gmres) also the FP64 fixed point by GMRES on I - P^K."""
    import numpy as np
    import torch

    import rte_inputs as ri
    from paper_1801_06364_amd.rte import Solver

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    n, tol, chunk = 256, 1e-6, 500

    def rel(x, y):
        return float(np.linalg.norm(np.ravel(x) - np.ravel(y)) / np.linalg.norm(np.ravel(y)))

    def log(msg):
        print(f"[cfg3] {msg}", file=sys.stderr, flush=True)

    def march(prec, limit, stop_tol):
        m = Solver.from_workload(ri.workload("p5_steady", n=n, steps=0, precision=prec), stream=stream,
                                 record_steps=0)
        steps, t = 0, 0.0
        while steps < limit:
            k = min(chunk, limit - steps)
            t0 = time.perf_counter()
            if stop_tol > 0:
                took = m.run(k, stop_tol)
            else:
                m.step(k)
                took = k
            stream.synchronize()
            t += time.perf_counter() - t0
            steps += took
            log(f"{prec} march: {steps} steps, {t:.1f} s")
            if stop_tol > 0 and took < chunk:
                break
        out = (steps, t, m.fluence(), m.fluence(1))
        m.close()
        return out

    s32, t32, f32, p32 = march("f32", a.cfg3_max_steps, tol)
    converged = s32 < a.cfg3_max_steps
    s64, t64, f64, p64 = march("f64", s32, 0.0)
    out = {"metric": "steady state of the 256^3 P_5 workload by FP32 marching, against FP64 marching",
           "value": t32, "unit": "s", "n_gpus": 1, "steps": s32, "warmup": 0,
           "ms_per_step": 1e3 * t32 / max(s32, 1), "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "p5_steady: P_5 (36 moments), 256^3, log-normal mu_a / mu_s "
                                  "(correlation 20 voxels), g 0.85, 32-voxel absorbing layer, "
                                  "constant collimated slab source; march until the relative fluence "
                                  "change of a step < 1e-6",
                      "n": n, "order_N": 5, "steady_tol": tol},
           "march_fp32": {"steps": s32, "converged": converged, "seconds": t32},
           "march_fp64_same_steps": {"steps": s64, "seconds": t64},
           "fp32_vs_fp64": {"fluence": rel(f32, f64), "integrated_fluence": rel(p32, p64)}}
    if a.cfg3_gmres:
        g = Solver.from_workload(ri.workload("p5_steady", n=n, steps=0, precision="f64"), stream=stream)
        t0 = time.perf_counter()
        it, res = 0, 1.0
        while it < a.cfg3_max_arnoldi:
            k, res = g.steady_gmres(tol=1e-8, restart=a.cfg3_restart, max_iters=a.cfg3_restart,
                                    steps_per_apply=a.steady_k)
            it += k
            log(f"f64 GMRES: {it} Arnoldi steps, residual {res:.2e}, {time.perf_counter() - t0:.1f} s")
            if res <= 1e-8 or k == 0:
                break
        f_ref = g.fluence()
        g.close()
        out["gmres_fp64"] = {"arnoldi_steps": it, "residual": res, "seconds": time.perf_counter() - t0,
                             "fp32_march_vs_fixed_point": rel(f32, f_ref),
                             "fp64_march_vs_fixed_point": rel(f64, f_ref)}
    print(json.dumps(out), flush=True)


def paper_bench(a):
    """The paper's two experiments as synthetic workloads (Sec. III.A: P_21,
    64^3, 400 Euler steps; Sec. III.B: P_7, 64^3 with absorbing layer,
    25,000 Euler steps), timed on the GPU beside the paper's reported wall
    times (Tesla K40: 70 s and 223 s; context, other hardware)."""
    import numpy as np
    import torch

    import rte_inputs as ri
    from paper_1801_06364_amd.rte import Solver

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    out = {}
    for key, name, paper_s in (("E1_transient_P21", "paper_transient", 70.0),
                               ("E2_steady_pml_P7", "paper_pml_steady", 223.0)):
        wl = ri.workload(name, precision="f32")
        t0 = time.perf_counter()
        s = Solver.from_workload(wl, stream=stream)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        s.step(wl.steps)
        ev1.record(stream)
        stream.synchronize()
        wall = time.perf_counter() - t0
        ms = ev0.elapsed_time(ev1)
        fl = s.fluence()
        assert s.steps_done() == wl.steps and np.all(np.isfinite(fl))
        upd = wl.n ** 3 * wl.M * wl.steps
        out[key] = {"workload": f"{name}: {wl.n}^3, P_{wl.N} ({wl.M} moments), {wl.steps} forward "
                                f"Euler steps of {wl.dt} ps, FP32",
                    "gpu_seconds_stepping": ms / 1e3, "wall_seconds_with_setup": wall,
                    "ms_per_step": ms / wl.steps, "updates_per_s": upd / (ms / 1e3),
                    "paper_seconds_k40": paper_s, "ratio_vs_paper": paper_s / wall}
        s.close()
        print(f"[paper] {key}: {ms / 1e3:.2f} s stepping, {wall:.2f} s with setup "
              f"(paper {paper_s} s on a K40)", file=sys.stderr, flush=True)
        if name == "paper_pml_steady":
            g = Solver.from_workload(ri.workload(name, precision="f32", steps=0), stream=stream)
            t0 = time.perf_counter()
            it, res = g.steady_gmres(tol=1e-6, restart=30, max_iters=2000, steps_per_apply=20)
            t_g = time.perf_counter() - t0
            fg = g.fluence()
            g.close()
            out[key]["gmres_same_steady_state"] = {
                "seconds": t_g, "arnoldi_steps": it, "residual": res,
                "fluence_rel_diff_vs_25000_steps": float(np.linalg.norm(fg - fl) / np.linalg.norm(fl))}
            print(f"[paper] E2 by GMRES: {t_g:.2f} s, {it} Arnoldi steps", file=sys.stderr, flush=True)
    line = {"metric": "wall time of the paper's experiments (synthetic stand-ins)",
            "value": out["E2_steady_pml_P7"]["wall_seconds_with_setup"], "unit": "s", "n_gpus": 1,
            "higher_is_better": False, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "Sec. III.A transient (P_21) and Sec. III.B steady state with "
                                   "absorbing layer (P_7), 64^3 each"},
            "vs_baseline": None, "experiments": out}
    print(json.dumps(line), flush=True)


def adjoint_bench(a):
    """The adjoint configuration: 96^3 / P_3 / FP32 inclusion phantom, 1000
    RK4 steps with checkpoints every 32, loss = squared differences of 16
    detector series against the readings of a second phantom (seed 1005);
    forward and adjoint timed with HIP events; gradient checked against
    FP64 central differences at 20 seeded voxels."""
    import numpy as np
    import torch

    import rte_inputs as ri
    from paper_1801_06364_amd.rte import Solver

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    wl = ri.workload("p3_adjoint", precision="f32")
    n, steps, every = wl.n, wl.steps, 32
    tgt = ri.sphere_maps(n, wl.W, 5, seed=1005, radius=(3, 12))

    def readings(w, mu_a, mu_s, g):
        s = Solver.from_workload(w, mu_a=mu_a, mu_s=mu_s, g=g, stream=stream)
        s.step(steps)
        r = s.readings()
        s.close()
        return r

    target = readings(wl, *tgt)
    s = Solver.from_workload(wl, stream=stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    s.forward_checkpointed(steps, every)
    ev[1].record(stream)
    stream.synchronize()
    ms_fwd = ev[0].elapsed_time(ev[1])
    r = s.readings()
    djdr = 2.0 * (r - target)
    loss = float(((r - target) ** 2).sum())
    t0 = time.perf_counter()
    ga, gs = s.adjoint(djdr)
    ms_adj = (time.perf_counter() - t0) * 1e3
    s.close()
    print(f"[adjoint] forward {ms_fwd:.1f} ms, adjoint {ms_adj:.1f} ms, loss {loss:.4e}", file=sys.stderr,
          flush=True)
    # FP64 gradient and central differences of the FP64 loss
    w64 = ri.workload("p3_adjoint", precision="f64")
    s = Solver.from_workload(w64, stream=stream)
    s.forward_checkpointed(steps, every)
    r64 = s.readings()
    ga64, gs64 = s.adjoint(2.0 * (r64 - target))
    s.close()
    rng = np.random.default_rng(5)
    inside = np.argwhere((np.arange(n)[:, None, None] >= wl.W) & (np.arange(n)[:, None, None] < n - wl.W)
                         & (np.arange(n)[None, :, None] >= wl.W) & (np.arange(n)[None, :, None] < n - wl.W)
                         & (np.arange(n)[None, None, :] >= wl.W) & (np.arange(n)[None, None, :] < n - wl.W))
    mags = np.abs(ga64[tuple(inside.T)])
    strong = inside[mags >= np.quantile(mags, 0.9)]
    pick = strong[rng.choice(len(strong), 20, replace=False)]
    worst64 = worst32 = 0.0
    for v in pick:
        v = tuple(v)
        ma = wl.mu_a.copy()
        h = 1e-3 * ma[v]
        ma[v] += h
        jp = float(((readings(w64, ma, wl.mu_s, wl.g) - target) ** 2).sum())
        ma[v] -= 2 * h
        jm = float(((readings(w64, ma, wl.mu_s, wl.g) - target) ** 2).sum())
        fd = (jp - jm) / (2 * h)
        worst64 = max(worst64, abs(ga64[v] - fd) / abs(fd))
        worst32 = max(worst32, abs(ga[v] - fd) / abs(fd))
    upd = n ** 3 * wl.M * 4 * steps
    out = {"metric": "adjoint gradient of detector readings w.r.t. mu_a, mu_s (checkpointed RK4)",
           "value": upd / (ms_adj / 1e3), "unit": "updates/s", "n_gpus": 1, "steps": steps,
           "warmup": 0, "ms_per_step": ms_adj / steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"p3_adjoint: {n}^3, P_3, 16 detectors, {steps} RK4 steps, checkpoints "
                                  f"every {every}, target readings from the seed-1005 phantom"},
           "forward_ms": ms_fwd, "adjoint_ms": ms_adj, "adjoint_over_forward": ms_adj / ms_fwd,
           "forward_updates_per_s": upd / (ms_fwd / 1e3),
           "fd_check": {"voxels": 20, "selection": "seeded among the 10% largest |dJ/dmu_a| in the real domain",
                        "step": "1e-3 mu_a, FP64 forward runs",
                        "max_rel_err_fp64_gradient": worst64, "max_rel_err_fp32_gradient": worst32},
           "fp32_vs_fp64_gradient_rel_l2": float(np.linalg.norm(ga - ga64) / np.linalg.norm(ga64))}
    print(json.dumps(out), flush=True)


def accuracy_timed(name, steps):
    """FP32 against the FP64 GPU path on the timed configuration itself
    (full size, `steps` RK4 steps from the recipe's initial state):
    relative L2 of the final fluence, the integrated fluence and the
    flattened detector series. The FP64 GPU path stands in for the oracle at
    this size (the oracle takes about 12 s per step here); it matches the
    oracle to <= 1e-12 on every parity case, the full 128^3 / P_7 grid
    included."""
    import numpy as np

    import rte_inputs as ri
    from paper_1801_06364_amd.rte import Solver

    def rel(x, y):
        return float(np.linalg.norm(np.ravel(x) - np.ravel(y)) / np.linalg.norm(np.ravel(y)))

    res = {}
    for prec in ("f64", "f32"):
        s = Solver.from_workload(ri.workload(name, steps=steps, precision=prec))
        s.step(steps)
        res[prec] = (s.fluence(), s.fluence(1), s.readings())
        s.close()
    f64, f32 = res["f64"], res["f32"]
    return {"workload": f"{name} (the timed configuration), {steps} RK4 steps, FP32 vs FP64 GPU",
            "fluence": rel(f32[0], f64[0]), "integrated_fluence": rel(f32[1], f64[1]),
            "readings_series": rel(f32[2], f64[2])}


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
    ap.add_argument("--budget-gib", type=float, default=160.0)
    ap.add_argument("--slots", type=int, default=16, help="largest batch per configuration class")
    ap.add_argument("--chunk", type=int, default=16, help="time steps per queued batch chunk")
    ap.add_argument("--big-slots", type=int, default=16,
                    help="slots per batch for configurations above 512 MiB per solve")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--accuracy-steps", type=int, default=200,
                    help="RK4 steps of the FP32-vs-FP64 comparison on the timed configuration")
    ap.add_argument("--expo", action="store_true",
                    help="exact propagation vs RK4 marching in a homogeneous medium (separate JSON line)")
    ap.add_argument("--expo-reps", type=int, default=5)
    ap.add_argument("--steady", action="store_true",
                    help="steady state by device GMRES vs time marching (separate JSON line)")
    ap.add_argument("--adjoint", action="store_true",
                    help="the adjoint configuration with a finite-difference check (separate JSON line)")
    ap.add_argument("--paper", action="store_true",
                    help="the paper's two experiments, timed (separate JSON line)")
    ap.add_argument("--steady-tol", type=float, default=1e-5)
    ap.add_argument("--steady-k", type=int, default=20,
                    help="time steps per operator application of the steady GMRES")
    ap.add_argument("--steady-march-limit", type=float, default=60.0)
    ap.add_argument("--steady-n", type=int, default=128, help="grid of the --steady comparison")
    ap.add_argument("--cfg3", action="store_true",
                    help="256^3 P_5 steady state: FP32 march to a 1e-6 change vs FP64 GMRES (JSON line)")
    ap.add_argument("--cfg3-max-steps", type=int, default=30000)
    ap.add_argument("--cfg3-restart", type=int, default=16)
    ap.add_argument("--cfg3-max-arnoldi", type=int, default=480)
    ap.add_argument("--cfg3-gmres", action="store_true",
                    help="also the FP64 fixed point by GMRES (long at 256^3)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the hot path is a single-GPU solve "
              "and no multi-GPU path is implemented (independent solves shard one "
              "per GPU without exchange)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import rte_inputs as ri
    from paper_1801_06364_amd.rte import Solver

    if a.serving:
        return serving_bench(a)
    if a.expo:
        return expo_bench(a)
    if a.steady:
        return steady_bench(a)
    if a.cfg3:
        return cfg3_bench(a)
    if a.paper:
        return paper_bench(a)
    if a.adjoint:
        return adjoint_bench(a)

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

    upd_step = wl.n ** 3 * wl.M * stages_per_step(wl.scheme)
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
        out["accuracy"]["timed_config"] = accuracy_timed(a.workload, a.accuracy_steps)
    if not a.no_cpu_baseline:
        workers = int(os.environ.get("OMP_NUM_THREADS", "0")) or min(16, os.cpu_count() or 1)
        wlc = ri.workload(a.workload, steps=1)
        out["cpu_baseline"] = cpu_baseline(wlc, workers)
        print(f"[bench] cpu baseline: {out['cpu_baseline']['value']:.3e} updates/s",
              file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
