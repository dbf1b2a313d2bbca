"""Continuous-batching request server for P_N transport solves on one GPU.

Requests (grid size, P_N order, optical maps, step count) arrive over time.
A request is admitted as soon as it has arrived, a slot is free and its
device workspace (``rte_workspace_bytes``) fits the HBM budget next to the
requests already resident; admission is first-come first-served (the head
of the queue is never overtaken, so no request starves). Each admitted
request gets its own solver handle, device-resident state and HIP stream,
and all of its RK4 steps are queued at once as replays of its captured
step graph; requests on different streams run concurrently on the GPU, so
small grids fill the compute units left idle by large ones and newly
admitted requests start while earlier ones are still running. A request
retires when the event recorded after its last step completes; its
workspace is released and the next request can be admitted.

Admission has two lanes, each first-come first-served: requests whose
workspace exceeds ``large_bytes`` (large grids / high orders, which on their
own already keep HBM busy) share ``large_slots`` slots, the others the
remaining slots, so a short request never queues behind a long one and no
request is overtaken within its lane (no starvation). The total resident
workspace never exceeds the budget.

The one-at-a-time baseline serves the same trace first-come first-served on
one stream: each request's service time is measured alone, and the FIFO
single-server queue is replayed from those times.

Every result is computed by the same kernels in the same order whether a
request runs alone or in the mix, so the fluence is bitwise identical.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import rte


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float = 0.0
    finished: float = 0.0
    ok: bool = False
    error: str = ""
    updates: int = 0
    checksum: float = 0.0
    fluence: Optional[np.ndarray] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class Report:
    mode: str
    results: Dict[int, Result] = field(default_factory=dict)
    makespan: float = 0.0
    peak_resident_bytes: int = 0
    peak_slots: int = 0

    def latencies(self) -> np.ndarray:
        return np.array([r.latency for r in self.results.values() if r.ok])

    def summary(self) -> dict:
        lat = self.latencies()
        ups = sum(r.updates for r in self.results.values() if r.ok)
        return {"mode": self.mode, "requests": len(self.results),
                "failed": sum(1 for r in self.results.values() if not r.ok),
                "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else None,
                "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else None,
                "mean_latency_s": float(lat.mean()) if lat.size else None,
                "makespan_s": self.makespan,
                "updates_per_s": ups / self.makespan if self.makespan > 0 else None,
                "peak_resident_GiB": self.peak_resident_bytes / 2 ** 30,
                "peak_concurrent": self.peak_slots}


def footprint(spec, precision: str = "f32") -> int:
    """Device bytes a request needs (its solver workspace)."""
    prec = rte.RTE_FP64 if precision == "f64" else rte.RTE_FP32
    cfg, _ = rte.make_config(spec.n, spec.N, prec, 0.25, 0.3, 0.0, spec.n // 8, 0.01, 1.0)
    return rte.rte_workspace_bytes(cfg)


def updates_of(spec) -> int:
    return spec.n ** 3 * (spec.N + 1) ** 2 * 4 * spec.steps


class Server:
    """Continuous batching over ``max_slots`` concurrent solves within an
    HBM budget of ``budget_bytes``; at most ``large_slots`` of them may be
    requests larger than ``large_bytes``."""

    def __init__(self, budget_bytes: int = 12 << 30, max_slots: int = 12,
                 precision: str = "f32", keep_fluence: bool = False,
                 large_bytes: int = 512 << 20, large_slots: int = 2):
        import torch
        self.torch = torch
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.large_bytes = int(large_bytes)
        self.large_slots = max(1, min(int(large_slots), self.max_slots - 1)) \
            if self.max_slots > 1 else 1
        self.precision = precision
        self.keep = keep_fluence
        self.streams = [torch.cuda.Stream() for _ in range(self.max_slots)]

    def _finish(self, res: Result, solver, t0: float):
        try:
            solver.steps_done()            # raises on a non-finite / runaway run
            fl = solver.fluence()
            res.ok = bool(np.all(np.isfinite(fl)))
            if not res.ok:
                res.error = "non-finite fluence"
            res.checksum = float(fl.sum())
            if self.keep:
                res.fluence = fl
        except rte.RteError as e:          # e.g. unstable run
            res.ok, res.error = False, str(e)
        res.finished = time.perf_counter() - t0

    def serve(self, specs: List, arrivals: List[float]) -> Report:
        """Serve requests whose arrival times (seconds from start) are given."""
        order = sorted(range(len(specs)), key=lambda i: arrivals[i])
        incoming = collections.deque(order)
        sizes = [footprint(sp, self.precision) for sp in specs]
        lanes = {False: collections.deque(), True: collections.deque()}   # large?
        slots = {True: list(range(self.large_slots)),
                 False: list(range(self.large_slots, self.max_slots))}
        if not slots[False]:
            slots[False] = slots[True]
        rep = Report("batched")
        active = {}            # slot -> (index, solver, event, bytes, large)
        resident = 0
        t0 = time.perf_counter()
        while incoming or active or lanes[False] or lanes[True]:
            now = time.perf_counter() - t0
            progressed = False
            for slot in list(active):
                i, solver, ev, nb, big = active[slot]
                if ev.query():
                    res = rep.results[specs[i].rid]
                    self._finish(res, solver, t0)
                    solver.close()
                    del active[slot]
                    slots[big].append(slot)
                    resident -= nb
                    progressed = True
            while incoming and arrivals[incoming[0]] <= now:
                i = incoming.popleft()
                lanes[sizes[i] > self.large_bytes].append(i)
            for big in (False, True):
                q = lanes[big]
                while q and slots[big]:
                    i = q[0]
                    nb = sizes[i]
                    if resident + nb > self.budget and active:
                        break               # wait for memory; keep FIFO order
                    q.popleft()
                    slot = slots[big].pop()
                    spec = specs[i]
                    res = Result(spec.rid, arrivals[i], admitted=time.perf_counter() - t0,
                                 updates=updates_of(spec))
                    rep.results[spec.rid] = res
                    try:
                        solver = rte.Solver.from_workload(spec.workload(self.precision),
                                                          stream=self.streams[slot], record_steps=0)
                        solver.step(spec.steps)
                    except rte.RteError as e:
                        res.ok, res.error = False, str(e)
                        res.finished = time.perf_counter() - t0
                        slots[big].append(slot)
                        continue
                    ev = self.torch.cuda.Event()
                    ev.record(self.streams[slot])
                    active[slot] = (i, solver, ev, nb, big)
                    resident += nb
                    rep.peak_resident_bytes = max(rep.peak_resident_bytes, resident)
                    rep.peak_slots = max(rep.peak_slots, len(active))
                    progressed = True
            if not progressed:
                time.sleep(2e-4)
        rep.makespan = time.perf_counter() - t0 - (min(arrivals) if arrivals else 0.0)
        return rep

    def service_times(self, specs: List) -> Dict[int, Result]:
        """Each request alone on one stream (back to back): the measured
        service time is finished - admitted."""
        out = {}
        st = self.streams[0]
        t0 = time.perf_counter()
        for spec in specs:
            res = Result(spec.rid, 0.0, admitted=time.perf_counter() - t0, updates=updates_of(spec))
            try:
                solver = rte.Solver.from_workload(spec.workload(self.precision), stream=st,
                                                  record_steps=0)
                solver.step(spec.steps)
                st.synchronize()
                self._finish(res, solver, t0)
                solver.close()
            except rte.RteError as e:
                res.ok, res.error = False, str(e)
                res.finished = time.perf_counter() - t0
            out[spec.rid] = res
        return out


def fifo_replay(specs: List, arrivals: List[float], alone: Dict[int, Result]) -> Report:
    """First-come first-served single-server queue with the measured
    one-at-a-time service times."""
    rep = Report("one_at_a_time")
    t_free = 0.0
    for i in sorted(range(len(specs)), key=lambda j: arrivals[j]):
        a = alone[specs[i].rid]
        svc = a.finished - a.admitted
        start = max(arrivals[i], t_free)
        t_free = start + svc
        rep.results[specs[i].rid] = Result(specs[i].rid, arrivals[i], start, t_free, a.ok, a.error,
                                           a.updates, a.checksum)
    first = min(arrivals) if arrivals else 0.0
    rep.makespan = t_free - first
    rep.peak_slots = 1
    return rep


def poisson_arrivals(specs: List, rate: float) -> List[float]:
    """Arrival times from the specs' unit-mean exponential gaps at ``rate``
    requests per second."""
    t, out = 0.0, []
    for s in specs:
        t += s.gap / rate
        out.append(t)
    return out
