"""Continuous-batching request server for P_N transport solves on one GPU.

Requests (grid size, P_N order, optical maps, step count) arrive over time.
Requests of one configuration class (grid size and order; spacing, time
step, layer and precision follow from them) share a batch engine
(``rte.Batch``): up to ``slots`` resident solves in one device workspace,
every kernel of a time step launched once for all of them (the slot is a grid
coordinate) from a captured graph, in chunks of ``chunk`` steps on the
engine's own stream. Engines of different classes run on different streams
and overlap on the GPU.

Admission: a request waits in its class's first-come first-served queue
until its engine has a free slot; an engine's workspace is allocated when
its class first needs it and counts against the HBM budget, and idle engines
are released when another class needs the memory. The oldest waiting request
has priority for memory (no other engine is created while it waits), so no
request starves. Building a request's phantom and uploading its tables and
state (``rte_batch_admit``) happen on worker threads; the serving thread only
queues chunks, polls the engines' control-block copies (non-blocking) and
reads finished results, so a large admission never delays the retirement of
other requests.

The one-at-a-time baseline serves the same trace first-come first-served:
each request's service time is measured alone (its own solver and step
graph), and the single-server queue is replayed from those times.

A slot runs the same kernels in the same order as a solver alone, so every
fluence is bitwise identical alone and in the mix.
"""
from __future__ import annotations

import collections
import hashlib
import time
from concurrent.futures import ThreadPoolExecutor
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
    digest: str = ""            # SHA-256 of the final fluence's bytes
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
    peak_slots: int = 0          # requests running at once (all engines)
    peak_batch: int = 0          # requests running at once in one batch (one launch per kernel)

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
                "peak_concurrent": self.peak_slots, "peak_batch": self.peak_batch}


def updates_of(spec) -> int:
    return spec.n ** 3 * (spec.N + 1) ** 2 * 4 * spec.steps


def digest_of(fl: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(fl).tobytes()).hexdigest()


def class_of(spec):
    """Configuration class of a request: requests of one class share a
    batch. A request's spacing, time step and layer follow from its grid
    size (RequestSpec.workload), so the class is (grid size, order)."""
    return (spec.n, spec.N)


class _Engine:
    """One batch of a configuration class and its serving state."""

    def __init__(self, key, wl, slots, precision, chunk):
        self.key = key
        self.batch = rte.Batch(wl.n, wl.N, wl.dx, wl.c, wl.dt, wl.W, slots, wl.mu0, wl.mu1,
                               precision=precision, n_det=0, record_steps=0)
        self.nbytes = self.batch.workspace.numel()
        self.free = list(range(slots - 1, -1, -1))
        self.pending = {}        # slot -> (index, future) while staging
        self.running = {}        # slot -> index
        self.chunk = chunk

    def busy(self) -> bool:
        return bool(self.pending or self.running)

    def close(self):
        self.batch.close()


class Server:
    """Continuous batching within an HBM budget of ``budget_bytes``; each
    class's engine holds up to ``max_slots`` solves (``big_slots`` for
    classes whose solves take more than ``big_bytes`` each, fewer if one
    class would take more than ``class_share`` of the budget)."""

    def __init__(self, budget_bytes: int = 48 << 30, max_slots: int = 16, precision: str = "f32",
                 keep_fluence: bool = False, chunk: int = 16, class_share: float = 0.25,
                 workers: int = 2, big_bytes: int = 512 << 20, big_slots: int = 16):
        import torch
        self.torch = torch
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.precision = precision
        self.keep = keep_fluence
        self.chunk = int(chunk)
        self.class_share = float(class_share)
        self.workers = int(workers)
        self.big_bytes = int(big_bytes)
        self.big_slots = int(big_slots)

    def _slots_for(self, spec):
        wl = spec.workload(self.precision)
        cfg, _ = rte.make_config(wl.n, wl.N, rte.RTE_FP64 if self.precision == "f64" else rte.RTE_FP32,
                                 wl.dx, wl.c, wl.dt, wl.W, wl.mu0, wl.mu1)
        per = int(rte.lib().rte_batch_slot_bytes(cfg))
        cap = self.big_slots if per > self.big_bytes else self.max_slots
        return max(1, min(cap, int(self.class_share * self.budget) // per)), per

    @staticmethod
    def _admit(engine, slot, spec, precision):
        wl = spec.workload(precision)
        engine.batch.admit(slot, wl.mu_a, wl.mu_s, wl.g, spec.steps, psi0=wl.psi0, q=wl.q)

    def serve(self, specs: List, arrivals: List[float]) -> Report:
        """Serve requests whose arrival times (seconds from start) are given."""
        order = sorted(range(len(specs)), key=lambda i: arrivals[i])
        incoming = collections.deque(order)
        waiting = collections.OrderedDict()     # class -> deque of request indices (FIFO)
        engines: Dict[tuple, _Engine] = {}
        slot_info = {}
        for i, sp in enumerate(specs):
            k = class_of(sp)
            if k not in slot_info:
                slot_info[k] = self._slots_for(sp)
        rep = Report("batched")
        resident = 0
        pool = ThreadPoolExecutor(self.workers)
        t0 = time.perf_counter()
        try:
            while incoming or any(waiting.values()) or any(e.busy() for e in engines.values()):
                now = time.perf_counter() - t0
                while incoming and arrivals[incoming[0]] <= now:
                    i = incoming.popleft()
                    waiting.setdefault(class_of(specs[i]), collections.deque()).append(i)
                # admissions: per class FIFO; the oldest waiting request has
                # priority for memory
                oldest = min((q[0] for q in waiting.values() if q), key=lambda j: arrivals[j], default=None)
                order_k = sorted((k for k, q in waiting.items() if q), key=lambda k: arrivals[waiting[k][0]])
                for k in order_k:
                    q = waiting[k]
                    if oldest is not None and k != class_of(specs[oldest]) and \
                            class_of(specs[oldest]) not in engines:
                        break   # the oldest request waits for memory: others do not overtake it
                    while q:
                        e = engines.get(k)
                        if e is None:
                            slots, per = slot_info[k]
                            if per > self.budget:
                                i = q.popleft()   # cannot fit even alone
                                rep.results[specs[i].rid] = Result(specs[i].rid, arrivals[i], now, now,
                                                                   False, "exceeds the HBM budget",
                                                                   updates_of(specs[i]))
                                continue
                            slots = min(slots, self.budget // per)
                            if resident + slots * per > self.budget:
                                for kk in [kk for kk, ee in engines.items() if not ee.busy()]:
                                    resident -= engines[kk].nbytes
                                    engines.pop(kk).close()
                            if resident + slots * per > self.budget:
                                break
                            e = engines[k] = _Engine(k, specs[q[0]].workload(self.precision), slots,
                                                     self.precision, self.chunk)
                            resident += e.nbytes
                            rep.peak_resident_bytes = max(rep.peak_resident_bytes, resident)
                        if not e.free:
                            break
                        i = q.popleft()
                        slot = e.free.pop()
                        sp = specs[i]
                        rep.results[sp.rid] = Result(sp.rid, arrivals[i], admitted=time.perf_counter() - t0,
                                                     updates=updates_of(sp))
                        e.pending[slot] = (i, pool.submit(self._admit, e, slot, sp, self.precision))
                # staged admissions become running at the engine's next chunk
                for e in engines.values():
                    for slot, (i, fut) in list(e.pending.items()):
                        if not fut.done():
                            continue
                        del e.pending[slot]
                        err = fut.exception()
                        if err is not None:
                            res = rep.results[specs[i].rid]
                            res.ok, res.error = False, str(err)
                            res.finished = time.perf_counter() - t0
                            e.free.append(slot)
                        else:
                            e.running[slot] = i
                rep.peak_slots = max(rep.peak_slots, sum(len(e.running) for e in engines.values()))
                rep.peak_batch = max([rep.peak_batch] + [len(e.running) for e in engines.values()])
                # queue chunks, poll, retire
                progressed = False
                for e in engines.values():
                    if not e.running:
                        continue
                    steps, status, in_flight = e.batch.poll()
                    for slot, i in list(e.running.items()):
                        st = status[slot]
                        if st not in (rte.RTE_SLOT_DONE, rte.RTE_SLOT_FAILED):
                            continue
                        res = rep.results[specs[i].rid]
                        if st == rte.RTE_SLOT_DONE:
                            fl = e.batch.fluence(slot)
                            res.ok = bool(np.all(np.isfinite(fl)))
                            res.error = "" if res.ok else "non-finite fluence"
                            res.digest = digest_of(fl)
                            if self.keep:
                                res.fluence = fl
                        else:
                            res.ok, res.error = False, "unstable run (non-finite or runaway fluence)"
                        res.finished = time.perf_counter() - t0
                        e.batch.release(slot)
                        del e.running[slot]
                        e.free.append(slot)
                        progressed = True
                    if e.running and in_flight < 2:
                        e.batch.step(e.chunk)     # keeps two chunks queued per engine
                        progressed = True
                if not progressed:
                    time.sleep(2e-4)
        finally:
            pool.shutdown(wait=True)
            for e in engines.values():
                e.close()
        rep.makespan = time.perf_counter() - t0 - (min(arrivals) if arrivals else 0.0)
        return rep

    def service_times(self, specs: List) -> Dict[int, Result]:
        """Each request alone on one stream (back to back), through its own
        solver and captured step graph: the measured service time is
        finished - admitted."""
        out = {}
        st = self.torch.cuda.Stream()
        t0 = time.perf_counter()
        for spec in specs:
            res = Result(spec.rid, 0.0, admitted=time.perf_counter() - t0, updates=updates_of(spec))
            try:
                solver = rte.Solver.from_workload(spec.workload(self.precision), stream=st,
                                                  record_steps=0)
                solver.step(spec.steps)
                st.synchronize()
                solver.steps_done()            # raises on a non-finite / runaway run
                fl = solver.fluence()
                res.ok = bool(np.all(np.isfinite(fl)))
                res.error = "" if res.ok else "non-finite fluence"
                res.digest = digest_of(fl)
                if self.keep:
                    res.fluence = fl
                res.finished = time.perf_counter() - t0
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
                                           a.updates, a.digest)
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
