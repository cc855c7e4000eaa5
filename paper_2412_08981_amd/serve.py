"""Continuous-batching serving loop over resident mesh hierarchies.

Requests (a hierarchy and a parameter of the coefficient) arrive over time.
A request is admitted when the device-memory budget has room for its system
(values, factors, Krylov workspace); its numeric setup (assembly + LU) runs
on a worker thread and its own stream, overlapping the solves in flight.
Every solve in flight advances one Arnoldi step per launch sequence of the
library's batch engine; when requests finish or new ones are ready, the
batch is re-formed at the next step boundary (each system keeps its solve
state on the device, so a re-formed batch continues where it was).  The
structure of every hierarchy (partition, transfers, patterns) is set up once
and reused by every request on it (the paper's parametric reuse of the mesh
hierarchy, Section 1 and Section 2.1).

Each system's arithmetic is independent of its batch neighbours, so a
request's result is the same alone and in the mix.
"""
from __future__ import annotations

import threading
import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import nnms


@dataclass
class Request:
    rid: int
    key: object  # hierarchy key
    kappa: object  # workloads.KappaField-like (kind/value/centres/mu/width)
    t_arrival: float  # seconds after the start of the run
    b: Optional[np.ndarray] = None  # None: the assembled load vector
    t_admit: float = float("nan")
    t_ready: float = float("nan")
    t_done: float = float("nan")
    status: str = "queued"  # queued, rejected, assembling, solving, done, failed
    iterations: int = 0
    relres: float = float("nan")
    x: Optional[np.ndarray] = None
    nbytes: int = 0
    error: str = ""
    shared_steps: int = 0  # steps this request ran with at least one other request in the batch


class DeviceEngine:
    """The device side of the serving loop: the library's systems and batches
    on PyTorch streams.  The loop itself only calls these methods, so its
    host logic runs unchanged against any object with the same methods."""

    def __init__(self, workers: int = 1):
        import torch

        self.torch = torch
        self.streams = [torch.cuda.Stream() for _ in range(workers)]
        # the loop's own stream: batch plans order themselves after it, so
        # forming a batch does not wait for the factorisations running on
        # the workers' streams (the null stream would)
        self.loop_stream = torch.cuda.Stream()
        self._tls = threading.local()
        self._ix = 0
        self._lock = threading.Lock()

    def system_bytes(self, h, restart: int) -> int:
        return h.system_bytes(restart)

    # numeric setup on the calling worker thread's own stream, within the
    # bytes admitted for it (the library refuses an assembly that needs more)
    def assemble(self, h, kappa, b, restart: int, nbytes: int):
        with self._lock:
            if not hasattr(self._tls, "stream"):
                self._tls.stream = self.streams[self._ix % len(self.streams)]
                self._ix += 1
        s = nnms.System(h, kappa, 1.0, stream=self._tls.stream, restart_cap=restart, budget=nbytes)
        b = s.rhs() if b is None else np.asarray(b, dtype=np.float64)
        bd = self.torch.from_numpy(b).to("cuda")
        self.torch.cuda.current_stream().synchronize()
        return s, bd

    def batch(self, systems, restart, rtol, max_it, graph):
        return nnms.Batch(systems, restart, rtol, max_it, graph=graph, stream=self.loop_stream)

    def start(self, batch, slot: int, bd) -> None:
        batch.start(slot, bd.data_ptr())

    def step(self, batch) -> None:
        batch.step(1)

    def result(self, batch, slot: int, system, keep_x: bool):
        """(info, x or None) of a slot; info.running tells whether it goes on."""
        torch = self.torch
        xo = torch.empty(system.n[0], dtype=torch.float64, device="cuda") if keep_x else None
        info = batch.result(slot, None if xo is None else xo.data_ptr())
        x = None
        if xo is not None and not info.running:
            torch.cuda.synchronize()
            x = xo.cpu().numpy()
        return info, x

    def release_batch(self, batch) -> None:
        batch.destroy()

    def release_system(self, system) -> None:
        system.destroy()


class Server:
    def __init__(self, hierarchies: Dict[object, "nnms.Hierarchy"], budget_bytes: int, restart: int = 30,
                 rtol: float = 1e-8, max_it: int = 1000, graph: bool = False, keep_x: bool = False,
                 workers: int = 1, engine=None):
        self.engine = engine if engine is not None else DeviceEngine(workers)
        self.h = hierarchies
        self.budget = int(budget_bytes)
        self.used = 0
        self.max_used = 0
        self.restart, self.rtol, self.max_it, self.graph = restart, rtol, max_it, graph
        self.keep_x = keep_x
        self.sizes = {k: self.engine.system_bytes(h, restart) for k, h in hierarchies.items()}
        self.pool = ThreadPoolExecutor(max_workers=workers)
        self.batch_forms = 0
        self.steps = 0
        self.max_active = 0  # most requests stepped together
        # host seconds spent in each part of the loop
        self.t_form = 0.0  # building and destroying batch plans, starting new slots
        self.t_create = 0.0  # of which: building plans
        self.t_release = 0.0  # of which: destroying plans
        self.t_start = 0.0  # of which: starting new slots
        self.t_step = 0.0  # launching one Arnoldi step and waiting for it
        self.t_result = 0.0  # reading slot results, releasing finished systems

    def _assemble(self, req: Request):
        return self.engine.assemble(self.h[req.key], req.kappa, req.b, self.restart, req.nbytes)

    def run(self, requests: List[Request], log=None) -> dict:
        eng = self.engine
        reqs = sorted(requests, key=lambda r: r.t_arrival)
        arrivals = deque(reqs)
        queue: deque = deque()
        assembling = {}  # future -> req
        active: List[tuple] = []  # (req, system, bdev)
        ready: List[tuple] = []
        batch = None
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        remaining = len(reqs)
        while remaining > 0:
            t = now()
            while arrivals and arrivals[0].t_arrival <= t:
                r = arrivals.popleft()
                r.nbytes = self.sizes[r.key]
                if r.nbytes > self.budget:
                    r.status, r.error = "rejected", "exceeds the device-memory budget"
                    remaining -= 1
                else:
                    queue.append(r)
            # admission in arrival order while the budget has room
            while queue and self.used + queue[0].nbytes <= self.budget:
                r = queue.popleft()
                self.used += r.nbytes
                self.max_used = max(self.max_used, self.used)
                r.t_admit, r.status = now(), "assembling"
                assembling[self.pool.submit(self._assemble, r)] = r
            for fut in [f for f in assembling if f.done()]:
                r = assembling.pop(fut)
                try:
                    s, bd = fut.result()
                    r.t_ready, r.status = now(), "solving"
                    ready.append((r, s, bd))
                except Exception as e:  # assembly failed: release its budget
                    r.status, r.error, r.t_done = "failed", str(e), now()
                    self.used -= r.nbytes
                    remaining -= 1
            if ready:
                # re-form the batch with the newcomers
                tf = time.perf_counter()
                old = batch
                members = active + ready
                batch = eng.batch([m[1] for m in members], self.restart, self.rtol, self.max_it, self.graph)
                self.batch_forms += 1
                t1 = time.perf_counter()
                if old is not None:
                    eng.release_batch(old)
                t2 = time.perf_counter()
                for k in range(len(active), len(members)):
                    eng.start(batch, k, members[k][2])
                active, ready = members, []
                t3 = time.perf_counter()
                self.t_form += t3 - tf
                self.t_create += t1 - tf
                self.t_release += t2 - t1
                self.t_start += t3 - t2
            if batch is None or not active:
                # idle: wait for the next arrival or assembly
                time.sleep(0.0005)
                continue
            ts = time.perf_counter()
            eng.step(batch)
            self.steps += 1
            self.max_active = max(self.max_active, len(active))
            if len(active) > 1:
                for m in active:
                    m[0].shared_steps += 1
            tr = time.perf_counter()
            self.t_step += tr - ts
            finished, still = [], []
            for k, (r, s, bd) in enumerate(active):
                info, x = eng.result(batch, k, s, self.keep_x)
                if not info.running:
                    r.iterations, r.relres = info.iterations, info.relres
                    r.status = "done" if info.status == 0 else "failed"
                    r.x = x
                    r.t_done = now()
                    finished.append((r, s, bd))
                else:
                    still.append((r, s, bd))
            self.t_result += time.perf_counter() - tr
            if finished:
                tf = time.perf_counter()
                old = batch
                batch = eng.batch([m[1] for m in still], self.restart, self.rtol, self.max_it, self.graph) if still else None
                self.batch_forms += 1
                t1 = time.perf_counter()
                eng.release_batch(old)
                t2 = time.perf_counter()
                self.t_form += t2 - tf
                self.t_create += t1 - tf
                self.t_release += t2 - t1
                tr = time.perf_counter()
                for r, s, bd in finished:
                    eng.release_system(s)
                    self.used -= r.nbytes
                    remaining -= 1
                    if log:
                        log(f"[serve] request {r.rid} ({r.key}) done: {r.iterations} its, latency "
                            f"{1e3 * (r.t_done - r.t_arrival):.1f} ms")
                self.t_result += time.perf_counter() - tr
                active = still
        if batch is not None:
            eng.release_batch(batch)
        self.pool.shutdown(wait=True)
        out = self.stats(reqs)
        setup = [r.t_ready - r.t_admit for r in reqs if r.status == "done"]
        out.update({"max_bytes_admitted": self.max_used, "host_s_batch_forms": self.t_form,
                    "host_s_batch_create": self.t_create, "host_s_batch_release": self.t_release,
                    "host_s_slot_start": self.t_start, "host_s_steps": self.t_step,
                    "host_s_results": self.t_result,
                    "numeric_setup_ms_mean": float(np.mean(setup) * 1e3) if setup else float("nan")})
        return out

    @staticmethod
    def stats(reqs: List[Request]) -> dict:
        done = [r for r in reqs if r.status == "done"]
        lat = np.array([r.t_done - r.t_arrival for r in done])
        out = {"requests": len(reqs), "completed": len(done),
               "rejected": sum(r.status == "rejected" for r in reqs),
               "failed": sum(r.status == "failed" for r in reqs)}
        if done:
            span = max(r.t_done for r in done) - min(r.t_arrival for r in reqs)
            out.update({
                "solves_per_s": len(done) / span if span > 0 else float("nan"),
                "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "mean_ms": float(lat.mean() * 1e3),
                "max_relres": float(max(r.relres for r in done)),
                "iterations_mean": float(np.mean([r.iterations for r in done])),
            })
        return out
