"""Host logic of the continuous-batching serving loop, run against a
deterministic stand-in for the device (no GPU): admission in arrival order
within the device-memory budget, rejection of requests larger than the
budget, joining a running batch at a step boundary, release of finished
requests and their budget, and the reported statistics."""
import threading
import time

import numpy as np
import pytest

serve = pytest.importorskip("paper_2412_08981_amd.serve")
Request, Server = serve.Request, serve.Server


class _Info:
    def __init__(self, running, iterations):
        self.running, self.iterations, self.relres, self.status = running, iterations, 1e-9, 0


class _System:
    def __init__(self, rid, need):
        self.rid, self.need, self.steps = rid, need, 0


class _Batch:
    def __init__(self, systems):
        self.systems = list(systems)


class FakeEngine:
    """Each request's system needs a fixed number of steps; a step of a batch
    advances every member by one and takes `step_s` seconds."""

    def __init__(self, sizes, need, step_s=0.001, setup_s=0.0):
        self.sizes, self.need, self.step_s, self.setup_s = sizes, need, step_s, setup_s
        self.events = []  # (kind, data) in order
        self.alive = set()
        self.lock = threading.Lock()

    def system_bytes(self, h, restart):
        return self.sizes[h]

    def assemble(self, h, kappa, b, restart, nbytes):
        assert nbytes == self.sizes[h]
        time.sleep(self.setup_s)
        s = _System(kappa, self.need[kappa])
        with self.lock:
            self.alive.add(s)
        return s, ("b", kappa)

    def batch(self, systems, restart, rtol, max_it, graph):
        self.events.append(("form", [x.rid for x in systems]))
        return _Batch(systems)

    def start(self, batch, slot, bd):
        assert bd == ("b", batch.systems[slot].rid)
        self.events.append(("start", batch.systems[slot].rid))

    def step(self, batch):
        time.sleep(self.step_s)
        for x in batch.systems:
            if x.steps < x.need:
                x.steps += 1
        self.events.append(("step", [x.rid for x in batch.systems]))

    def result(self, batch, slot, system, keep_x):
        return _Info(system.steps < system.need, system.steps), None

    def release_batch(self, batch):
        pass

    def release_system(self, system):
        with self.lock:
            self.alive.remove(system)


def _req(rid, key, t):
    return Request(rid, key, rid, t)  # the "kappa" carries the request id for the fake


def test_budget_admission_order_and_rejection():
    sizes = {"small": 3, "big": 5, "huge": 20}
    keys = ["big", "big", "small", "huge", "small", "big", "small"]
    need = {i: 3 + (i % 3) for i in range(len(keys))}
    eng = FakeEngine(sizes, need)
    srv = Server({k: k for k in sizes}, 10, engine=eng)
    reqs = [_req(i, k, 0.0) for i, k in enumerate(keys)]
    st = srv.run(reqs)
    assert st["rejected"] == 1 and reqs[3].status == "rejected"
    assert st["completed"] == len(keys) - 1
    assert srv.max_used <= 10 and srv.used == 0 and not eng.alive
    done = [r for r in reqs if r.status == "done"]
    assert all(r.iterations == need[r.rid] for r in done)
    # admission strictly in arrival order (the queue head blocks the rest)
    t_adm = [r.t_admit for r in done]
    assert t_adm == sorted(t_adm)
    # latencies and throughput are reported
    assert st["p50_ms"] > 0 and st["p99_ms"] >= st["p50_ms"] and st["solves_per_s"] > 0


def test_late_request_joins_the_running_batch():
    sizes = {"a": 1}
    need = {0: 40, 1: 4}
    eng = FakeEngine(sizes, need, step_s=0.002)
    srv = Server({"a": "a"}, 10, engine=eng)
    reqs = [_req(0, "a", 0.0), _req(1, "a", 0.02)]
    st = srv.run(reqs)
    assert st["completed"] == 2
    # request 1 started while request 0 was running: a batch holding both was
    # formed after request 0 had already taken steps
    first_step = next(i for i, e in enumerate(eng.events) if e[0] == "step")
    joint = [i for i, e in enumerate(eng.events) if e == ("form", [0, 1])]
    assert joint and joint[0] > first_step
    # and the short request finished first, leaving request 0 to finish alone
    assert reqs[1].t_done < reqs[0].t_done
    assert ("form", [0]) in eng.events[joint[0]:]
    assert reqs[0].iterations == 40 and reqs[1].iterations == 4


def test_budget_holds_back_until_release():
    sizes = {"x": 6}
    need = {0: 5, 1: 5}
    eng = FakeEngine(sizes, need)
    srv = Server({"x": "x"}, 10, engine=eng)  # room for one at a time
    reqs = [_req(0, "x", 0.0), _req(1, "x", 0.0)]
    st = srv.run(reqs)
    assert st["completed"] == 2 and srv.max_used == 6
    assert reqs[1].t_admit >= reqs[0].t_done
