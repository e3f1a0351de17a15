"""Continuous batching of independent CTMRG environment solves on one GPU.

Requests (site tensors of one (d, D, chi) each) arrive over time, e.g. from a
variational optimiser or a parameter sweep.  The server admits a request as
soon as a slot is free and its exact workspace (ctm_workspace_size) fits the
HBM budget, gives it its own HIP stream and keeps its environment resident.
Every tick it enqueues one CTM iteration (with the corner-spectrum change
delta) for each admitted solve whose previous iteration has finished, so the
GPU works on many solves at once; a solve that has converged (delta < tol) or
reached max_iters is finished with its energy, and its slot and memory are
freed for the next request.  Latency is arrival -> energy returned.

A request may carry a starting environment (`env`, the 16 named tensors of
an earlier solve of nearby tensors): the solve then resumes from it instead
of the traced-boundary start, the reuse of environments across optimisation
steps that the paper relies on (Sec. V, fast full update; Sec. IV,
environments "iteratively updated and reused").  With `return_env` the
final environment comes back with the result, for the next request.

Results do not depend on the mix: each solve runs the same kernels on its own
data and stream, with fixed reduction orders, so a solve alone and a solve in
the mix give identical numbers.

The scheduling logic is independent of the GPU: ``GpuBackend`` drives
libctm.so, ``FakeBackend`` (tests) scripts durations and sizes on a virtual
clock.
"""

from __future__ import annotations

import time
from dataclasses import dataclass
from typing import Any, Dict, List, Optional


@dataclass
class Request:
    id: int
    d: int
    D: int
    chi: int
    seed: int
    t_arrival: float = 0.0
    max_iters: int = 30
    tol: float = 1e-6
    precision: int = 1          # FP32 chains
    env: Optional[Dict[str, Any]] = None   # warm start: {name: array} of the 16 tensors
    return_env: bool = False    # hand the final environment back in Result.env


@dataclass
class Result:
    id: int
    D: int
    chi: int
    t_arrival: float
    t_admit: float
    t_done: float
    iters: int
    delta: float
    e_site: Optional[float]
    e_bond: Optional[list]
    status: str = "ok"
    env: Optional[Dict[str, Any]] = None

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


@dataclass
class _Active:
    req: Request
    handle: object
    nbytes: int
    t_admit: float
    iters: int = 0
    inflight: bool = False
    delta: float = float("inf")


class GpuBackend:
    """libctm.so solves, one torch stream per solve, workspace from torch."""

    def __init__(self):
        import torch

        import paper_2306_08212_amd as P
        from synth import site_tensors
        self.torch, self.P, self.site_tensors = torch, P, site_tensors
        self._streams: List = []

    def now(self) -> float:
        return time.perf_counter()

    def free_bytes(self) -> int:
        free, _ = self.torch.cuda.mem_get_info()
        return int(free)

    def workspace_size(self, r: Request) -> int:
        return self.P.workspace_size(self._cfg(r))

    def _cfg(self, r: Request):
        return self.P.Config(d=r.d, D=r.D, chi=r.chi, method=self.P.REDUCED,
                             precision=r.precision)

    def start(self, r: Request):
        torch = self.torch
        stream = self._streams.pop() if self._streams else torch.cuda.Stream()
        A, B = self.site_tensors(r.d, r.D, r.seed)
        with torch.cuda.stream(stream):
            s = self.P.Solver(self._cfg(r), A, B, stream=stream)
            if r.env is not None:
                s.set_env_dict(r.env)
        s._event = torch.cuda.Event()
        return s

    def enqueue_iteration(self, s):
        s.iterate_delta()
        s._event.record(s.stream)

    def ready(self, s) -> bool:
        return s._event.query()

    def read_delta(self, s) -> float:
        return s.read_delta()

    def finish(self, s):
        e, eb = s.energy()
        return e, eb

    def final_env(self, s):
        return s.get_env_dict()

    def release(self, s):
        stream = s.stream
        s.close()
        self._streams.append(stream)


class FakeBackend:
    """Virtual-clock backend for host-only tests: each iteration of request
    r takes iter_time(r) seconds of 'GPU' time, solves run concurrently, and
    delta halves every iteration from delta0."""

    def __init__(self, budget_free: int, iter_time, bytes_of, delta0: float = 1.0,
                 fail_ids=()):
        self.t = 0.0
        self.free = budget_free
        self.iter_time = iter_time
        self.bytes_of = bytes_of
        self.delta0 = delta0
        self.fail_ids = set(fail_ids)
        self.live: Dict[int, dict] = {}
        self.peak_bytes = 0
        self.in_use = 0
        self.max_concurrent = 0

    def now(self) -> float:
        return self.t

    def free_bytes(self) -> int:
        return self.free

    def workspace_size(self, r: Request) -> int:
        return self.bytes_of(r)

    def start(self, r: Request):
        h = {"req": r, "done_at": None, "k": 0}
        self.live[r.id] = h
        self.in_use += self.bytes_of(r)
        self.peak_bytes = max(self.peak_bytes, self.in_use)
        self.max_concurrent = max(self.max_concurrent, len(self.live))
        return h

    def enqueue_iteration(self, h):
        h["done_at"] = self.t + self.iter_time(h["req"])
        h["k"] += 1

    def ready(self, h) -> bool:
        return h["done_at"] is not None and self.t >= h["done_at"]

    def read_delta(self, h) -> float:
        if h["req"].id in self.fail_ids:
            raise RuntimeError("numeric failure")
        return self.delta0 * 0.5 ** h["k"]

    def finish(self, h):
        return -0.5, [-0.25] * 4

    def final_env(self, h):
        return {"iterations": h["k"], "start": h["req"].env}

    def release(self, h):
        self.in_use -= self.bytes_of(h["req"])
        del self.live[h["req"].id]

    def advance(self, dt: float):
        self.t += dt

    def next_event_time(self) -> Optional[float]:
        times = [h["done_at"] for h in self.live.values() if h["done_at"] is not None]
        return min(times) if times else None


class Server:
    """Continuous-batching scheduler.

    budget_bytes: HBM the solves may use together (0.8 x free memory at start
    if None); max_slots: solves admitted at once.
    """

    def __init__(self, backend, budget_bytes: Optional[int] = None, max_slots: int = 16,
                 on_result=None):
        self.b = backend
        self.on_result = on_result     # called with each Result as it completes
        self.budget = int(budget_bytes if budget_bytes is not None
                          else 0.8 * backend.free_bytes())
        self.max_slots = max_slots
        self.used = 0
        self.active: List[_Active] = []
        self.results: List[Result] = []
        self.rejected: List[int] = []

    def _admit(self, queue: List[Request], now: float):
        while queue and queue[0].t_arrival <= now and len(self.active) < self.max_slots:
            r = queue[0]
            need = self.b.workspace_size(r)
            if need > self.budget:
                self.rejected.append(r.id)     # can never fit
                queue.pop(0)
                continue
            if self.used + need > self.budget:
                break                          # wait for memory (FIFO)
            queue.pop(0)
            h = self.b.start(r)
            self.used += need
            self.active.append(_Active(r, h, need, self.b.now()))

    def _tick(self):
        """Enqueue work for idle solves; collect finished iterations."""
        progressed = False
        for a in list(self.active):
            if a.inflight:
                if not self.b.ready(a.handle):
                    continue
                a.inflight = False
                progressed = True
                try:
                    a.delta = self.b.read_delta(a.handle)
                except Exception:
                    self._finish(a, status="numeric")
                    continue
                a.iters += 1
                if a.delta < a.req.tol or a.iters >= a.req.max_iters:
                    self._finish(a)
                    continue
            self.b.enqueue_iteration(a.handle)
            a.inflight = True
            progressed = True
        return progressed

    def _finish(self, a: _Active, status: str = "ok"):
        e = eb = env = None
        if status == "ok":
            e, eb = self.b.finish(a.handle)
            if a.req.return_env:
                env = self.b.final_env(a.handle)
        self.results.append(Result(a.req.id, a.req.D, a.req.chi, a.req.t_arrival, a.t_admit,
                                   self.b.now(), a.iters, a.delta, e, eb, status, env))
        if self.on_result is not None:
            self.on_result(self.results[-1])
        self.b.release(a.handle)
        self.used -= a.nbytes
        self.active.remove(a)

    def run(self, requests: List[Request], t0: Optional[float] = None) -> List[Result]:
        """Serve a stream; arrival times are relative to t0 (now if None)."""
        queue = sorted(requests, key=lambda r: (r.t_arrival, r.id))
        start = self.b.now() if t0 is None else t0
        shifted = [Request(**{**r.__dict__, "t_arrival": start + r.t_arrival}) for r in queue]
        queue = shifted
        fake = hasattr(self.b, "advance")
        while queue or self.active:
            self._admit(queue, self.b.now())
            progressed = self._tick()
            if fake and not progressed:
                # jump the virtual clock to the next completion or arrival
                now = self.b.now()
                cand = [t for t in (self.b.next_event_time(),
                                    queue[0].t_arrival if queue else None)
                        if t is not None and t > now]
                if cand:
                    self.b.advance(min(cand) - now)
                elif queue and not self.active:
                    raise RuntimeError("scheduler stalled")
            elif not progressed:
                time.sleep(0.0005)
        return sorted(self.results, key=lambda r: r.id)


def summarize(results: List[Result], t_first_arrival: float = None) -> dict:
    ok = [r for r in results if r.status == "ok"]
    lat = sorted(r.latency for r in ok)

    def pct(p):
        if not lat:
            return None
        i = min(len(lat) - 1, max(0, int(round(p / 100.0 * (len(lat) - 1)))))
        return lat[i]

    if ok:
        t0 = min(r.t_arrival for r in ok) if t_first_arrival is None else t_first_arrival
        span = max(r.t_done for r in ok) - t0
    else:
        span = 0.0
    return {"solves": len(ok), "failed": len(results) - len(ok),
            "p50_s": pct(50), "p99_s": pct(99),
            "solves_per_s": (len(ok) / span) if span > 0 else None}
