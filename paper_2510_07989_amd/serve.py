"""Continuous batching of MOT solves on one GPU.

Requests are scattering solves. Each names a mesh with its boundary data, the
media, dt, a set of plane waves and a number of steps, and each arrives at its
own time.

Admission: a request is admitted, in arrival order, when a slot is free and its
peak device footprint (``mot_footprint``) fits in the memory budget next to the
peak footprints of the solves already running.

Execution: every admitted solve keeps its lag matrices and history resident,
and runs on its own HIP stream driven by its own host thread. The C library
releases the interpreter lock and takes device memory from the stream-ordered
pool, so the solves' kernels overlap on the device. A solve marches in windows
of steps. Requests that arrive meanwhile are admitted as slots and memory free
up.

Per request the server records:
* queue wait and setup time;
* the latency of every step (each window's wall time over its steps);
* end-to-end latency, from arrival to outputs on the host.

Overall it records p50/p99 step and end-to-end latency and aggregate steps/s.

The backend is pluggable: ``GpuBackend`` drives ``paper_2510_07989_amd.Solver``;
tests substitute a host-only backend to check the scheduling on its own.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field
from typing import Any, Callable, Dict, List, Optional

import numpy as np

__all__ = ["Request", "Result", "Server", "GpuBackend", "latency_stats"]


@dataclass
class Request:
    """One scattering solve: ``problem`` carries the mot_create inputs and the
    raw lag blocks (keys V, F, E, eps_r, mu_r, dt, T0s, T0h, G, waves, raw,
    kmax); ``arrival`` is seconds after the server starts."""
    rid: int
    problem: Dict[str, Any]
    nsteps: int
    arrival: float = 0.0
    options: Optional[Dict[str, Any]] = None


@dataclass
class Result:
    rid: int
    nsteps: int
    footprint: int
    t_arrival: float
    t_admit: float = 0.0
    t_ready: float = 0.0
    t_done: float = 0.0
    step_latency: List[float] = field(default_factory=list)
    outputs: Dict[str, np.ndarray] = field(default_factory=dict)
    error: Optional[str] = None

    @property
    def end_to_end(self) -> float:
        return self.t_done - self.t_arrival

    @property
    def queue_wait(self) -> float:
        return self.t_admit - self.t_arrival


def latency_stats(values) -> Dict[str, float]:
    v = np.asarray(list(values), dtype=np.float64)
    if v.size == 0:
        return {"n": 0, "p50": float("nan"), "p99": float("nan"), "mean": float("nan"), "max": float("nan")}
    return {"n": int(v.size), "p50": float(np.percentile(v, 50)), "p99": float(np.percentile(v, 99)),
            "mean": float(v.mean()), "max": float(v.max())}


class GpuBackend:
    """Runs a request on the current GPU through the C ABI, on a stream of its own."""

    def __init__(self, options: Optional[Dict[str, Any]] = None, keep_outputs: bool = True):
        self.options = dict(options or {})
        self.keep_outputs = keep_outputs

    def _opts(self, req: Request):
        import paper_2510_07989_amd as mot
        o = dict(self.options)
        o.update(req.options or {})
        o.setdefault("max_steps", req.nsteps + 8)
        return mot.default_options(**o)

    def footprint(self, req: Request) -> int:
        import paper_2510_07989_amd as mot
        p = req.problem
        _, peak = mot.footprint(p["V"], p["F"], p["E"], p["eps_r"], p["mu_r"], p["dt"], len(p["waves"]), p["G"],
                                self._opts(req))
        return peak

    def execute(self, req: Request, window: int, clock: Callable[[], float], res: Result) -> None:
        import torch
        import paper_2510_07989_amd as mot
        torch.cuda.set_device(0)
        stream = torch.cuda.Stream()          # default priority
        with torch.cuda.stream(stream):       # output tensors belong to this stream
            self._march(mot, torch, stream, req, window, clock, res)

    def _march(self, mot, torch, stream, req, window, clock, res):
        p = req.problem
        s = mot.Solver(p["V"], p["F"], p["E"], p["eps_r"], p["mu_r"], p["dt"], p["T0s"], p["T0h"], p["G"],
                       p["waves"], options=self._opts(req), stream=stream.cuda_stream)
        try:
            s.load_raw(p["raw"], p["kmax"])
            stream.synchronize()
            res.t_ready = clock()
            parts = {"w": [], "loop": [], "star": []}
            done = 0
            while done < req.nsteps:
                nw = min(window, req.nsteps - done)
                t0 = clock()
                out = s.run(nw, w=self.keep_outputs, loop=self.keep_outputs, star=self.keep_outputs, device=True)
                stream.synchronize()
                dt = clock() - t0
                res.step_latency.extend([dt / nw] * nw)
                if self.keep_outputs:
                    for k in parts:
                        parts[k].append(out[k])
                done += nw
            if self.keep_outputs:
                for k, v in parts.items():
                    res.outputs[k] = torch.cat(v).cpu().numpy()
        finally:
            s.close()


class Server:
    """Admission by memory footprint and concurrent execution (see module doc)."""

    def __init__(self, backend, mem_budget: int, max_active: int = 8, window: int = 64, poll: float = 0.001,
                 request_timeout: float = 600.0, log: Optional[Callable[[str], None]] = None):
        self.backend = backend
        self.mem_budget = int(mem_budget)
        self.max_active = int(max_active)
        self.window = int(window)
        self.poll = poll
        self.request_timeout = float(request_timeout)
        self.log = log
        self.trace: List[tuple] = []          # (time, event, rid, active, used bytes)

    def run(self, requests: List[Request]):
        """Serve every request; returns (results by rid, summary dict)."""
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        fp = {r.rid: int(self.backend.footprint(r)) for r in reqs}
        for r in reqs:
            if fp[r.rid] > self.mem_budget:
                raise ValueError("request %d needs %d bytes, more than the budget %d" % (r.rid, fp[r.rid],
                                                                                          self.mem_budget))
        t_start = time.perf_counter()

        def clock():
            return time.perf_counter() - t_start

        results = {r.rid: Result(r.rid, r.nsteps, fp[r.rid], r.arrival) for r in reqs}
        pending = list(reqs)
        queue: List[Request] = []
        active: Dict[int, threading.Thread] = {}
        used = 0
        lock = threading.Lock()
        finished: List[int] = []

        def worker(req: Request):
            res = results[req.rid]
            try:
                self.backend.execute(req, self.window, clock, res)
            except Exception as e:          # reported per request
                res.error = "%s: %s" % (type(e).__name__, e)
            res.t_done = clock()
            with lock:
                finished.append(req.rid)

        while pending or queue or active:
            now = clock()
            while pending and pending[0].arrival <= now:
                queue.append(pending.pop(0))
            with lock:
                done_now, finished[:] = list(finished), []
            for rid in done_now:
                active.pop(rid).join()
                used -= fp[rid]
                self.trace.append((clock(), "done", rid, len(active), used))
                if self.log:
                    r = results[rid]
                    self.log("[serve %.2fs] request %d done (%d steps, %.3f s end to end%s); %d active"
                             % (clock(), rid, r.nsteps, r.end_to_end, ", " + r.error if r.error else "", len(active)))
            # a request past its time limit is reported and its slot and memory
            # stay held (its thread cannot be stopped from here)
            for rid in list(active):
                r = results[rid]
                if r.error is None and clock() - r.t_admit > self.request_timeout:
                    r.error = "TimeoutError: still running after %.0f s" % self.request_timeout
                    if self.log:
                        self.log("[serve %.2fs] request %d exceeded %.0f s" % (clock(), rid, self.request_timeout))
            if active and all(results[rid].error for rid in active) and not queue and not pending:
                break
            # strict arrival order: the head waits until it fits
            while queue and len(active) < self.max_active and used + fp[queue[0].rid] <= self.mem_budget:
                req = queue.pop(0)
                used += fp[req.rid]
                results[req.rid].t_admit = clock()
                th = threading.Thread(target=worker, args=(req,), daemon=True)
                active[req.rid] = th
                self.trace.append((clock(), "admit", req.rid, len(active), used))
                if self.log:
                    self.log("[serve %.2fs] request %d admitted (%d steps, %d waves, %.1f MB); %d active"
                             % (clock(), req.rid, req.nsteps, len(req.problem["waves"]), fp[req.rid] / 1e6,
                                len(active)))
                th.start()
            if not (pending or queue or active):
                break
            wait = self.poll
            if pending and not queue:
                wait = min(max(pending[0].arrival - clock(), 0.0), 0.05) or self.poll
            time.sleep(wait)
        wall = clock()
        nrhs = {q.rid: len(q.problem["waves"]) for q in reqs}
        steps = sum(r.nsteps for r in results.values() if r.error is None)
        rhs_steps = sum(r.nsteps * nrhs[r.rid] for r in results.values() if r.error is None)
        summary = {
            "requests": len(reqs),
            "errors": sum(1 for r in results.values() if r.error),
            "wall_s": wall,
            "steps": steps,
            "steps_per_s": steps / wall if wall > 0 else float("nan"),
            "rhs_steps_per_s": rhs_steps / wall if wall > 0 else float("nan"),
            "step_latency_s": latency_stats(x for r in results.values() for x in r.step_latency),
            "end_to_end_s": latency_stats(r.end_to_end for r in results.values() if r.error is None),
            "queue_wait_s": latency_stats(r.queue_wait for r in results.values()),
            "max_concurrent": max((t[3] for t in self.trace), default=0),
            "peak_budget_used": max((t[4] for t in self.trace), default=0),
        }
        return results, summary
