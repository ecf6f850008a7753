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

Two servers share the admission rule:

* ``Server`` runs every admitted solve on its own HIP stream and host thread
  (windows of ``mot_run``);
* ``BatchServer`` keeps one marching thread that steps all active solves
  together through ``mot_run_batch`` (their windows interleaved across their
  streams, as one host thread can queue them), while a small pool of setup
  threads creates and loads newly admitted solves; a solve joins the batch at
  the next window after its setup and leaves it when done.

A request past its time limit, or still running when the server's time box
closes, is stopped with ``mot_cancel`` at its next window boundary; its slot
and memory are then released.

The backend is pluggable: ``GpuBackend`` drives ``paper_2510_07989_amd.Solver``;
tests substitute a host-only backend to check the scheduling on its own.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field
from typing import Any, Callable, Dict, List, Optional

import numpy as np

__all__ = ["Request", "Result", "Server", "BatchServer", "GpuBackend", "latency_stats", "CancelledRun",
           "stop_if_cancelled"]


@dataclass
class Request:
    """One scattering solve: ``problem`` carries the mot_create inputs and the
    raw lag blocks (keys V, F, E, eps_r, mu_r, dt, T0s, T0h, G, waves, and
    raw with kmax, or instead a callable ``loader(solver)`` that uploads the
    blocks itself); ``arrival`` is seconds after the server starts."""
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
    cancel_requested: bool = False      # set by the server (time limit, time box); the backend stops there

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


class CancelledRun(RuntimeError):
    """A solve stopped by mot_cancel (time limit or time box)."""


def stop_if_cancelled(s):
    """For loaders (Request.problem['loader']): raise CancelledRun between
    uploads once the server has cancelled solver s, so that a request whose
    time ran out during its setup does not finish assembling its inputs."""
    if getattr(s, "_serve_cancelled", False):
        raise CancelledRun("cancelled during setup")


class GpuBackend:
    """Runs a request on the current GPU through the C ABI, on a stream of its own."""

    # execute() stops a request whose Result.cancel_requested is set, also
    # before its solver exists (waiting for a setup slot, building inputs)
    honors_cancel_requested = True

    def __init__(self, options: Optional[Dict[str, Any]] = None, keep_outputs: bool = True,
                 setup_slots: Optional[int] = None):
        """setup_slots: at most this many requests build their inputs and
        solvers at once (execute; None: no limit); the others wait, admitted."""
        self.options = dict(options or {})
        self.keep_outputs = keep_outputs
        self._setup_gate = threading.Semaphore(setup_slots) if setup_slots else None
        self._live: Dict[int, Any] = {}
        self._live_lock = threading.Lock()

    def cancel(self, rid: int) -> bool:
        """Stop request rid's march at its next window boundary (mot_cancel).
        False if it has no solver here (a request of the per-thread server
        that is still setting up stops by its result's cancel_requested)."""
        with self._live_lock:
            s = self._live.get(rid)
        if s is None:
            return False
        self._stop(s)
        return True

    @staticmethod
    def _stop(s):
        # the flag lets a loader that is still uploading stop between lags
        # (stop_if_cancelled); mot_cancel stops the march
        s._serve_cancelled = True
        s.cancel()

    def _register(self, rid, s, res=None):
        with self._live_lock:
            self._live[rid] = s
        if res is not None and res.cancel_requested:      # asked before the solver existed
            self._stop(s)

    def _unregister(self, rid):
        with self._live_lock:
            self._live.pop(rid, None)

    def _load(self, s, p):
        if p.get("loader") is not None:
            p["loader"](s)
        else:
            s.load_raw(p["raw"], p["kmax"])

    def setup(self, req: Request):
        """Create and load request req's solver on a stream of its own (batch server)."""
        import torch
        import paper_2510_07989_amd as mot
        torch.cuda.set_device(0)
        stream = torch.cuda.Stream()          # default priority
        with torch.cuda.stream(stream):
            p = self._inputs(req.problem)
            s = mot.Solver(p["V"], p["F"], p["E"], p["eps_r"], p["mu_r"], p["dt"], p["T0s"], p["T0h"],
                           p["G"], p["waves"], options=self._opts(req), stream=stream.cuda_stream)
            try:
                self._load(s, p)
                stream.synchronize()
            except Exception:
                s.close()
                raise
        s._serve_stream = stream
        self._register(req.rid, s)
        return s

    def outputs(self, req: Request, s, nsteps: int) -> Dict[str, np.ndarray]:
        if not self.keep_outputs or nsteps == 0:
            return {}
        out = s.steps(0, nsteps)
        return {k: out[k] for k in ("w", "loop", "star")}

    def close(self, req: Request, s) -> None:
        self._unregister(req.rid)
        s.close()

    def run_batch(self, solvers, nsteps):
        """March the solvers together (mot_run_batch); per solver 0 (done or
        iteration cap), "cancelled", or an error message."""
        import paper_2510_07989_amd as mot
        from paper_2510_07989_amd import _lib as L
        lib = L.load()
        import ctypes
        n = len(solvers)
        hs = (ctypes.c_void_p * n)(*[s._h.value for s in solvers])
        st = (ctypes.c_int32 * n)()
        lib.mot_run_batch(hs, n, int(nsteps), st)
        out = []
        for i, s in enumerate(solvers):
            c = st[i]
            if c in (L.MOT_OK, L.MOT_ENOCONV):
                out.append(0)
            elif c == L.MOT_ECANCEL:
                out.append("cancelled")
            else:
                out.append("MotError(%d): %s" % (c, lib.mot_last_error(s._h).decode()))
        return out

    def _opts(self, req: Request):
        import paper_2510_07989_amd as mot
        o = dict(self.options)
        o.update(req.options or {})
        o.setdefault("max_steps", req.nsteps + 8)
        return mot.default_options(**o)

    def footprint(self, req: Request) -> int:
        """Peak device bytes of the solve (mot_footprint), plus the request's
        own extra_bytes (device memory its loader needs while it runs)."""
        import paper_2510_07989_amd as mot
        p = req.problem
        _, peak = mot.footprint(p["V"], p["F"], p["E"], p["eps_r"], p["mu_r"], p["dt"], len(p["waves"]), p.get("G"),
                                self._opts(req), gnnz=p.get("gnnz"))
        return peak + int(p.get("extra_bytes", 0))

    @staticmethod
    def _inputs(p):
        """A request whose inputs are built at setup carries prepare() -> the
        missing keys (G, T0s, T0h, and raw with kmax or a loader)."""
        if p.get("prepare") is not None:
            p = dict(p)
            p.update(p.pop("prepare")())
        return p

    def execute(self, req: Request, window: int, clock: Callable[[], float], res: Result) -> None:
        import torch
        import paper_2510_07989_amd as mot
        torch.cuda.set_device(0)
        stream = torch.cuda.Stream()          # default priority
        with torch.cuda.stream(stream):       # output tensors belong to this stream
            self._march(mot, torch, stream, req, window, clock, res)

    def _march(self, mot, torch, stream, req, window, clock, res):
        gate = self._setup_gate
        if gate is not None:
            gate.acquire()
        s = None
        try:
            if res.cancel_requested:                  # stopped while it waited for a setup slot
                raise CancelledRun("cancelled before its setup")
            p = self._inputs(req.problem)
            s = mot.Solver(p["V"], p["F"], p["E"], p["eps_r"], p["mu_r"], p["dt"], p["T0s"], p["T0h"], p["G"],
                           p["waves"], options=self._opts(req), stream=stream.cuda_stream)
            self._register(req.rid, s, res)
            self._load(s, p)
            stream.synchronize()
        except BaseException:
            if s is not None:
                self._unregister(req.rid)
                s.close()
            raise
        finally:
            if gate is not None:
                gate.release()
        try:
            res.t_ready = clock()
            parts = {"w": [], "loop": [], "star": []}
            done = 0
            while done < req.nsteps:
                nw = min(window, req.nsteps - done)
                t0 = clock()
                out = s.run(nw, w=self.keep_outputs, loop=self.keep_outputs, star=self.keep_outputs, device=True)
                stream.synchronize()
                dt = clock() - t0
                got = nw if not out["cancelled"] else s.info()["steps_done"] - done
                if got:
                    res.step_latency.extend([dt / got] * got)
                if self.keep_outputs:
                    for k in parts:
                        parts[k].append(out[k])
                done += got
                if out["cancelled"]:
                    raise CancelledRun("stopped by mot_cancel after %d of %d steps" % (done, req.nsteps))
            if self.keep_outputs:
                for k, v in parts.items():
                    res.outputs[k] = torch.cat(v).cpu().numpy()
        finally:
            self._unregister(req.rid)
            s.close()


class Server:
    """Admission by memory footprint and concurrent execution (see module doc)."""

    def __init__(self, backend, mem_budget: int, max_active: int = 8, window: int = 64, poll: float = 0.001,
                 request_timeout: float = 600.0, time_box: Optional[float] = None,
                 log: Optional[Callable[[str], None]] = None, cancel_grace: float = 60.0):
        """time_box: seconds after start when every request still running is
        cancelled (at its next window boundary; it is then reported as
        cancelled with the steps it completed) and requests not yet admitted
        are not served.  cancel_grace: seconds a cancelled request's thread
        may take to end; past it the request is reported as stalled and no
        longer waited on (its memory stays counted, and requests that only
        stalled ones keep out of the budget are not served), so the server
        ends instead of waiting silently on a thread that never returns."""
        self.backend = backend
        self.mem_budget = int(mem_budget)
        self.max_active = int(max_active)
        self.window = int(window)
        self.poll = poll
        self.time_box = time_box
        self.request_timeout = float(request_timeout)
        self.log = log
        self.cancel_grace = float(cancel_grace)
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
        cancelled: Dict[int, float] = {}       # rid -> time of its cancel
        stalled = set()

        def worker(req: Request):
            res = results[req.rid]
            err = None
            try:
                self.backend.execute(req, self.window, clock, res)
            except Exception as e:          # reported per request
                err = "%s: %s" % (type(e).__name__, e)
            with lock:
                if req.rid not in stalled:  # a stalled request keeps its report
                    if err is not None:
                        res.error = err
                    res.t_done = clock()
                finished.append(req.rid)

        boxed = False
        while pending or queue or active:
            now = clock()
            while pending and pending[0].arrival <= now:
                queue.append(pending.pop(0))
            if self.time_box is not None and now >= self.time_box and not boxed:
                # the box closes: nothing more is admitted, running requests stop at their next window
                boxed = True
                for req in pending + queue:
                    results[req.rid].error = "NotServed: the time box closed before admission"
                pending, queue = [], []
                for rid in list(active):
                    if rid not in cancelled:
                        cancelled[rid] = now
                        results[rid].cancel_requested = True
                        getattr(self.backend, "cancel", lambda _rid: False)(rid)
                if self.log:
                    self.log("[serve %.2fs] time box closed; %d running cancelled" % (now, len(active)))
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
            # a request past its time limit is stopped at its next window
            # boundary (mot_cancel); its thread then ends and frees the slot
            for rid in list(active):
                r = results[rid]
                if r.error is None and rid not in cancelled and clock() - r.t_admit > self.request_timeout:
                    cancelled[rid] = clock()
                    r.cancel_requested = True
                    stopped = (getattr(self.backend, "cancel", lambda _rid: False)(rid)
                               or getattr(self.backend, "honors_cancel_requested", False))
                    if self.log:
                        self.log("[serve %.2fs] request %d exceeded %.0f s%s" % (clock(), rid, self.request_timeout,
                                                                              ", cancelled" if stopped else ""))
                    if not stopped:
                        r.error = "TimeoutError: still running after %.0f s" % self.request_timeout
            # a cancelled request whose thread does not end is reported, not waited on
            for rid in list(active):
                r = results[rid]
                with lock:
                    late = (rid in cancelled and rid not in stalled and rid not in finished
                            and clock() - cancelled[rid] > self.cancel_grace)
                    if late:
                        stalled.add(rid)
                        r.error = "Stalled: still running %.1f s after its cancel" % (clock() - cancelled[rid])
                        r.t_done = clock()
                if late:
                    self.trace.append((clock(), "stalled", rid, len(active), used))
                    if self.log:
                        self.log("[serve %.2fs] request %d: %s" % (clock(), rid, r.error))
            if stalled and queue and all(rid in stalled for rid in active) and \
                    used + fp[queue[0].rid] > self.mem_budget:
                # only stalled requests hold the budget the head needs
                for req in queue:
                    results[req.rid].error = "NotServed: the budget is held by a stalled request"
                if self.log:
                    self.log("[serve %.2fs] %d queued requests not served: the budget is held by %d stalled"
                             % (clock(), len(queue), len(stalled)))
                queue = []
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
        ok = [r for r in results.values() if r.error is None]
        steps = sum(r.nsteps for r in ok)
        marched = sum(len(r.step_latency) for r in results.values())
        rhs_marched = sum(len(r.step_latency) * nrhs[r.rid] for r in results.values())
        stopped = ("CancelledRun", "NotServed")
        summary = {
            "requests": len(reqs),
            "completed": len(ok),
            "cancelled": sum(1 for r in results.values() if r.error and r.error.startswith("CancelledRun")),
            "not_served": sum(1 for r in results.values() if r.error and r.error.startswith("NotServed")),
            "errors": sum(1 for r in results.values() if r.error and not r.error.startswith(stopped)),
            "stalled": len(stalled),
            "wall_s": wall,
            "steps": steps,
            "steps_marched": marched,
            "steps_per_s": marched / wall if wall > 0 else float("nan"),
            "rhs_steps_per_s": rhs_marched / wall if wall > 0 else float("nan"),
            "step_latency_s": latency_stats(x for r in results.values() for x in r.step_latency),
            "end_to_end_s": latency_stats(r.end_to_end for r in ok),
            "queue_wait_s": latency_stats(r.queue_wait for r in results.values() if r.t_admit > 0),
            "max_concurrent": max((t[3] for t in self.trace), default=0),
            "peak_budget_used": max((t[4] for t in self.trace), default=0),
        }
        return results, summary


class BatchServer:
    """Continuous batching from one marching thread (see module doc).

    The backend provides footprint(req), setup(req) -> solver (created and
    loaded, on its own stream), outputs(req, solver, nsteps), close(req,
    solver), and a run_batch(solvers, nsteps) -> codes that marches them
    together and returns each one's code (0, or "cancelled" for one stopped by
    its cancel()).  window: steps per batch call; a solve joins or leaves the
    batch between calls.  time_box: seconds after start when every solve still
    running is cancelled and requests not yet admitted are dropped (reported
    as not served).  setup_timeout: seconds a setup may run (default: the
    request time limit); a setup past it is reported as stalled and the
    server stops waiting for it.  Its memory stays counted until it returns
    (its solver is then closed); requests that only a stalled setup keeps out
    of the budget are not served, so the server ends instead of waiting
    silently on a setup that never returns."""

    def __init__(self, backend, mem_budget: int, max_active: int = 8, window: int = 128, setup_workers: int = 2,
                 poll: float = 0.002, request_timeout: float = 600.0, time_box: Optional[float] = None,
                 log: Optional[Callable[[str], None]] = None, setup_timeout: Optional[float] = None):
        self.backend = backend
        self.mem_budget = int(mem_budget)
        self.max_active = int(max_active)
        self.window = int(window)
        self.setup_workers = int(setup_workers)
        self.poll = poll
        self.request_timeout = float(request_timeout)
        self.time_box = time_box
        self.log = log
        self.setup_timeout = float(request_timeout if setup_timeout is None else setup_timeout)
        self.trace: List[tuple] = []          # (time, event, rid, active, used bytes)

    def _close_late(self, req, f):
        try:
            self.backend.close(req, f.result())
        except Exception:
            pass

    def run(self, requests: List[Request]):
        """Serve every request; returns (results by rid, summary dict)."""
        from concurrent.futures import ThreadPoolExecutor
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        fp = {r.rid: int(self.backend.footprint(r)) for r in reqs}
        for r in reqs:
            if fp[r.rid] > self.mem_budget:
                raise ValueError("request %d needs %d bytes, more than the budget %d" % (r.rid, fp[r.rid],
                                                                                          self.mem_budget))
        t_start = time.perf_counter()

        def clock():
            return time.perf_counter() - t_start

        def say(msg):
            if self.log:
                self.log("[batch %.2fs] %s" % (clock(), msg))

        results = {r.rid: Result(r.rid, r.nsteps, fp[r.rid], r.arrival) for r in reqs}
        byid = {r.rid: r for r in reqs}
        pending = list(reqs)
        queue: List[Request] = []
        setting_up: Dict[int, Any] = {}        # rid -> future
        running: Dict[int, Any] = {}           # rid -> solver
        stalled: Dict[int, Any] = {}           # rid -> future of a setup past its limit
        nstalled = 0
        done_steps: Dict[int, int] = {}
        used = 0
        closed = threading.Event()             # the time box has closed
        deadline_hit = set()
        lock = threading.Lock()

        def watchdog():
            # cancels solves past their time limit and, at the time box, every
            # solve still running: their batch call returns at the next window
            # (under the lock: the marching thread removes a solve from
            # `running` under it before closing the solve)
            while not stop_watch.is_set():
                now = clock()
                box = self.time_box is not None and now >= self.time_box
                if box and not closed.is_set():
                    closed.set()
                with lock:
                    for rid, s in running.items():
                        if rid in deadline_hit:
                            continue
                        if box or now - results[rid].t_admit > self.request_timeout:
                            deadline_hit.add(rid)
                            s.cancel()
                stop_watch.wait(0.01)

        stop_watch = threading.Event()
        wd = threading.Thread(target=watchdog, daemon=True)
        wd.start()
        pool = ThreadPoolExecutor(max_workers=max(1, self.setup_workers))

        def finish(rid, s, error=None):
            nonlocal used
            r = results[rid]
            req = byid[rid]
            if error is None and s is not None:
                try:
                    r.outputs = self.backend.outputs(req, s, done_steps.get(rid, 0))
                except Exception as e:
                    error = "%s: %s" % (type(e).__name__, e)
            if s is not None:
                try:
                    self.backend.close(req, s)
                except Exception as e:
                    error = error or "%s: %s" % (type(e).__name__, e)
            r.error = error
            r.t_done = clock()
            used -= fp[rid]
            self.trace.append((clock(), "done", rid, len(running) + len(setting_up), used))
            say("request %d done (%d of %d steps, %.3f s end to end%s)" % (
                rid, done_steps.get(rid, 0), req.nsteps, r.end_to_end, ", " + error if error else ""))

        try:
            while pending or queue or setting_up or running:
                now = clock()
                while pending and pending[0].arrival <= now:
                    queue.append(pending.pop(0))
                if closed.is_set():
                    # the time box has closed: nothing more is admitted
                    for req in pending + queue:
                        results[req.rid].error = "NotServed: the time box closed before admission"
                    pending, queue = [], []
                # strict arrival order: the head waits until it fits
                while (queue and len(running) + len(setting_up) < self.max_active
                       and used + fp[queue[0].rid] <= self.mem_budget):
                    req = queue.pop(0)
                    used += fp[req.rid]
                    results[req.rid].t_admit = clock()
                    setting_up[req.rid] = pool.submit(self.backend.setup, req)
                    self.trace.append((clock(), "admit", req.rid, len(running) + len(setting_up), used))
                    say("request %d admitted (%d steps, %d waves, %.1f MB)" % (
                        req.rid, req.nsteps, len(req.problem["waves"]), fp[req.rid] / 1e6))
                for rid in [q for q, f in stalled.items() if f.done()]:
                    # a stalled setup that came back: close its solver, free its bytes
                    f = stalled.pop(rid)
                    try:
                        self.backend.close(byid[rid], f.result())
                    except Exception:
                        pass
                    used -= fp[rid]
                    say("stalled setup of request %d returned after %.1f s; closed" % (
                        rid, clock() - results[rid].t_admit))
                for rid in [q for q, f in setting_up.items()
                            if not f.done() and clock() - results[q].t_admit > self.setup_timeout]:
                    stalled[rid] = setting_up.pop(rid)
                    nstalled += 1
                    r = results[rid]
                    r.error = "SetupStalled: setup still running after %.1f s" % (clock() - r.t_admit)
                    r.t_done = clock()
                    self.trace.append((clock(), "stalled", rid, len(running) + len(setting_up), used))
                    say("request %d: %s" % (rid, r.error))
                if stalled and queue and not running and not setting_up and \
                        used + fp[queue[0].rid] > self.mem_budget:
                    # only stalled setups hold the budget the head needs
                    for req in queue:
                        results[req.rid].error = "NotServed: the budget is held by a stalled setup"
                    say("%d queued requests not served: the budget is held by %d stalled setups" % (
                        len(queue), len(stalled)))
                    queue = []
                for rid in [q for q, f in setting_up.items() if f.done()]:
                    f = setting_up.pop(rid)
                    try:
                        s = f.result()
                    except Exception as e:
                        finish(rid, None, "%s: %s" % (type(e).__name__, e))
                        continue
                    results[rid].t_ready = clock()
                    if closed.is_set():
                        finish(rid, s, "CancelledRun: the time box closed during setup")
                        continue
                    with lock:
                        running[rid] = s
                    done_steps[rid] = 0
                if running:
                    rids = list(running)
                    n = min([self.window] + [byid[q].nsteps - done_steps[q] for q in rids])
                    t0 = clock()
                    codes = self.backend.run_batch([running[q] for q in rids], n)
                    el = clock() - t0
                    for q, code in zip(rids, codes):
                        s = running[q]
                        if code == "cancelled":
                            got = s.info()["steps_done"] - done_steps[q]
                        elif isinstance(code, str):
                            got = 0
                        else:
                            got = n
                        if got:
                            results[q].step_latency.extend([el / n] * got)
                        done_steps[q] += got
                        err = None
                        if code == "cancelled":
                            err = "CancelledRun: stopped by mot_cancel after %d of %d steps" % (done_steps[q],
                                                                                               byid[q].nsteps)
                        elif isinstance(code, str):
                            err = code
                        if err or done_steps[q] >= byid[q].nsteps:
                            with lock:
                                running.pop(q)
                            finish(q, s, err)
                    continue
                wait = self.poll
                if pending and not queue and not setting_up:
                    wait = min(max(pending[0].arrival - clock(), 0.0), 0.05) or self.poll
                time.sleep(wait)
        finally:
            stop_watch.set()
            wd.join()
            # a setup that never returns must not hold the caller here; one
            # that returns later closes its own solver
            for rid, f in stalled.items():
                f.add_done_callback(lambda f, req=byid[rid]: self._close_late(req, f))
            pool.shutdown(wait=not stalled)
        wall = clock()
        nrhs = {q.rid: len(q.problem["waves"]) for q in reqs}
        ok = [r for r in results.values() if r.error is None]
        steps = sum(r.nsteps for r in ok)
        rhs_steps = sum(r.nsteps * nrhs[r.rid] for r in ok)
        summary = {
            "requests": len(reqs),
            "completed": len(ok),
            "cancelled": sum(1 for r in results.values() if r.error and r.error.startswith("CancelledRun")),
            "not_served": sum(1 for r in results.values() if r.error and r.error.startswith("NotServed")),
            "errors": sum(1 for r in results.values() if r.error and not r.error.startswith(("CancelledRun",
                                                                                             "NotServed"))),
            "stalled_setups": nstalled,
            "wall_s": wall,
            "steps": steps,
            "steps_marched": sum(len(r.step_latency) for r in results.values()),
            "steps_per_s": sum(len(r.step_latency) for r in results.values()) / wall if wall > 0 else float("nan"),
            "rhs_steps_per_s": (sum(len(r.step_latency) * nrhs[r.rid] for r in results.values()) / wall
                                if wall > 0 else float("nan")),
            "step_latency_s": latency_stats(x for r in results.values() for x in r.step_latency),
            "end_to_end_s": latency_stats(r.end_to_end for r in ok),
            "queue_wait_s": latency_stats(r.queue_wait for r in results.values() if r.t_admit > 0),
            "max_concurrent": max((t[3] for t in self.trace), default=0),
            "peak_budget_used": max((t[4] for t in self.trace), default=0),
        }
        return results, summary
