"""Scheduling of the serving loop, on the host (a backend that only sleeps)."""
import threading
import time

import pytest

from paper_2510_07989_amd.serve import Request, Server, latency_stats


class SleepBackend:
    """Footprint from the request; 'execution' sleeps per step and records
    how many requests were executing at once and the budget in use."""

    def __init__(self, step_s=0.002):
        self.step_s = step_s
        self.lock = threading.Lock()
        self.running = {}
        self.max_running = 0
        self.max_bytes = 0

    def footprint(self, req):
        return req.problem["bytes"]

    def execute(self, req, window, clock, res):
        with self.lock:
            self.running[req.rid] = req.problem["bytes"]
            self.max_running = max(self.max_running, len(self.running))
            self.max_bytes = max(self.max_bytes, sum(self.running.values()))
        res.t_ready = clock()
        done = 0
        while done < req.nsteps:
            nw = min(window, req.nsteps - done)
            t0 = clock()
            time.sleep(self.step_s * nw)
            res.step_latency.extend([(clock() - t0) / nw] * nw)
            done += nw
        with self.lock:
            del self.running[req.rid]


def _req(rid, nbytes, nsteps, arrival):
    return Request(rid, {"bytes": nbytes, "waves": [None]}, nsteps, arrival)


def test_budget_is_never_exceeded_and_all_finish():
    be = SleepBackend()
    reqs = [_req(i, 300 + 100 * (i % 3), 20 + 5 * i, 0.003 * i) for i in range(12)]
    srv = Server(be, mem_budget=1000, max_active=8, window=8)
    res, summ = srv.run(reqs)
    assert summ["errors"] == 0 and all(r.t_done > 0 for r in res.values())
    assert be.max_bytes <= 1000
    assert summ["peak_budget_used"] <= 1000
    assert be.max_running >= 2                     # requests overlapped
    for r in res.values():
        assert r.t_admit >= r.t_arrival and r.t_done >= r.t_admit
        assert len(r.step_latency) == r.nsteps


def test_late_arrival_admitted_while_others_run():
    """Continuous batching: a request arriving during a long solve starts
    before that solve ends when it fits."""
    be = SleepBackend(step_s=0.004)
    long = _req(0, 400, 100, 0.0)              # ~0.4 s
    late = _req(1, 400, 10, 0.05)
    res, _ = Server(be, mem_budget=1000, window=10).run([long, late])
    assert res[1].t_admit < res[0].t_done
    assert res[1].t_done < res[0].t_done


def test_admission_waits_for_memory_in_arrival_order():
    be = SleepBackend(step_s=0.003)
    a = _req(0, 700, 30, 0.0)
    b = _req(1, 600, 10, 0.01)                 # does not fit beside a
    c = _req(2, 100, 10, 0.02)                 # would fit, but queues behind b
    res, _ = Server(be, mem_budget=1000, window=5).run([a, b, c])
    assert res[1].t_admit >= res[0].t_done - 1e-3
    assert res[2].t_admit >= res[1].t_admit


def test_slot_limit():
    be = SleepBackend()
    reqs = [_req(i, 10, 10, 0.0) for i in range(6)]
    Server(be, mem_budget=10 ** 6, max_active=2, window=5).run(reqs)
    assert be.max_running <= 2


def test_request_larger_than_budget_is_refused():
    with pytest.raises(ValueError):
        Server(SleepBackend(), mem_budget=100).run([_req(0, 200, 5, 0.0)])


def test_latency_stats():
    s = latency_stats(range(1, 101))
    assert s["n"] == 100 and abs(s["p50"] - 50.5) < 1e-12 and 99 < s["p99"] <= 100


def test_request_time_limit_is_reported():
    """A request that runs past the server's limit is reported as an error and
    does not keep the server waiting."""
    be = SleepBackend(step_s=0.05)
    lines = []
    srv = Server(be, mem_budget=1000, window=2, request_timeout=0.3, log=lines.append)
    res, summ = srv.run([_req(0, 100, 40, 0.0), _req(1, 100, 1, 0.0)])     # 2 s and 0.05 s of work
    assert res[0].error and "Timeout" in res[0].error
    assert res[1].error is None
    assert any("exceeded" in l for l in lines) and any("admitted" in l for l in lines)


class FakeSolver:
    def __init__(self):
        self.k = 0
        self.cancel_flag = False
        self.closed = False

    def cancel(self):
        assert not self.closed
        self.cancel_flag = True

    def info(self):
        return {"steps_done": self.k}


class SleepBatchBackend:
    """The batch server's backend on the host: setup sleeps, a batch call
    sleeps per step (once for all its solvers) and honours cancel flags at
    its start and halfway through, as mot_run_batch does at window
    boundaries."""

    def __init__(self, step_s=0.001, setup_s=0.01):
        self.step_s, self.setup_s = step_s, setup_s
        self.lock = threading.Lock()
        self.live = {}
        self.max_live = 0
        self.max_batch = 0
        self.max_bytes = 0

    def footprint(self, req):
        return req.problem["bytes"]

    def setup(self, req):
        time.sleep(self.setup_s)
        s = FakeSolver()
        with self.lock:
            self.live[req.rid] = req.problem["bytes"]
            self.max_live = max(self.max_live, len(self.live))
            self.max_bytes = max(self.max_bytes, sum(self.live.values()))
        return s

    def run_batch(self, solvers, n):
        self.max_batch = max(self.max_batch, len(solvers))
        codes = []
        half = n // 2
        time.sleep(self.step_s * half)
        for s in solvers:
            if s.cancel_flag:
                s.cancel_flag = False
                codes.append("cancelled")
            else:
                s.k += half
                codes.append(None)
        time.sleep(self.step_s * (n - half))
        for i, s in enumerate(solvers):
            if codes[i] is None:
                if s.cancel_flag:
                    s.cancel_flag = False
                    codes[i] = "cancelled"
                else:
                    s.k += n - half
                    codes[i] = 0
        return codes

    def outputs(self, req, s, nsteps):
        return {"w": [s.k]}

    def close(self, req, s):
        s.closed = True
        with self.lock:
            del self.live[req.rid]


def test_batch_server_budget_overlap_and_all_finish():
    from paper_2510_07989_amd.serve import BatchServer
    be = SleepBatchBackend()
    reqs = [_req(i, 300 + 100 * (i % 3), 40 + 7 * i, 0.004 * i) for i in range(12)]
    srv = BatchServer(be, mem_budget=1000, max_active=8, window=16)
    res, summ = srv.run(reqs)
    assert summ["errors"] == 0 and summ["completed"] == 12 and summ["cancelled"] == 0
    assert be.max_bytes <= 1000 and summ["peak_budget_used"] <= 1000
    assert be.max_batch >= 2                       # solves marched together
    for r in res.values():
        assert len(r.step_latency) == r.nsteps and r.outputs["w"] == [r.nsteps]
        assert r.t_arrival <= r.t_admit <= r.t_ready <= r.t_done


def test_batch_server_time_box_cancels_and_drops():
    """At the time box every running solve is cancelled at its next window
    boundary (its completed steps counted), requests not yet admitted are not
    served, and every slot and byte is given back."""
    from paper_2510_07989_amd.serve import BatchServer
    be = SleepBatchBackend(step_s=0.002)
    reqs = [_req(i, 400, 400, 0.05 * i) for i in range(8)]
    srv = BatchServer(be, mem_budget=1000, max_active=2, window=32, time_box=0.3)
    res, summ = srv.run(reqs)
    assert summ["cancelled"] >= 1 and summ["not_served"] >= 1 and summ["errors"] == 0
    assert summ["completed"] + summ["cancelled"] + summ["not_served"] == 8
    assert not be.live                              # every solve closed
    for r in res.values():
        if r.error and r.error.startswith("CancelledRun"):
            assert 0 < len(r.step_latency) < r.nsteps
    assert summ["wall_s"] < 0.3 + 0.5


def test_batch_server_request_timeout_frees_the_slot():
    """A request past its time limit is cancelled and its slot goes to the
    next one, which completes."""
    from paper_2510_07989_amd.serve import BatchServer
    be = SleepBatchBackend(step_s=0.002)
    reqs = [_req(0, 900, 100000, 0.0), _req(1, 900, 50, 0.01)]
    srv = BatchServer(be, mem_budget=1000, max_active=2, window=32, request_timeout=0.2)
    res, summ = srv.run(reqs)
    assert res[0].error.startswith("CancelledRun") and res[1].error is None
    assert res[1].t_admit >= res[0].t_done - 1e-6
    assert summ["completed"] == 1 and summ["cancelled"] == 1


class CancellableSleepBackend(SleepBackend):
    """SleepBackend whose requests stop at a window boundary once cancelled."""

    def __init__(self, step_s=0.002):
        super().__init__(step_s)
        self.flags = {}

    def cancel(self, rid):
        self.flags[rid] = True
        return True

    def execute(self, req, window, clock, res):
        from paper_2510_07989_amd.serve import CancelledRun
        res.t_ready = clock()
        done = 0
        while done < req.nsteps:
            if self.flags.pop(req.rid, False):
                raise CancelledRun("stopped after %d steps" % done)
            nw = min(window, req.nsteps - done)
            t0 = clock()
            time.sleep(self.step_s * nw)
            res.step_latency.extend([(clock() - t0) / nw] * nw)
            done += nw


def test_thread_server_cancels_a_request_past_its_limit():
    """The per-thread server stops a request past its time limit through the
    backend's cancel; its slot and memory then go to the next request."""
    be = CancellableSleepBackend()
    reqs = [_req(0, 900, 100000, 0.0), _req(1, 900, 40, 0.01)]
    srv = Server(be, mem_budget=1000, max_active=2, window=16, request_timeout=0.2)
    res, summ = srv.run(reqs)
    assert res[0].error.startswith("CancelledRun") and res[1].error is None
    assert res[1].t_admit >= res[0].t_done - 1e-6


def test_thread_server_time_box_cancels_and_drops():
    """At the time box the per-thread server cancels every running request at
    its next window boundary (the steps it completed are kept and counted),
    admits nothing more and reports the rest as not served; every request is
    accounted for once."""
    be = CancellableSleepBackend(step_s=0.002)
    reqs = [_req(i, 400, 400, 0.05 * i) for i in range(8)]
    srv = Server(be, mem_budget=1000, max_active=2, window=32, time_box=0.3)
    res, summ = srv.run(reqs)
    assert summ["cancelled"] >= 1 and summ["not_served"] >= 1 and summ["errors"] == 0
    assert summ["completed"] + summ["cancelled"] + summ["not_served"] == 8
    for r in res.values():
        if r.error and r.error.startswith("CancelledRun"):
            assert 0 < len(r.step_latency) < r.nsteps
        if r.error and r.error.startswith("NotServed"):
            assert not r.step_latency and r.t_admit == 0
    assert summ["steps_marched"] == sum(len(r.step_latency) for r in res.values())
    assert summ["wall_s"] < 0.3 + 0.5


def test_thread_server_reports_a_request_that_ignores_its_cancel():
    """A cancelled request whose thread does not end within the grace period
    is reported as stalled and no longer waited on; the request that only its
    memory keeps out is not served, the others complete, and the server ends.
    The thread's later end does not overwrite the report."""
    release = threading.Event()

    class StuckBackend(CancellableSleepBackend):
        def execute(self, req, window, clock, res):
            if req.rid == 0:
                res.t_ready = clock()
                release.wait(30.0)             # never looks at its cancel flag
                raise RuntimeError("ended late")
            return super().execute(req, window, clock, res)

    be = StuckBackend(step_s=0.001)
    reqs = [_req(0, 600, 100000, 0.0), _req(1, 300, 40, 0.01), _req(2, 700, 40, 0.02)]
    lines = []
    srv = Server(be, mem_budget=1000, max_active=3, window=16, request_timeout=0.2, cancel_grace=0.2,
                 log=lines.append)
    t0 = time.perf_counter()
    res, summ = srv.run(reqs)
    assert time.perf_counter() - t0 < 5.0
    assert res[0].error.startswith("Stalled") and summ["stalled"] == 1
    assert res[1].error is None
    assert res[2].error.startswith("NotServed")     # 700 B fit only once the stalled 600 B are back
    assert any("Stalled" in l for l in lines)
    release.set()
    time.sleep(0.1)
    assert res[0].error.startswith("Stalled")


def test_gpu_backend_cancel_bookkeeping_without_a_device():
    """The GPU backend's cancel path on the host: a request flagged before its
    solver exists is stopped when the solver registers (mot_cancel and the
    loader flag), a live solver is stopped by cancel(), an unknown request is
    left alone, and a loader that checks stop_if_cancelled stops between lags."""
    from paper_2510_07989_amd.serve import CancelledRun, GpuBackend, Result, stop_if_cancelled

    class FakeSolver:
        def __init__(self):
            self.cancels = 0

        def cancel(self):
            self.cancels += 1

    be = GpuBackend(setup_slots=2)
    assert be.cancel(7) is False
    early = Result(1, 10, 0, 0.0)
    early.cancel_requested = True
    s1 = FakeSolver()
    be._register(1, s1, early)
    assert s1.cancels == 1 and s1._serve_cancelled
    with pytest.raises(CancelledRun):
        stop_if_cancelled(s1)
    s2 = FakeSolver()
    be._register(2, s2, Result(2, 10, 0, 0.0))
    stop_if_cancelled(s2)                       # not cancelled: the loader goes on
    assert s2.cancels == 0 and be.cancel(2) is True and s2.cancels == 1
    with pytest.raises(CancelledRun):
        stop_if_cancelled(s2)
    be._unregister(1)
    be._unregister(2)
    assert be.cancel(1) is False and be.cancel(2) is False and not be._live


def test_batch_server_reports_a_stalled_setup_and_ends():
    """A setup that does not return within the setup time limit is reported
    as stalled; the server stops waiting for it, serves the others, reports
    the requests that only the stalled setup's memory keeps out as not
    served, and ends. The setup, once it returns, closes its solver."""
    from paper_2510_07989_amd.serve import BatchServer
    release = threading.Event()

    class StallingBackend(SleepBatchBackend):
        def setup(self, req):
            if req.rid == 1:
                release.wait(30.0)
            return super().setup(req)

    be = StallingBackend(step_s=0.001)
    reqs = [_req(0, 300, 64, 0.0), _req(1, 500, 64, 0.0), _req(2, 300, 64, 0.01), _req(3, 800, 64, 0.02)]
    lines = []
    srv = BatchServer(be, mem_budget=1000, max_active=4, window=16, setup_timeout=0.3, log=lines.append)
    t0 = time.perf_counter()
    res, summ = srv.run(reqs)
    assert time.perf_counter() - t0 < 5.0
    assert summ["stalled_setups"] == 1
    assert res[1].error.startswith("SetupStalled")
    assert res[0].error is None and res[2].error is None
    assert res[3].error.startswith("NotServed")   # 800 B fit only once the stalled 500 B are back
    assert summ["completed"] == 2
    assert any("stalled" in l for l in lines)
    release.set()
    for _ in range(200):
        with be.lock:
            if not be.live:
                break
        time.sleep(0.01)
    assert not be.live                              # the late setup's solver was closed
