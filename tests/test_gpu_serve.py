"""Serving on the GPU: admission by footprint, overlap, same result alone and in the mix."""
import numpy as np
import pytest

from tests._problems import problem

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("name,opts", [("sphere_480", {}), ("sphere_480", dict(precond=2)),
                                       ("sphere_480_r16", dict(precond=2)),
                                       ("sphere_480_r16", dict(precond=2, precision=1))])
def test_footprint_matches_allocations(name, opts):
    """mot_footprint before create equals the bytes the handle holds after
    setup and the fold, and bounds the high-water mark through a run."""
    import paper_2510_07989_amd as p
    print("case", name, opts, flush=True)
    prob = problem(name)
    o = p.default_options(max_steps=200, **opts)
    res, peak = p.footprint(prob["V"], prob["F"], prob["E"], prob["eps_r"], prob["mu_r"], prob["dt"],
                            len(prob["waves"]), prob["G"], o)
    s = p.Solver(prob["V"], prob["F"], prob["E"], prob["eps_r"], prob["mu_r"], prob["dt"], prob["T0s"],
                 prob["T0h"], prob["G"], prob["waves"], options=o)
    s.load_raw(prob["raw"], prob["kmax"])
    inf = s.info()
    print("resident estimate %d, held %d; peak estimate %d" % (res, inf["device_bytes"], peak), flush=True)
    assert abs(inf["device_bytes"] - res) <= 1e-3 * res
    s.run(150, device=True)
    inf = s.info()
    print("high-water mark %d" % inf["peak_bytes"], flush=True)
    assert inf["peak_bytes"] <= peak
    s.close()


def test_same_result_alone_and_in_the_mix():
    """Five solves on different meshes (one with two waves, one with 16 waves
    in mixed precision) arrive staggered under a budget that makes some wait;
    each result equals the same request served alone (to 1e-12, in practice
    bit for bit, mixed precision included), solves ran concurrently, and the
    served sphere matches the FP64 oracle (eq. (MOT), eq. (dis_jm))."""
    from paper_2510_07989_amd.serve import GpuBackend, Request, Server
    specs = [("tiny", 60), ("tiny_torus", 60), ("tiny_box", 40), ("sphere_480", 150), ("sphere_480_r16", 80)]
    reqs = [Request(i, problem(n), ns, arrival=0.03 * i,
                    options=dict(precond=2, precision=1 if n == "sphere_480_r16" else 0))
            for i, (n, ns) in enumerate(specs)]
    be = GpuBackend()
    alone = {}
    for r in reqs:
        print("alone", r.rid, specs[r.rid][0], flush=True)
        res, _ = Server(be, mem_budget=1 << 40, window=32).run([Request(r.rid, r.problem, r.nsteps, 0.0, r.options)])
        assert res[r.rid].error is None, res[r.rid].error
        alone[r.rid] = res[r.rid].outputs
    fps = sorted(be.footprint(r) for r in reqs)
    budget = fps[-1] + fps[-2] + fps[0]          # the largest two and the smallest fit together
    print("mix, budget %d" % budget, flush=True)
    srv = Server(be, mem_budget=budget, max_active=3, window=32)
    res, summ = srv.run(reqs)
    print("summary", {k: summ[k] for k in ("wall_s", "steps_per_s", "max_concurrent", "peak_budget_used")}, flush=True)
    assert summ["errors"] == 0, [r.error for r in res.values()]
    assert summ["max_concurrent"] >= 2
    assert summ["peak_budget_used"] <= budget
    for rid, r in res.items():
        for k in ("w", "loop", "star"):
            e = _rel(r.outputs[k], alone[rid][k])
            assert e <= 1e-12, (rid, k, e)
    lat = summ["step_latency_s"]
    assert lat["n"] == sum(ns for _, ns in specs) and lat["p99"] >= lat["p50"] > 0
    from tests._problems import oracle
    ref = oracle("sphere_480").run(150)
    for k, r in (("w", "W"), ("loop", "loop"), ("star", "star")):
        assert _rel(res[3].outputs[k], ref[r]) < 1e-10, k
    ref16 = oracle("sphere_480_r16").run(80)
    for k, r in (("w", "W"), ("loop", "loop"), ("star", "star")):
        assert _rel(res[4].outputs[k], ref16[r]) < 1e-6, k
