"""Parity at the benchmark sizes, in the configuration bench.py times: the
oracle computes a prefix of the march; properties cover the rest."""
import numpy as np
import pytest

from tests._problems import problem

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _solver(prob, **opts):
    import paper_2510_07989_amd as p
    o = p.default_options(**opts)
    s = p.Solver(prob["V"], prob["F"], prob["E"], prob["eps_r"], prob["mu_r"], prob["dt"], prob["T0s"],
                 prob["T0h"], prob["G"], prob["waves"], options=o)
    s.load_raw(prob["raw"], prob["kmax"])
    return s


def test_torus_6144_prefix_and_late_time():
    """Torus, 6144 unknowns, dt = 2 (the headline workload), FP64 approximate
    inverse and speculative stepping as in the benchmark: the first 20 steps
    against the oracle to 1e-10; over 2000 steps, no late-time growth."""
    from oracle.mot_oracle import Oracle
    print("case torus_3072", flush=True)
    prob = problem("torus_3072", 2000)
    s = _solver(prob, precond=2, max_steps=2000)
    out = s.run(2000)
    s.close()
    ref = Oracle(prob).run(20)
    e = [_rel(out[k][:20], ref[r]) for k, r in (("w", "W"), ("loop", "loop"), ("star", "star"))]
    print("prefix errors", e, flush=True)
    assert max(e) < 1e-10
    nrm = np.linalg.norm(out["w"].reshape(2000, -1), axis=1)
    late = np.log10(nrm[-500:] + 1e-300)
    slope = np.polyfit(np.arange(late.size), late, 1)[0]
    print("late-time slope %.3e decades/step, last/peak %.2e" % (slope, nrm[-1] / nrm.max()), flush=True)
    assert slope <= 0.0 and nrm[-1] < 1e-6 * nrm.max()


@pytest.mark.parametrize("precision,bound", [(0, 1e-10), (1, 1e-6)])
def test_sphere_3840_16_waves_prefix(precision, bound):
    """Sphere, 3840 unknowns, 16 waves (the batched workload), FP64 and mixed:
    the first 10 steps against the oracle."""
    from oracle.mot_oracle import Oracle
    print("case sphere_1920_r16 precision", precision, flush=True)
    prob = problem("sphere_1920_r16", 40)
    s = _solver(prob, precond=2, precision=precision, max_steps=40)
    out = s.run(10)
    s.close()
    ref = Oracle(prob).run(10)
    e = [_rel(out[k], ref[r]) for k, r in (("w", "W"), ("loop", "loop"), ("star", "star"))]
    print("prefix errors", e, flush=True)
    assert e[0] < bound and e[1] < bound
