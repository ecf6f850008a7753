"""Conditioning of the qHP Q_0 seen by the GPU solver (Sec. VI): without the
approximate inverse, the GMRES iterations per step stay flat as c dt grows
past the diameter, and each march matches the oracle of its time step
(MI355X only)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_gmres_iterations_flat_in_dt():
    import paper_2510_07989_amd as p
    from fixture.problem import CONFIGS, build_problem
    from oracle.mot_oracle import Oracle
    its = []
    for dt in (4.0, 16.0, 64.0):
        print("dt", dt, flush=True)
        prob = build_problem(cfg=dict(CONFIGS["tiny_box"], dt=dt), nsteps=20)
        waves = prob["waves"][:1]
        s = p.Solver(prob["V"], prob["F"], prob["E"], prob["eps_r"], prob["mu_r"], prob["dt"], prob["T0s"],
                     prob["T0h"], prob["G"], waves, options=p.default_options(precond=0, gmres_tol=1e-12))
        s.load_raw(prob["raw"], prob["kmax"])
        out = s.run(20)
        its.append(s.info()["gmres_iters_total"] / 20.0)
        s.close()
        ref = Oracle(dict(prob, waves=waves)).run(20)
        e = np.linalg.norm(out["w"] - ref["W"]) / np.linalg.norm(ref["W"])
        print("iterations per step %.2f, error %.2e" % (its[-1], e), flush=True)
        assert e < 1e-9
    assert max(its) / min(its) < 1.5, its
