"""Conditioning of the qHP Q_0 seen by the GPU solver (Sec. VI): without the
approximate inverse, the GMRES iterations per step stay flat as c dt grows
past the diameter and as the mesh is refined, and each march matches the
oracle of its problem (MI355X only)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_gmres_iterations_flat_in_dt():
    import paper_2510_07989_amd as p
    from fixture.problem import CONFIGS, build_problem
    from oracle.mot_oracle import Oracle
    its = []
    for dt in (4.0, 16.0, 64.0, 256.0, 512.0):         # c dt up to 512 m, as in Sec. VI
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


def test_gmres_iterations_flat_in_h():
    """Sphere refined from 120 to 480 edges at dt = 1: the GMRES iteration
    count per step (no approximate inverse, tolerance 1e-12) does not grow."""
    import paper_2510_07989_amd as p
    from fixture.problem import CONFIGS, build_problem
    from oracle.mot_oracle import Oracle
    its = []
    for nu in (2, 3, 4):
        print("icosphere", nu, flush=True)
        prob = build_problem(cfg=dict(CONFIGS["sphere_480"], mesh=("icosphere", nu), dt=1.0), nsteps=30)
        s = p.Solver(prob["V"], prob["F"], prob["E"], prob["eps_r"], prob["mu_r"], prob["dt"], prob["T0s"],
                     prob["T0h"], prob["G"], prob["waves"], options=p.default_options(precond=0, gmres_tol=1e-12))
        s.load_raw(prob["raw"], prob["kmax"])
        out = s.run(30)
        its.append(s.info()["gmres_iters_total"] / 30.0)
        s.close()
        ref = Oracle(prob).run(30)
        e = np.linalg.norm(out["w"] - ref["W"]) / np.linalg.norm(ref["W"])
        print("edges %d: iterations per step %.2f, error %.2e" % (prob["E"].shape[0], its[-1], e), flush=True)
        assert e < 1e-9
    assert max(its) / min(its) < 1.5, its
