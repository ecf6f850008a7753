"""The GPU march against itself under the invariances the oracle is pinned
to (MI355X only): the sphere turned and scaled, with the step, the pulse and
the wave scaled and turned with it, marches to the same unknowns; with the
media swapped and the wave's polarisation turned, to the dual unknowns. The
properties hold at any size, so they check the path where the oracle does
not march."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _device_problem(name, cfg, move):
    import fixture.problem as fp
    from fixture import gpu
    orig = fp.make_mesh

    def moved_mesh(spec):
        V, F, E = orig(spec)
        return move(V), F, E
    fp.make_mesh = moved_mesh
    try:
        return gpu.build_problem_device(name, cfg=cfg)
    finally:
        fp.make_mesh = orig


def _march(prob, nsteps):
    import torch
    import paper_2510_07989_amd as mot
    from fixture import gpu
    s = mot.Solver(prob["V"], prob["F"], prob["E"], prob["eps_r"], prob["mu_r"], prob["dt"], prob["T0s"],
                   prob["T0h"], prob["G"], prob["waves"], options=mot.default_options(precond=2),
                   stream=torch.cuda.current_stream().cuda_stream)
    gpu.load_solvers([s], prob)
    out = s.run(nsteps)
    s.close()
    return out


@pytest.mark.parametrize("name,n,scale,seed", [("sphere_480", 200, 1.7, 11),
                                               ("sphere_1920_r16", 60, 0.6, 13)])
def test_turned_and_scaled_sphere_marches_the_same(name, n, scale, seed):
    """One wave on the 960-unknown sphere; 16 waves (the multi-RHS tile
    products) on the 3840-unknown sphere."""
    from fixture.problem import CONFIGS, Wave
    print("case", name, n, scale, flush=True)
    rng = np.random.Generator(np.random.PCG64(seed))
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    cfg = dict(CONFIGS[name])
    ref = _march(_device_problem(name, cfg, lambda V: V), n)
    cfg_s = dict(cfg, dt=cfg["dt"] * scale, sigma=cfg["sigma"] * scale)
    prob = _device_problem(name, cfg_s, lambda V: scale * V @ Q.T)
    prob["waves"] = [Wave(w.amp, Q @ w.pol, Q @ w.dir, w.width, w.t0) for w in prob["waves"]]
    got = _march(prob, n)
    for k in ("w", "loop", "star"):
        e = _rel(got[k], ref[k])
        print(k, "%.2e" % e, flush=True)
        assert e < 1e-10, (k, e)


def test_swapped_media_march_is_the_dual():
    """Duality of the PMCHWT: eps' and mu' swapped and the polarisation
    turned from p to k x p give (v; -u) of the first march, for w and the
    loop and star parts."""
    from fixture.problem import CONFIGS, Wave
    name, n = "sphere_480", 150
    print("case duality", name, n, flush=True)
    cfg = dict(CONFIGS[name])
    pa = _device_problem(name, dict(cfg, eps_r=3.0, mu_r=1.5), lambda V: V)
    pb = _device_problem(name, dict(cfg, eps_r=1.5, mu_r=3.0), lambda V: V)
    pb["waves"] = [Wave(w.amp, np.cross(w.dir, w.pol), w.dir, w.width, w.t0) for w in pa["waves"]]
    ne = pa["E"].shape[0]
    A, B = _march(pa, n), _march(pb, n)
    for k in ("w", "loop", "star"):
        a, b = A[k], B[k]
        e = (np.linalg.norm(b[:, :ne] - a[:, ne:]) + np.linalg.norm(b[:, ne:] + a[:, :ne])) / np.linalg.norm(a)
        print(k, "%.2e" % e, flush=True)
        assert e < 1e-10, (k, e)
