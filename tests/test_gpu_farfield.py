"""Spectra and far fields of the loop and star currents (mot_far_field)
against the oracle's, and against the oracle's transform of the GPU's own
currents (MI355X only)."""
import numpy as np
import pytest

from oracle import mot_oracle as mo
from tests._problems import problem, oracle

pytestmark = pytest.mark.gpu


def _solver(name, **opts):
    import paper_2510_07989_amd as p
    prob = problem(name)
    s = p.Solver(prob["V"], prob["F"], prob["E"], prob["eps_r"], prob["mu_r"], prob["dt"],
                 prob["T0s"], prob["T0h"], prob["G"], prob["waves"], options=p.default_options(**opts))
    s.load_raw(prob["raw"], prob["kmax"])
    return s


def _dirs(n=13):
    th = np.linspace(0, np.pi, n)
    ph = np.linspace(0.3, 2.0, n)
    return np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], 1)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("name,nsteps,opts", [
    ("sphere_480", 200, {}),
    ("tiny_torus", 160, dict(recovery=1)),          # P^Sigma by incidence products and CG
    ("tiny_box", 120, {}),                           # two waves
    ("sphere_480_r16", 120, {}),                     # sixteen waves
])
def test_far_field_matches_oracle(name, nsteps, opts):
    print("case", name, nsteps, opts, flush=True)
    prob = problem(name)
    s = _solver(name, **opts)
    out = s.run(nsteps)
    O = oracle(name)
    ref = O.run(nsteps)
    dirs = _dirs()
    dt = prob["dt"]
    for freq, first, count in ((0.1, 0, nsteps), (0.0, 0, nsteps), (0.003, 0, nsteps), (0.37 / dt, 17, nsteps - 30)):
        got = s.far_field(first, count, freq, dirs)
        exp = O.far_field(ref, freq, dirs, first, count)
        e_spec = _rel(got["spec"], exp["spec"])
        e_field = _rel(got["field"], exp["field"])
        # the GPU's own currents transformed by the oracle: the transform alone
        own = {"loop": out["loop"], "star": out["star"], "W": out["w"]}
        mine = O.far_field(own, freq, dirs, first, count)
        e_own = max(_rel(got["spec"], mine["spec"]), _rel(got["field"], mine["field"]))
        print("  f %.4g first %d count %d: spec %.2e field %.2e vs own currents %.2e"
              % (freq, first, count, e_spec, e_field, e_own), flush=True)
        assert e_own < 1e-12
        assert e_spec < 1e-9 and e_field < 1e-9
        for part in range(2):
            assert _rel(got["field"][:, :, part], exp["field"][:, :, part]) < 1e-9
    s.close()


def test_far_field_arguments():
    import paper_2510_07989_amd as p
    s = _solver("tiny_box")
    with pytest.raises(p.MotError):
        s.far_field(0, 1, 0.1, _dirs())                 # no step taken yet
    s.run(20, w=False, loop=False, star=False)
    with pytest.raises(p.MotError):
        s.far_field(5, 16, 0.1, _dirs())                # step 20 not taken
    with pytest.raises(p.MotError):
        s.far_field(0, 20, -0.1, _dirs())
    with pytest.raises(p.MotError):
        s.far_field(0, 20, 0.1, 2 * _dirs())            # not unit vectors
    r = s.far_field(0, 20, 0.1)                         # spectra only
    assert r["field"].shape == (0, s.nrhs, 2, 3)
    assert np.abs(r["spec"]).max() > 0
    s.close()
    s = _solver("tiny_box", keep_history=0)
    s.run(10, w=False, loop=False, star=False)
    with pytest.raises(p.MotError):
        s.far_field(0, 10, 0.1, _dirs())                # nothing kept
    s.close()


def test_gpu_far_field_matches_mie():
    """The GPU's far field of the 480-edge sphere (eps_r = 2) against the
    Mie series, through the C ABI: within 5% in magnitude at k a = 0.63 and
    6e-5, and at the low frequency equal to the Mie field times the faceted
    sphere's volume fraction."""
    from tests.test_oracle import _mie_amplitudes
    prob = problem("sphere_480")
    s = _solver("sphere_480")
    s.run(prob["nsteps"], w=False, loop=False, star=False)
    wv = prob["waves"][0]
    kh, p = np.asarray(wv.dir, float), np.asarray(wv.pol, float)
    q = np.cross(kh, p)
    V, F = prob["V"], prob["F"]
    vol_ratio = np.einsum("ij,ij->i", V[F[:, 0]], np.cross(V[F[:, 1]], V[F[:, 2]])).sum() / 6.0 / (4 * np.pi / 3)
    th = np.radians(np.arange(0, 181, 10.0))
    for ph in (0.0, np.pi / 2):
        side = np.cos(ph) * p + np.sin(ph) * q
        dirs = np.array([np.cos(t) * kh + np.sin(t) * side for t in th])
        e_th = np.array([-np.sin(t) * kh + np.cos(t) * side for t in th])
        e_ph = np.broadcast_to(-np.sin(ph) * p + np.cos(ph) * q, dirs.shape)
        for f in (1e-5, 0.1):
            k = 2 * np.pi * f
            E = s.far_field(0, prob["nsteps"], f, dirs)["field"][:, 0].sum(axis=1)
            got = np.hypot(np.abs(np.einsum("ad,ad->a", E, e_th)), np.abs(np.einsum("ad,ad->a", E, e_ph)))
            S1, S2 = _mie_amplitudes(np.sqrt(prob["eps_r"]), k, np.cos(th))
            ref = wv.amp * np.exp(-(k * wv.width / 8) ** 2) / k * np.hypot(np.abs(S2 * np.cos(ph)),
                                                                             np.abs(S1 * np.sin(ph)))
            err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            print("phi %.2f f %g: %.3e vs Mie" % (ph, f, err), flush=True)
            assert err < 0.05
            if f < 1e-3:
                keep = ref > 1e-3 * ref.max()
                assert np.allclose(got[keep] / ref[keep], vol_ratio, rtol=2e-3)
    s.close()


def test_step_norms_match_kept_unknowns():
    """mot_step_norms against the norms of the unknowns read back, and the
    late-time decay of the march they show (Sec. VI-A)."""
    import paper_2510_07989_amd as p
    for name in ("sphere_480", "sphere_480_r16"):
        prob = problem(name)
        s = _solver(name)
        n = 200 if name == "sphere_480" else 120
        out = s.run(n, loop=False, star=False)
        nr = s.step_norms(0, n)
        ref = np.linalg.norm(out["w"], axis=1)              # (n, nrhs)
        assert np.allclose(nr, ref, rtol=1e-13, atol=0)
        assert np.allclose(s.step_norms(37, 11), ref[37:48], rtol=1e-13, atol=0)
        late = np.log10(nr[-n // 4:, 0])
        assert np.polyfit(np.arange(late.size), late, 1)[0] < 0
        with pytest.raises(p.MotError):
            s.step_norms(n - 5, 6)
        s.close()
