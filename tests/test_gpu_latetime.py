"""A march that decays through the bottom of the FP64 range (MI355X only).

The 960-unknown sphere's unknowns fall by about 0.05 decades per step once
the pulse has passed (Sec. VI-A: no late-time growth), so near step 3,000
their entries drop below 1.5e-154, where a plain sum of their squares
underflows, and near step 6,000 below the normal range.  The GMRES openings
take their norms from scaled sums there; without that, the first Krylov
vector is off unit length and every step runs to the iteration cap.  Every
step must converge in the usual few iterations, the decay must go on at the
same rate through that band, and the march must keep its pace."""
import time

import numpy as np
import pytest

from tests._problems import problem

pytestmark = pytest.mark.gpu

NST = 8200


def _scaled_norms(w):
    """||w_s|| per step and wave without underflow (scaling by the largest entry)."""
    a = np.abs(w).max(axis=1, keepdims=True)
    a = np.where(a > 0, a, 1.0)
    return (np.sqrt(((w / a) ** 2).sum(axis=1)) * a[:, 0, :])


@pytest.mark.parametrize("name", ["sphere_480", "sphere_480_r16"])
def test_march_through_the_underflow_range(name):
    import paper_2510_07989_amd as p
    print("case", name, NST, "steps: inputs", flush=True)
    prob = problem(name)
    s = p.Solver(prob["V"], prob["F"], prob["E"], prob["eps_r"], prob["mu_r"], prob["dt"], prob["T0s"],
                 prob["T0h"], prob["G"], prob["waves"], options=p.default_options(precond=2, max_steps=NST))
    s.load_raw(prob["raw"], prob["kmax"])
    rates, its = [], []
    it0 = s.info()["gmres_iters_total"]
    for c in range(0, NST, 1025):
        n = min(1025, NST - c)
        t = time.perf_counter()
        out = s.run(n, w=False, loop=False, star=False)
        el = time.perf_counter() - t
        it1 = s.info()["gmres_iters_total"]
        rates.append(n / el)
        its.append((it1 - it0) / n)
        it0 = it1
        print("steps %d-%d: %.0f steps/s, %.2f GMRES its/step, last converged %d"
              % (c, c + n - 1, n / el, its[-1], out["last"]["converged"]), flush=True)
        assert out["last"]["converged"]
    # the few iterations of the early steps all along, and the same pace
    assert max(its) <= its[0] + 1.0, its
    assert min(rates) >= rates[1] / 3, rates
    # decay at one rate across the band where the squares underflow
    band = s.steps(2400, 1200, loop=False, star=False)["w"]
    lg = np.log10(_scaled_norms(band).max(axis=1))
    x = np.arange(lg.size)
    fin = np.isfinite(lg)
    lo, hi = fin & (x < 500), fin & (x >= 700)
    s_lo = np.polyfit(x[lo], lg[lo], 1)[0]
    s_hi = np.polyfit(x[hi], lg[hi], 1)[0]
    print("log10 ||w|| at steps 2400, 3000, 3599: %.1f %.1f %.1f; slopes %.4f / %.4f decades/step"
          % (lg[0], lg[600], lg[-1], s_lo, s_hi), flush=True)
    assert lg[-1] < -160 < -150 < lg[0]
    assert s_lo < 0 and abs(s_hi - s_lo) <= 0.2 * abs(s_lo)
    s.close()
