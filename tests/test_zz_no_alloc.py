"""The allocation-free call mot_step_norms_noalloc against mot_step_norms
(MI355X only): the same kernel writes both, once into a buffer allocated for
the call, once into the device's static scratch array, so the results agree
bit for bit, on consecutive calls of different sizes and across handles that
share the array."""
import ctypes

import numpy as np
import pytest

from tests._problems import problem

pytestmark = pytest.mark.gpu

MAXV = 131072          # MOT_NOALLOC_DOUBLES


def _solver(name, max_steps):
    import paper_2510_07989_amd as p
    print("inputs", name, flush=True)
    prob = problem(name)
    print("create", name, flush=True)
    o = p.default_options(precond=2, max_steps=max_steps)
    s = p.Solver(prob["V"], prob["F"], prob["E"], prob["eps_r"], prob["mu_r"], prob["dt"], prob["T0s"],
                 prob["T0h"], prob["G"], prob["waves"], options=o)
    s.load_raw(prob["raw"], prob["kmax"])
    return s


def _noalloc(s, first, count):
    out = np.full((max(count, 0), s.nrhs), np.nan)
    rc = s._lib.mot_step_norms_noalloc(s._h, int(first), int(count), out.ctypes.data_as(ctypes.c_void_p))
    return rc, out


def test_noalloc_norms_equal_allocating_call():
    from paper_2510_07989_amd import _lib as L
    nst = 240
    s = _solver("sphere_480_r16", nst)
    for i in range(2):
        print("march", 120 * i, flush=True)
        s.run(120, w=False, loop=False, star=False)
    print("norms", flush=True)
    rc, got = _noalloc(s, 0, nst)
    assert rc == L.MOT_OK, s._lib.mot_last_error(s._h)
    ref = s.step_norms(0, nst)
    assert np.array_equal(got, ref)
    assert np.isfinite(got).all() and got.max() > 0
    # a second, smaller call: nothing of the first may show
    rc, got2 = _noalloc(s, 100, 37)
    assert rc == L.MOT_OK
    assert np.array_equal(got2, s.step_norms(100, 37))
    assert np.array_equal(got2, ref[100:137])
    # beyond the static array: refused with a clear message, nothing written;
    # exactly at it, only the range decides
    big = MAXV // s.nrhs
    rc, over = _noalloc(s, 0, big + 1)
    assert rc == L.MOT_EINVAL
    assert b"static scratch" in s._lib.mot_last_error(s._h)
    assert np.isnan(over).all()
    rc, _ = _noalloc(s, 0, big)
    assert rc == L.MOT_EINVAL and b"out of range" in s._lib.mot_last_error(s._h)
    # a second handle on the same GPU shares the array
    t = _solver("tiny", 60)
    print("march tiny", flush=True)
    t.run(60, w=False, loop=False, star=False)
    rc, gt = _noalloc(t, 0, 60)
    assert rc == L.MOT_OK
    assert np.array_equal(gt, t.step_norms(0, 60))
    rc, got3 = _noalloc(s, 0, 3)
    assert rc == L.MOT_OK and np.array_equal(got3, ref[:3])
    # empty and bad ranges
    assert _noalloc(s, 10, 0)[0] == L.MOT_OK
    assert _noalloc(s, nst - 2, 5)[0] == L.MOT_EINVAL
    assert _noalloc(s, -1, 2)[0] == L.MOT_EINVAL
    t.close()
    s.close()
    print("done", flush=True)
