"""Checkpoint and restore of the march (MI355X only): a march resumed in a new
handle from a checkpoint continues bit for bit as the original, with the full
kept history or with the last step only; mismatched handles are refused."""
import numpy as np
import pytest

from tests._problems import problem

pytestmark = pytest.mark.gpu


def _solver(name, **opts):
    import paper_2510_07989_amd as p
    prob = problem(name)
    s = p.Solver(prob["V"], prob["F"], prob["E"], prob["eps_r"], prob["mu_r"], prob["dt"],
                 prob["T0s"], prob["T0h"], prob["G"], prob["waves"], options=p.default_options(**opts))
    s.load_raw(prob["raw"], prob["kmax"])
    return s


@pytest.mark.parametrize("name,opts,n1,n2", [
    ("sphere_480", dict(precond=2), 150, 130),
    ("sphere_480", dict(precond=1), 137, 140),            # FP32 inverse: halts, grown Arnoldi count
    ("tiny_torus", dict(precond=2, spec_window=-1), 61, 50),
    ("sphere_480_r16", dict(precond=2, precision=1), 90, 60),
    ("sphere_480", dict(precond=2, history_form=1), 150, 130),   # projected rings rebuilt at the restore
])
def test_resume_is_bit_identical(name, opts, n1, n2):
    import paper_2510_07989_amd as p
    print("case", name, opts, n1, n2, flush=True)
    a = _solver(name, **opts)
    first = a.run(n1)
    full = a.checkpoint(True)
    last = a.checkpoint(False)
    assert last.size < full.size
    ref = a.run(n2)
    ia = a.info()
    a.close()
    for buf, with_hist in ((full, True), (last, False)):
        b = _solver(name, **opts)
        b.restore(buf)
        assert b.info()["steps_done"] == n1
        out = b.run(n2)
        for k in ("w", "loop", "star"):
            assert np.array_equal(out[k], ref[k]), (with_hist, k)
        assert b.info()["gmres_iters_total"] == ia["gmres_iters_total"]
        if with_hist:
            got = b.steps(0, n1)
            for k in ("w", "loop", "star"):
                assert np.array_equal(got[k], first[k]), k
        else:
            with pytest.raises(p.MotError):
                b.steps(0, n1)                          # not held
            tail = b.steps(n1 - 1, 1)
            assert np.array_equal(tail["w"], first["w"][-1:])
        b.close()


def test_restore_refuses_a_mismatch():
    import paper_2510_07989_amd as p
    a = _solver("tiny_torus", precond=2)
    a.run(20, w=False, loop=False, star=False)
    buf = a.checkpoint(False)
    a.close()
    for other, opts in (("tiny", dict(precond=2)), ("tiny_torus", dict(precond=1))):
        b = _solver(other, **opts)
        with pytest.raises(p.MotError):
            b.restore(buf)
        b.close()
    b = _solver("tiny_torus", precond=2)
    with pytest.raises(p.MotError):
        b.restore(buf[:100])                            # truncated
    bad = buf.copy()
    bad[:8] = 0
    with pytest.raises(p.MotError):
        b.restore(bad)                                  # not a checkpoint
    b.restore(buf)                                      # the right one still works
    assert b.info()["steps_done"] == 20
    b.close()


def test_checkpoint_after_marching_past_the_kept_capacity():
    """A march without outputs may pass max_steps; the last step is then not
    kept, and a checkpoint holds no history (rather than reading past the kept
    range).  A handle restored from it continues bit for bit: the state saved
    after ten more steps on each is byte-identical."""
    print("case tiny_torus max_steps=30", flush=True)
    a = _solver("tiny_torus", precond=2, max_steps=30)
    a.run(45, w=False, loop=False, star=False)
    full, last = a.checkpoint(True), a.checkpoint(False)
    assert full.size == last.size                      # neither holds kept steps
    b = _solver("tiny_torus", precond=2, max_steps=30)
    b.restore(last)
    assert b.info()["steps_done"] == 45
    a.run(10, w=False, loop=False, star=False)
    b.run(10, w=False, loop=False, star=False)
    assert np.array_equal(a.checkpoint(False), b.checkpoint(False))
    a.close()
    b.close()


def test_checkpoint_chained_through_a_restore_without_history():
    """Restore a last-step-only checkpoint, then checkpoint again before any
    step: the saved slot k-1 is the one that was restored, and a handle that
    restores the second checkpoint continues bit for bit."""
    print("case sphere_480 chained checkpoints", flush=True)
    a = _solver("sphere_480", precond=2)
    a.run(40)
    buf1 = a.checkpoint(False)
    ref = a.run(25)
    a.close()
    b = _solver("sphere_480", precond=2)
    b.restore(buf1)
    buf2 = b.checkpoint(False)
    b.close()
    c = _solver("sphere_480", precond=2)
    c.restore(buf2)
    out = c.run(25)
    for k in ("w", "loop", "star"):
        assert np.array_equal(out[k], ref[k]), k
    c.close()
