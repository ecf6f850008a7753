"""Several solves marched together by mot_run_batch (their speculative windows
interleaved across streams) give exactly what each gives alone, and
mot_get_steps returns what mot_run returned for the same steps (MI355X only)."""
import numpy as np
import pytest

from tests._problems import problem, oracle

pytestmark = pytest.mark.gpu

# FP64 inverse; FP32 inverse (halted steps finished on the host); 16 plane
# waves; host-waited steps (not speculative); graph replay; mixed precision
CASES = [("sphere_480", dict(precond=2)), ("tiny_torus", dict(precond=1)),
         ("sphere_480_r16", dict(precond=2)), ("tiny_box", dict(precond=2, spec_window=-1)),
         ("sphere_480", dict(precond=2, graph=1)), ("sphere_480_r16", dict(precond=2, precision=1))]


def _solver(name, opts, stream=True):
    import torch
    import paper_2510_07989_amd as p
    prob = problem(name)
    st = torch.cuda.Stream() if stream else None
    s = p.Solver(prob["V"], prob["F"], prob["E"], prob["eps_r"], prob["mu_r"], prob["dt"],
                 prob["T0s"], prob["T0h"], prob["G"], prob["waves"], options=p.default_options(**opts),
                 stream=st.cuda_stream if st is not None else None)
    s.load_raw(prob["raw"], prob["kmax"])
    s._keep_stream = st
    return s


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("streams", [True, False])
def test_batch_equals_alone(streams):
    import paper_2510_07989_amd as p
    print("batch of", [c[0] for c in CASES], "own streams" if streams else "default stream", flush=True)
    alone = []
    for name, opts in CASES:
        s = _solver(name, opts, streams)
        out = s.run(300)
        alone.append((out, s.info()))
        s.close()
    ss = [_solver(name, opts, streams) for name, opts in CASES]
    st = p.run_batch(ss, 170)                   # not a multiple of any window
    assert all(c == 0 for c in st), st
    st = p.run_batch(ss, 130)
    assert all(c == 0 for c in st), st
    for (name, opts), s, (ref, iref) in zip(CASES, ss, alone):
        got = s.steps(0, 300)
        info = s.info()
        print(name, "iters", info["gmres_iters_total"], iref["gmres_iters_total"], flush=True)
        assert info["steps_done"] == 300
        assert info["gmres_iters_total"] == iref["gmres_iters_total"], name
        for k in ("w", "loop", "star"):
            assert np.array_equal(got[k], ref[k]), (name, k)
        tail = s.steps(280, 20, loop=False, star=False)
        assert np.array_equal(tail["w"], ref["w"][280:]), name
        s.close()
    ref = oracle("sphere_480").run(300)
    assert _rel(alone[0][0]["w"], ref["W"]) < 1e-10
    if streams:
        assert alone[4][1]["graph_windows"] >= 1            # the graph case replayed windows


def test_batch_arguments():
    import paper_2510_07989_amd as p
    s = _solver("sphere_480", dict(precond=2))
    with pytest.raises(p.MotError):
        p.run_batch([s, s], 10)                 # a handle listed twice
    assert s.info()["steps_done"] == 0
    assert p.run_batch([], 10) == []
    assert p.run_batch([s], 0) == [0]
    p.run_batch([s], 20)
    with pytest.raises(p.MotError):
        s.steps(10, 11)                         # step 20 not taken yet
    with pytest.raises(p.MotError):
        s.steps(-1, 2)
    a = s.steps(5, 10)
    b = s.run(5)
    assert a["w"].shape == (10, s.n, s.nrhs)
    c = s.steps(20, 5)
    for k in ("w", "loop", "star"):
        assert np.array_equal(b[k], c[k]), k
    s.close()
