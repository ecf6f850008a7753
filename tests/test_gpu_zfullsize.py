"""Parity at the benchmark sizes, in the configuration bench.py times: the
oracle computes a prefix of the march; properties cover the rest."""
import time

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
    """Torus, 6144 unknowns, dt = 2 (the torus workload), FP64 approximate
    inverse and speculative stepping as in the benchmark, for the whole
    10,000-step march: the first 20 steps against the oracle to 1e-10
    (Section V-A eq. (MOT), eq. (dis_jm)); no late-time growth (Section VI-A):
    over the last 2000 steps the least-squares slope of log10 ||w_k|| is not
    positive and ||w_k|| stays below 1e-10 of its peak."""
    from oracle.mot_oracle import Oracle
    print("case torus_3072 10000 steps", flush=True)
    nt = 10000
    prob = problem("torus_3072", 20)
    s = _solver(prob, precond=2, max_steps=nt)
    s.run(nt, w=False, loop=False, star=False)
    head = s.steps(0, 20)
    nrm = s.step_norms(0, nt)[:, 0]
    s.close()
    ref = Oracle(prob).run(20)
    e = [_rel(head[k], ref[r]) for k, r in (("w", "W"), ("loop", "loop"), ("star", "star"))]
    print("prefix errors", e, flush=True)
    assert max(e) < 1e-10
    late = np.log10(nrm[-2000:] + 1e-300)
    slope = np.polyfit(np.arange(late.size), late, 1)[0]
    print("late-time slope %.3e decades/step, late max/peak %.2e" % (slope, nrm[-2000:].max() / nrm.max()),
          flush=True)
    assert slope <= 0.0 and nrm[-2000:].max() <= 1e-10 * nrm.max()


@pytest.mark.parametrize("precision,bound", [(0, 1e-10), (1, 1e-6)])
def test_sphere_3840_16_waves_prefix(precision, bound):
    """Sphere, 3840 unknowns, 16 waves, FP64 and mixed (FP32 storage, FP64
    products): the first 10 steps against the oracle, w, loop and star parts."""
    from oracle.mot_oracle import Oracle
    print("case sphere_1920_r16 precision", precision, flush=True)
    prob = problem("sphere_1920_r16", 40)
    s = _solver(prob, precond=2, precision=precision, max_steps=40)
    out = s.run(10)
    s.close()
    ref = _oracle_1920().run(10)
    e = [_rel(out[k], ref[r]) for k, r in (("w", "W"), ("loop", "loop"), ("star", "star"))]
    print("prefix errors", e, flush=True)
    assert max(e) < bound, e


_O1920 = {}


def _oracle_1920():
    """The oracle of the 3840-unknown sphere (its lag matrices do not depend on
    the waves; the right-hand sides do)."""
    from oracle.mot_oracle import Oracle
    if "o" not in _O1920:
        _O1920["o"] = Oracle(problem("sphere_1920_r16", 40))
    return _O1920["o"]


@pytest.mark.parametrize("precision,bound_w,bound_star", [(1, 1e-6, 1e-6), (2, 1e-5, 1e-4)])
def test_sphere_3840_64_waves_mixed_prefix(precision, bound_w, bound_star):
    """64 seeded waves on the 3840-unknown sphere, the width at which the
    history is a matrix-core product: the first 10 steps against the oracle.
    MOT_MIXED (FP64 products of FP32-stored lags) meets 1e-6 on w, loop and
    star; MOT_MIXED32 (FP32 matrix-core products, 4-index FP32 sums) is held
    to its measured bounds (w 1e-5, star 1e-4) and is not the mixed path that
    meets the 1e-6 target."""
    import copy
    from fixture.problem import make_waves, CONFIGS
    print("case sphere_1920 64 waves precision", precision, flush=True)
    prob = dict(problem("sphere_1920_r16", 40))
    prob["waves"] = make_waves(64, CONFIGS["sphere_1920_r16"]["sigma"], True)
    O = copy.copy(_oracle_1920())
    O.prob = prob
    ref = O.run(10)
    s = _solver(prob, precond=2, precision=precision, max_steps=40)
    out = s.run(10)
    s.close()
    e = [_rel(out[k], ref[r]) for k, r in (("w", "W"), ("loop", "loop"), ("star", "star"))]
    print("prefix errors (precision %d): w %.3e loop %.3e star %.3e" % (precision, *e), flush=True)
    assert e[0] < bound_w and e[1] < bound_w and e[2] < bound_star


NL_C3 = 4
C3_STEPS = 38
C3_CHECK = (31, 34, 38)     # every one of the 31 lags active from step 31; the pulses pass by step 50


def _step_equation(prob, runs, checks, log):
    """eq. (MOT) on given unknowns: for each k in checks,
    || sum_j Q_j w_{k-j} - r_k || / || r_k || per run, every Q_j applied from
    the raw blocks of its lag as a second device assembly pass hands them over
    (lag_products, then C1b, C2b of eq. (CP)); r_k by eq. (rhs).
    runs: name -> W (K, 2 ne, R) with W[m - 1] = w_m.  Returns name -> errors."""
    import torch
    from fixture import gpu
    from oracle.mot_oracle import (incidence, projectors, preconditioner, lag_products, tested_fields, rhs, blk,
                                   time_constants)
    V, F, E = prob["V"], prob["F"], prob["E"]
    ne, R = E.shape[0], len(prob["waves"])
    _, Tmax, kmax = time_constants(V, prob["dt"], prob["eps_r"], prob["mu_r"])
    L = kmax + 2
    log("oracle: projectors")
    P = projectors(*incidence(E, V.shape[0], F.shape[0]))
    log("oracle: preconditioner")
    pre = preconditioner(prob["T0s"], prob["T0h"], prob["G"], P)
    names = list(runs)
    proj = {}
    for nm in names:
        W = runs[nm]
        XL = np.concatenate([P["PL"] @ W[:, :ne], P["PL"] @ W[:, ne:]], axis=1)
        proj[nm] = (XL, W - XL)
    Y1 = {(nm, k): np.zeros((2 * ne, R)) for nm in names for k in checks}
    Y2 = {(nm, k): np.zeros((2 * ne, R)) for nm in names for k in checks}
    codes = {(0, 0): "T_h", (0, 1): "K_h", (1, 0): "T_hat", (1, 1): "K_hat", (2, 0): "T_tilde", (2, 1): "K_tilde"}
    raw_i = {"ext": {}, "int": {}}
    t0 = time.perf_counter()

    def keep(fam, lag, med, op, t):
        raw_i[("ext", "int")[med]][codes[(fam, op)]] = t.cpu().numpy()

    def lag_done(j):
        cols = [(nm, k) for nm in names for k in checks if k - j >= 1]
        if cols:
            xl = np.concatenate([proj[nm][0][k - j - 1] for nm, k in cols], axis=1)
            xs = np.concatenate([proj[nm][1][k - j - 1] for nm, k in cols], axis=1)
            y1, y2 = lag_products(raw_i, prob["eps_r"], prob["mu_r"], Tmax, kmax, j, xl, xs)
            for c, key in enumerate(cols):
                Y1[key] += y1[:, c * R:(c + 1) * R]
                Y2[key] += y2[:, c * R:(c + 1) * R]
        raw_i["ext"].clear()
        raw_i["int"].clear()
        log("oracle: lag %d of %d applied (%.0f s)" % (j, L - 1, time.perf_counter() - t0))

    gpu.upload_lags(keep, V, F, E, prob["dt"], prob["eps_r"], prob["mu_r"], kmax, nq=prob["nq"], on_lag=lag_done)
    torch.cuda.empty_cache()
    fields = [tested_fields(V, F, E, prob["waves"], prob["dt"], k) for k in checks]
    r = rhs(pre, Tmax, np.concatenate([f[0] for f in fields], axis=1), np.concatenate([f[1] for f in fields], axis=1))
    C1b, C2b = blk(pre["C1"]), blk(pre["C2"])
    errs = {nm: [] for nm in names}
    for nm in names:
        for c, k in enumerate(checks):
            rk = r[:, c * R:(c + 1) * R]
            res = C1b @ Y1[(nm, k)] + C2b @ Y2[(nm, k)] - rk
            errs[nm].append(np.linalg.norm(res) / np.linalg.norm(rk))
            log("%s step %d: ||r_k|| %.3e, ||sum_j Q_j w_(k-j) - r_k|| / ||r_k|| = %.3e"
                % (nm, k, np.linalg.norm(rk), errs[nm][-1]))
    return errs, P, Tmax


def _say(msg):
    print(msg, flush=True)


def test_sphere_15360_64_waves_prefix():
    """The 15,360-unknown sphere with 64 seeded waves (the batched benchmark
    solve) in the configuration the benchmark times (FP64 approximate inverse,
    speculative stepping, autotuned tiles, all 31 lags folded): one device
    assembly pass feeds an FP64 and a mixed solver, each marched 38 steps.
    The first 4 steps against the oracle on the same inputs (Q_0 dense with
    its LU, the later lags as operators; eq. (MOT), eq. (dis_jm)): FP64 to
    1e-10, MOT_MIXED to 1e-6 on w, loop and star.  Then eq. (MOT) with all 31
    lags at steps 31, 34 and 38 (every Q_j applied from a second assembly
    pass): FP64 to 1e-9 of ||r_k||, MOT_MIXED (lags stored in FP32) to 1e-6."""
    import torch
    import paper_2510_07989_amd as p
    from fixture import gpu
    from oracle.mot_oracle import Oracle
    print("case sphere_7680 64 waves: inputs", flush=True)
    prob = gpu.build_problem_device("sphere_7680")
    ne = prob["E"].shape[0]
    assert len(prob["waves"]) == 64
    st = torch.cuda.current_stream().cuda_stream
    ss = [p.Solver(prob["V"], prob["F"], prob["E"], prob["eps_r"], prob["mu_r"], prob["dt"], prob["T0s"],
                   prob["T0h"], prob["G"], prob["waves"], stream=st,
                   options=p.default_options(precond=2, precision=prec, max_steps=C3_STEPS + 8)) for prec in (0, 1)]
    names = {(0, 0): "T_h", (0, 1): "K_h", (1, 0): "T_hat", (1, 1): "K_hat", (2, 0): "T_tilde", (2, 1): "K_tilde"}
    raw = {m: {k: np.zeros((NL_C3, ne, ne)) for k in names.values()} for m in ("ext", "int")}

    def upload(fam, lag, med, op, t):
        for s in ss:
            s.set_lag_device(fam, lag, med, op, t)
        if lag < NL_C3:
            raw[("ext", "int")[med]][names[(fam, op)]][lag] = t.cpu().numpy()

    def progress(i):
        if i % 8 == 0:
            print("lag", i, "uploaded", flush=True)

    gpu.upload_lags(upload, prob["V"], prob["F"], prob["E"], prob["dt"], prob["eps_r"], prob["mu_r"],
                    prob["kmax"], nq=prob["nq"], on_lag=progress)
    assert all(s.info()["folded"] == 1 for s in ss)
    print("march", flush=True)
    outs = [s.run(C3_STEPS) for s in ss]
    for s in ss:
        s.close()
    del ss
    torch.cuda.empty_cache()
    print("oracle", flush=True)
    ref = Oracle(dict(prob, raw=raw), nlag=NL_C3, operators=True,
                 log=lambda stage: print("oracle:", stage, flush=True)).run(NL_C3)
    del raw
    for out, bound, tag in ((outs[0], 1e-10, "fp64"), (outs[1], 1e-6, "mixed")):
        e = [_rel(out[k][:NL_C3], ref[r]) for k, r in (("w", "W"), ("loop", "loop"), ("star", "star"))]
        print("%s prefix errors: w %.3e loop %.3e star %.3e" % (tag, *e), flush=True)
        assert max(e) < bound, (tag, e)
    del ref
    errs, _, _ = _step_equation(prob, {"fp64": outs[0]["w"], "mixed": outs[1]["w"]}, C3_CHECK, _say)
    assert max(errs["fp64"]) < 1e-9, errs["fp64"]
    assert max(errs["mixed"]) < 1e-6, errs["mixed"]


C5_STEPS = 30
C5_CHECK = (9, 12, 16, 20, 25, 30)     # every lag active from step 9; the pulses cross the cube by step 40


def test_cube_30720_16_waves_step_equation():
    """The 30,720-unknown cube with 16 seeded waves (the headline solve) in
    the configuration the benchmark times (FP64 approximate inverse,
    speculative stepping, autotuned tiles, all 9 lags folded), 30 steps on the
    device.  The oracle then checks eq. (MOT) on those unknowns at six steps
    spread over the pulse: sum_j Q_j w_{k-j} = r_k, with every Q_j applied from
    the raw blocks of its lag (a second device assembly pass, lag by lag; the
    oracle's lag_products, C1 and C2 of eq. (CP), the RHS of eq. (rhs)), to
    1e-9 of ||r_k|| (GMRES stops at 1e-13 of its right-hand side); and the
    loop and star parts of every step against eq. (dis_jm) to 1e-10."""
    import torch
    import paper_2510_07989_amd as p
    from fixture import gpu
    from oracle.mot_oracle import recover
    print("case cube_15360 16 waves: inputs", flush=True)
    prob = gpu.build_problem_device("cube_15360")
    V, F, E = prob["V"], prob["F"], prob["E"]
    ne, R, K = E.shape[0], len(prob["waves"]), C5_STEPS
    assert R == 16 and ne == 15360
    st = torch.cuda.current_stream().cuda_stream
    s = p.Solver(V, F, E, prob["eps_r"], prob["mu_r"], prob["dt"], prob["T0s"], prob["T0h"], prob["G"],
                 prob["waves"], stream=st, options=p.default_options(precond=2, max_steps=K + 8))
    t0 = time.perf_counter()
    gpu.load_solvers([s], prob, on_lag=lambda i: print("lag %d folded (%.0f s)" % (i, time.perf_counter() - t0),
                                                      flush=True))
    assert s.info()["folded"] == 1
    print("march", flush=True)
    out = s.run(K)
    s.close()
    del s
    torch.cuda.empty_cache()
    errs, P, Tmax = _step_equation(prob, {"fp64": out["w"]}, C5_CHECK, _say)
    assert max(errs["fp64"]) < 1e-9, errs["fp64"]
    loop, star = recover(P, Tmax, prob["dt"], out["w"])
    for part, ref in (("loop", loop), ("star", star)):
        e = _rel(out[part], ref)
        print("%s part vs eq. (dis_jm): %.3e" % (part, e), flush=True)
        assert e < 1e-10, (part, e)
