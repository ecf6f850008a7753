"""HIP path against the FP64 oracle, through the C ABI (MI355X only)."""
import sys

import numpy as np
import pytest

from tests._problems import problem, oracle

pytestmark = pytest.mark.gpu


def _solver(name, **opts):
    import paper_2510_07989_amd as p
    prob = problem(name)
    o = p.default_options(**opts)
    s = p.Solver(prob["V"], prob["F"], prob["E"], prob["eps_r"], prob["mu_r"], prob["dt"],
                 prob["T0s"], prob["T0h"], prob["G"], prob["waves"], options=o)
    s.load_raw(prob["raw"], prob["kmax"])
    return s


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("name", ["tiny", "tiny_torus", "sphere_480", "tiny_pyramid"])
def test_setup_operators(name):
    print("case", name, flush=True)
    O = oracle(name)
    s = _solver(name)
    inf = s.info()
    assert inf["kmax"] == O.kmax and inf["nlags"] == O.kmax + 2
    assert abs(inf["Tmax"] - O.Tmax) < 1e-12 * O.Tmax
    assert _rel(s.matrix(3), O.P["PS"]) < 1e-11
    assert _rel(s.matrix(4), O.P["BL"]) < 1e-11
    assert _rel(s.matrix(5), O.pre["Ginv"]) < 1e-11
    assert _rel(s.matrix(1), O.pre["C1"]) < 1e-10
    assert _rel(s.matrix(2), O.pre["C2"]) < 1e-10
    for i in range(O.kmax + 2):
        assert _rel(s.matrix(0, i), O.Q[i]) < 1e-10, i
    s.close()


@pytest.mark.parametrize("name", ["tiny", "sphere_480"])
def test_rhs(name):
    print("case", name, flush=True)
    O = oracle(name)
    prob = problem(name)
    s = _solver(name)
    from oracle import mot_oracle as mo
    for k in (1, 5, 17, 40):
        eb, Eb = mo.tested_fields(prob["V"], prob["F"], prob["E"], prob["waves"], prob["dt"], k)
        r = mo.rhs(O.pre, O.Tmax, eb, Eb)
        assert _rel(s.matrix(6, k), r) < 1e-11, k
    s.close()


@pytest.mark.parametrize("name,nsteps", [("tiny", 40), ("tiny_torus", 60), ("sphere_480", 200),
                                          ("tiny_pyramid", 60), ("pyramid_648", 300)])
def test_march_parity(name, nsteps):
    print("case", name, nsteps, flush=True)
    O = oracle(name)
    ref = O.run(nsteps)
    s = _solver(name)
    out = s.run(nsteps)
    assert out["rc"] == 0
    e_w = _rel(out["w"], ref["W"])
    e_l = _rel(out["loop"], ref["loop"])
    e_s = _rel(out["star"], ref["star"])
    print("errors w %.3e loop %.3e star %.3e" % (e_w, e_l, e_s), flush=True)
    assert e_w < 1e-10 and e_l < 1e-10 and e_s < 1e-10
    # e_max: worst step error against the peak
    dw = np.linalg.norm((out["w"] - ref["W"]).reshape(nsteps, -1), axis=1).max()
    assert dw < 1e-10 * np.linalg.norm(ref["W"].reshape(nsteps, -1), axis=1).max()
    s.close()


def test_step_api_matches_run():
    s = _solver("tiny")
    infos = [s.step() for _ in range(10)]
    assert all(i["converged"] for i in infos)
    assert infos[-1]["step"] == 10
    s.reset()
    out = s.run(10)
    s2 = _solver("tiny")
    out2 = s2.run(10)
    assert np.array_equal(out["w"], out2["w"])        # deterministic reductions
    s.close(); s2.close()


def test_reset_after_halted_windows_equals_new_handle():
    """FP32 approximate inverse: speculative windows halt and raise the
    Arnoldi count per step; after mot_reset the march is again bit for bit
    that of a new handle."""
    s = _solver("sphere_480", precond=1)
    s.run(300, w=False, loop=False, star=False)
    s.reset()
    out = s.run(300)
    s2 = _solver("sphere_480", precond=1)
    out2 = s2.run(300)
    for k in ("w", "loop", "star"):
        assert np.array_equal(out[k], out2[k]), k
    assert s.info()["gmres_iters_total"] == s2.info()["gmres_iters_total"]
    s.close(); s2.close()


def test_lag_errors():
    import paper_2510_07989_amd as p
    from paper_2510_07989_amd import _lib as L
    prob = problem("tiny")
    s = p.Solver(prob["V"], prob["F"], prob["E"], prob["eps_r"], prob["mu_r"], prob["dt"],
                 prob["T0s"], prob["T0h"], prob["G"], prob["waves"])
    ne = prob["E"].shape[0]
    z = np.zeros((ne, ne))
    with pytest.raises(p.MotError) as e:
        s.set_lag(L.FAM_TILDE, prob["kmax"], L.MED_EXT, L.OP_T, z)      # beyond k_max - 1
    assert e.value.code == L.MOT_EINVAL
    with pytest.raises(p.MotError) as e:
        s.step()                                                          # lags missing
    assert e.value.code == L.MOT_ESTATE
    s.set_lag(L.FAM_H, 0, L.MED_EXT, L.OP_T, z)
    with pytest.raises(p.MotError) as e:
        s.set_lag(L.FAM_H, 0, L.MED_EXT, L.OP_T, z)                      # twice
    assert e.value.code == L.MOT_ESTATE
    s.close()


@pytest.mark.parametrize("pc", [0, 1, 2])
def test_preconditioner_variants(pc):
    """Unpreconditioned, FP32 and FP64 approximate-inverse right preconditioning
    of the Q_0 GMRES all reach the oracle's solution."""
    print("precond", pc, flush=True)
    O = oracle("sphere_480")
    ref = O.run(120)
    s = _solver("sphere_480", precond=pc)
    out = s.run(120)
    inf = s.info()
    its = inf["gmres_iters_total"] / 120
    print("precond %d: %.2f iterations/step, NS iterations %d, resid %.2e, err %.2e"
          % (pc, its, inf["precond_iters"], inf["precond_resid"], _rel(out["w"], ref["W"])), flush=True)
    assert _rel(out["w"], ref["W"]) < 1e-10
    assert _rel(out["star"], ref["star"]) < 1e-10
    if pc:
        assert its < 6
    s.close()


@pytest.mark.parametrize("name,precond,window,precision", [("sphere_480", 2, 0, 0), ("sphere_480", 1, 0, 0),
                                                           ("sphere_480", 2, 5, 0), ("sphere_480", 1, 3, 0),
                                                           ("sphere_480_r16", 2, 0, 0), ("sphere_480_r16", 2, 7, 1),
                                                           ("tiny_box", 1, 0, 0)])
def test_speculative_stepping_matches_host_driven(name, precond, window, precision):
    """Steps queued without host waits (device halt word, host fallback for a
    step whose solve did not converge in the queued iterations) give the
    host-driven march bit for bit, for one wave and for several (one GMRES per
    column), also across run() calls and windows that straddle RHS batches.
    The FP32 preconditioner needs several iterations, so its first steps
    exercise the halt and the fallback."""
    print("case", name, "precond", precond, "window", window, "precision", precision, flush=True)
    s0 = _solver(name, precond=precond, spec_window=-1, precision=precision)
    ref = s0.run(300)
    it0 = s0.info()["gmres_iters_total"]
    s0.close()
    s = _solver(name, precond=precond, spec_window=window, precision=precision)
    a = s.run(130)
    b = s.run(170)
    it1 = s.info()["gmres_iters_total"]
    s.close()
    print("iterations host-driven %d, speculative %d" % (it0, it1), flush=True)
    assert np.array_equal(np.concatenate([a["w"], b["w"]]), ref["w"])
    # recovery solves per run() call: its CG stops on the call's columns together
    for k in ("loop", "star"):
        assert _rel(np.concatenate([a[k], b[k]]), ref[k]) < 1e-12, k


@pytest.mark.parametrize("opts", [dict(history_order=2), dict(stream_split=2), dict(stream_split=4),
                                  dict(history_order=2, precond=1), dict(history_order=2, stream_split=2),
                                  dict(recovery=1), dict(stream_split=12), dict(stream_split=14),
                                  dict(stream_split=18), dict(stream_split=14, precond=2),
                                  dict(stream_split=18, precond=2), dict(stream_split=14, precond=0),
                                  dict(stream_split=12, precond=2, history_order=1),
                                  dict(stream_split=12, precond=2, history_order=3),
                                  dict(stream_split=14, precond=2, history_order=3),
                                  dict(stream_split=32, precond=2), dict(stream_split=34, precond=2),
                                  dict(stream_split=34, precond=1), dict(stream_split=32, precond=0),
                                  dict(stream_split=11, precond=2), dict(stream_split=11, precond=1)])
def test_kernel_variants(opts):
    """Loop-order and row-split variants of the streaming kernels, and the
    graph-Laplacian CG recovery, give the oracle's march."""
    print("variant", opts, flush=True)
    O = oracle("sphere_480")
    ref = O.run(100)
    s = _solver("sphere_480", **opts)
    out = s.run(100)
    assert _rel(out["w"], ref["W"]) < 1e-10
    assert _rel(out["loop"], ref["loop"]) < 1e-10
    assert _rel(out["star"], ref["star"]) < 1e-10
    s.close()


@pytest.mark.parametrize("name,nsteps,opts", [("tiny", 40, {}), ("sphere_480", 200, dict(precond=2)),
                                               ("sphere_480", 100, dict(precond=0)),
                                               ("tiny_pyramid", 60, dict(precond=2)),
                                               ("pyramid_648_fine", 150, dict(precond=2))])
def test_raw_family_history_parity(name, nsteps, opts):
    """history_form 1 (Sec. V-B without the fold: the media-summed raw families
    of every lag >= 1 applied to the projected unknowns P^{Lambda H} w and
    P^Sigma w, C1 and C2 once per step) marches the oracle's solution, and the
    folded form's up to the order of the sums; Q_0 is folded as before and the
    folded Q_i of later lags do not exist."""
    import paper_2510_07989_amd as p
    print("case raw history", name, nsteps, opts, flush=True)
    O = oracle(name)
    ref = O.run(nsteps)
    f = _solver(name, **opts)
    fo = f.run(nsteps)
    q0 = f.matrix(0, 0)
    f.close()
    s = _solver(name, history_form=1, **opts)
    assert np.array_equal(s.matrix(0, 0), q0)
    with pytest.raises(p.MotError):
        s.matrix(0, 1)
    out = s.run(nsteps)
    assert out["rc"] == 0
    for k, r in (("w", "W"), ("loop", "loop"), ("star", "star")):
        e, ef = _rel(out[k], ref[r]), _rel(out[k], fo[k])
        print("%s: against the oracle %.3e, against the folded lags %.3e" % (k, e, ef), flush=True)
        assert e < 1e-10 and ef < 1e-10, k
    s.close()


@pytest.mark.parametrize("name,nsteps", [("tiny_box", 40), ("sphere_480_r16", 100)])
def test_multi_rhs_parity(name, nsteps):
    """R plane waves marched together (tall-skinny GEMM history and Q_0 products,
    one GMRES per column) against the oracle."""
    print("case", name, flush=True)
    O = oracle(name)
    ref = O.run(nsteps)
    s = _solver(name, precond=2)
    out = s.run(nsteps)
    assert out["rc"] == 0
    e = [_rel(out[k], ref[r]) for k, r in (("w", "W"), ("loop", "loop"), ("star", "star"))]
    print("errors", e, flush=True)
    assert max(e) < 1e-10
    s.close()


def test_multi_rhs_column_equals_alone():
    """Column r of a batched march equals the march of wave r alone."""
    import paper_2510_07989_amd as p
    prob = problem("sphere_480_r16")
    s = _solver("sphere_480_r16", precond=2)
    out = s.run(60)
    s.close()
    for r in (0, 7, 15):
        o = p.default_options(precond=2)
        s1 = p.Solver(prob["V"], prob["F"], prob["E"], prob["eps_r"], prob["mu_r"], prob["dt"],
                      prob["T0s"], prob["T0h"], prob["G"], [prob["waves"][r]], options=o)
        s1.load_raw(prob["raw"], prob["kmax"])
        one = s1.run(60)
        s1.close()
        assert _rel(out["w"][:, :, r], one["w"][:, :, 0]) < 1e-12


def _waves_problem(name, R):
    """The named problem with R seeded plane waves instead of its own."""
    from fixture.problem import CONFIGS, make_waves
    prob = dict(problem(name))
    prob["waves"] = make_waves(R, CONFIGS[name]["sigma"], True)
    return prob


@pytest.mark.parametrize("R,precision,wg", [(24, 0, 0), (40, 0, 0), (40, 1, 0), (40, 0, 4), (40, 0, 8),
                                             (40, 1, 8)])
def test_multi_rhs_wide(R, precision, wg):
    """24 and 40 waves (2 and 4 column blocks of 16, the last partly masked) on
    the 960-unknown sphere, FP64 and mixed, against the oracle; with four
    column blocks also each tile workgroup shape fixed (wg 4, or 8 with the
    history slices prefetched into registers)."""
    import paper_2510_07989_amd as p
    from oracle.mot_oracle import Oracle
    print("case sphere_480 R", R, "precision", precision, "tile_wg", wg, flush=True)
    prob = _waves_problem("sphere_480", R)
    ref = Oracle(prob).run(80)
    s = p.Solver(prob["V"], prob["F"], prob["E"], prob["eps_r"], prob["mu_r"], prob["dt"], prob["T0s"],
                 prob["T0h"], prob["G"], prob["waves"],
                 options=p.default_options(precond=2, precision=precision, tile_wg=wg))
    s.load_raw(prob["raw"], prob["kmax"])
    out = s.run(80)
    s.close()
    e = [_rel(out[k], ref[r]) for k, r in (("w", "W"), ("loop", "loop"), ("star", "star"))]
    print("errors", e, flush=True)
    assert max(e) < (1e-10 if precision == 0 else 1e-6)


@pytest.mark.parametrize("name,nsteps,precision,hilo,group,bound_w,bound_star", [
    ("tiny_box", 60, 1, 2, 4, 1e-6, 1e-6),
    ("sphere_480_r16", 200, 1, 2, 4, 1e-6, 1e-6),
    ("sphere_480_r16", 200, 1, -1, 4, 1e-6, 1e-6),
    ("sphere_480_r16", 200, 2, 2, 4, 1e-6, 3e-5),
    ("sphere_480_r16", 200, 2, 2, 64, 6e-6, 1e-4),
])
def test_mixed_precision(name, nsteps, precision, hilo, group, bound_w, bound_star):
    """FP32 storage of Q_1..Q_{L-1}; Q_0, GMRES, projectors and recovery in FP64.

    Stated bounds, relative L2 over all steps against the FP64 oracle, for the
    currents w and their loop parts, and for the star parts, which are
    (T_max/dt) times a first difference of the unknowns:
      MOT_MIXED (FP64 MFMA products of the FP32-stored entries): w, loop and
        star <= 1e-6 (measured 5e-8 and 1.5e-7 on this sphere);
      MOT_MIXED32 (FP32 MFMA, FP32 sums of 4 indices per half added in FP64):
        w <= 1e-6, star <= 3e-5 on this mesh; 64-index sums are a few times
        less accurate.
    No late-time growth in any case."""
    print("case", name, nsteps, precision, hilo, group, flush=True)
    O = oracle(name)
    ref = O.run(nsteps)
    s = _solver(name, precond=2, precision=precision, hilo_lags=hilo, mix_group=group)
    out = s.run(nsteps)
    e = [_rel(out[k], ref[r]) for k, r in (("w", "W"), ("loop", "loop"), ("star", "star"))]
    print("mixed errors (precision %d, hilo %d, group %d): w %.3e loop %.3e star %.3e"
          % (precision, hilo, group, *e), flush=True)
    assert e[0] < bound_w and e[1] < bound_w and e[2] < bound_star
    nrm = np.linalg.norm(out["w"].reshape(nsteps, -1), axis=1)
    late = np.log10(nrm[-nsteps // 4:] + 1e-300)
    assert np.polyfit(np.arange(late.size), late, 1)[0] <= 0.0     # no late-time growth
    s.close()


def test_mixed_option_errors():
    """Invalid accumulator length and single-RHS mixed precision are refused at create."""
    import paper_2510_07989_amd as p
    prob = problem("tiny_box")
    with pytest.raises(p.MotError):
        _solver("tiny_box", precond=2, precision=2, mix_group=8)
    for prec in (1, 2):
        with pytest.raises(p.MotError):
            p.Solver(prob["V"], prob["F"], prob["E"], prob["eps_r"], prob["mu_r"], prob["dt"], prob["T0s"],
                     prob["T0h"], prob["G"], prob["waves"][:1], options=p.default_options(precision=prec))
    with pytest.raises(p.MotError):
        _solver("tiny_box", precond=2, precision=3)


def test_csr_upload_equals_dense():
    """Lag blocks sent as CSR (mot_set_lag_csr, including an empty block with
    nnz = 0) fold into the same Q_i as the same blocks sent dense, and the two
    marches are identical (Section V-B blocks; eq. (MOT))."""
    import scipy.sparse as sp
    import paper_2510_07989_amd as p
    from paper_2510_07989_amd import _lib as L
    print("case tiny_torus csr", flush=True)
    prob = problem("tiny_torus")
    km = prob["kmax"]
    raw = {m: {k: v.copy() for k, v in prob["raw"][m].items()} for m in ("ext", "int")}
    raw["int"]["K_h"][km] = 0.0                      # one block sent empty through CSR
    def make():
        return p.Solver(prob["V"], prob["F"], prob["E"], prob["eps_r"], prob["mu_r"], prob["dt"], prob["T0s"],
                        prob["T0h"], prob["G"], prob["waves"], options=p.default_options(precond=2))
    dense, csr = make(), make()
    dense.load_raw(raw, km)
    fams = (("h", L.FAM_H, km), ("hat", L.FAM_HAT, km + 1), ("tilde", L.FAM_TILDE, km - 1))
    for lag in range(km + 2):
        for fname, fid, lim in fams:
            if lag > lim:
                continue
            for mname, mid in (("ext", L.MED_EXT), ("int", L.MED_INT)):
                for oname, oid in (("T", L.OP_T), ("K", L.OP_K)):
                    B = raw[mname]["%s_%s" % (oname, fname)][lag]
                    A = sp.csr_matrix(B)
                    if fname == "h" and mname == "int" and oname == "K" and lag == km:
                        assert A.nnz == 0
                    csr.set_lag_csr(fid, lag, mid, oid, A)
    for i in range(km + 2):
        assert np.array_equal(csr.matrix(0, i), dense.matrix(0, i)), i
    a, b = dense.run(40), csr.run(40)
    for k in ("w", "loop", "star"):
        assert np.array_equal(a[k], b[k]), k
    dense.close()
    csr.close()
