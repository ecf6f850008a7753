#!/usr/bin/env python3
"""MOT throughput on one MI355X: steps/s of the qHP TD-PMCHWT march.

Headline workload (the largest single solve): unit cube, 32 x 32 x 24 cells,
10,240 triangles / 15,360 edges -> 30,720 unknowns, eps_r = 4, mu_r = 1,
dt = 0.5 (k_max 7, 9 lag matrices), 16 seeded Gaussian plane waves marched
together, plain FP64.  A step is the whole hot path: tested incident fields,
preconditioned RHS, history convolution over Q_1..Q_8, GMRES on Q_0 (FP64
approximate inverse as right preconditioner), ring update, and the loop/star
current recovery of the timed steps into device buffers.  The inputs (static
blocks and the retarded blocks of both media, lag by lag) are assembled on
the device and folded before the timed region.

`batched` compares, on the 5120-triangle sphere (15,360 unknowns, eps_r = 2,
dt = 0.1, 31 lag matrices) with 64 seeded waves: plain FP64 against the mixed
path (FP32-stored lags with an FP32 low part on the first two, FP64 products;
Q_0, GMRES, projectors and recovery FP64), with the recovery inside the timed
region, and the mixed error against the FP64 run.

`torus` marches the 2048-triangle torus (6144 unknowns, dt = 2, one wave) for
10,000 steps: steps/s of the one-RHS path and its late-time behaviour.

Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}
WORKLOADS = {
    "cube_15360": "unit cube 32x32x24 cells, 10240 triangles / 15360 edges -> 30720 unknowns, eps_r=4, mu_r=1, "
                  "dt=0.5 (k_max 7, 9 lags), 16 seeded Gaussian plane waves marched together",
    "sphere_7680": "sphere r=1, 5120 triangles / 7680 edges -> 15360 unknowns, eps_r=2, mu_r=1, dt=0.1 "
                   "(k_max 29, 31 lags), 64 seeded Gaussian plane waves marched together",
    "torus_3072": "torus R=1 r=0.4, 2048 triangles / 3072 edges -> 6144 unknowns, eps_r=4, mu_r=1, "
                  "dt=2.0, 1 Gaussian plane wave",
}
PRECISION = {0: "fp64", 1: "mixed: fp32-stored lags, fp64 mfma products",
             2: "mixed32: fp32-stored lags, fp32 mfma products"}
# committed PMC summary of the dominant kernels (HBM bytes per dispatch)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        n = [d.get("num_threads", 1) for d in info if d.get("user_api") == "blas"]
        return max(n) if n else 1
    except Exception:
        return os.cpu_count() or 1


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def blas_name():
    try:
        from threadpoolctl import threadpool_info
        for d in threadpool_info():
            if d.get("user_api") == "blas":
                return "%s %s (%s)" % (d.get("internal_api", "?"), d.get("version", "?"), d.get("architecture", "?"))
    except Exception:
        pass
    return "unknown"


def source_digest(rel):
    try:
        with open(os.path.join(ROOT, rel), "rb") as f:
            return hashlib.sha256(f.read()).hexdigest()[:16]
    except OSError:
        return None


def measured_traffic(kernel, workload):
    """HBM bytes per dispatch from the committed counter runs, if they were taken
    on the same workload and the kernel's source file is unchanged since; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    for e in t.get("kernels", []):
        if (e.get("kernel") == kernel and e.get("workload") == workload
                and e.get("source_sha256_16") == source_digest(e.get("source", ""))):
            return e.get("bytes_per_dispatch")
    return None


def cpu_baseline(n, R, L, budget_s, seed=251007989):
    """The oracle's march (eq. (MOT), oracle.mot_oracle.march as it stands) on
    a bounded sample of the workload's shape: n unknowns, R waves, L - 1
    history lags, every timed step with the whole history active (resumed
    from L - 1 earlier steps), the Q_0 solve through a given LU factorization.
    The matrices are synthetic (one n x n array serves every history lag,
    a unit triangular pair the LU): the dense products and triangular solves
    cost what they cost on the real values, without the O(n^3) setup (fold
    of the lag matrices, LU of Q_0) that a bench run cannot afford on the
    host."""
    import numpy as np
    from oracle.mot_oracle import march
    rng = np.random.Generator(np.random.PCG64(seed))
    t = time.perf_counter()
    Qh = np.full((n, n), 1e-4)
    lu = np.full((n, n), 1e-6)
    np.fill_diagonal(lu, 1.0)
    piv = np.arange(n, dtype=np.int32)
    Q = [None] + [Qh] * (L - 1)
    W0 = rng.standard_normal((L - 1, n, R))
    prep = time.perf_counter() - t
    t = time.perf_counter()
    march(Q, rng.standard_normal((1, n, R)), lu=(lu, piv), W0=W0)
    one = time.perf_counter() - t
    ns = int(max(2, min(200, budget_s / max(one, 1e-6))))
    r = rng.standard_normal((ns, n, R))
    t = time.perf_counter()
    march(Q, r, lu=(lu, piv), W0=W0)
    el = time.perf_counter() - t
    return dict(steps=ns, seconds=el, prep_s=prep)


def history_model(ne, n, L, R, precision, hilo):
    """Algorithmic bytes and flops of one history launch (all lags of one step):
    the (L-1) lag matrices, 3 ne^2 stored entries each ([[q1, -qk], [qk, q2]]),
    at 8 B (FP64) or 4 B (FP32, plus 4 B on the lags with a low part); the L-1
    ring vectors and the RHS slice read once, the result written once.
    flops: 4 ne^2 products per lag and column (qk acts twice), 2 flops each;
    the split hi/lo FP32 products triple them on the low-part lags."""
    ent = 3.0 * ne * ne
    nl = L - 1
    lo = min(max(hilo, 0), nl) if precision else 0
    qbytes = ent * nl * 8.0 if precision == 0 else ent * (nl + lo) * 4.0
    vbytes = 8.0 * (nl * n * R + 2 * n * R)
    flops = 2.0 * 4 * ne * ne * R * (nl + (2 * lo if precision == 2 else 0))
    return qbytes + vbytes, flops


def roofline(kernel, nbytes, flops, us, dtype, mfma, traffic):
    """Bound by the larger of bytes/HBM peak and flops/MFMA peak (MFMA kernels)."""
    t = us * 1e-6
    t_hbm = nbytes / (HBM_PEAK_GBS * 1e9)
    t_mma = flops / (MFMA_PEAK_TFLOPS[dtype] * 1e12) if mfma else 0.0
    if t_mma > t_hbm:
        ach = flops / t / 1e12
        return {"bound": "mfma", "kernel": kernel, "achieved": round(ach, 2), "peak": MFMA_PEAK_TFLOPS[dtype],
                "unit": "TFLOP/s", "frac": round(ach / MFMA_PEAK_TFLOPS[dtype], 4), "traffic": traffic,
                "flops_per_launch": flops, "bytes_per_launch": nbytes, "avg_launch_us": round(us, 2),
                "hbm_gbs": round(nbytes / t / 1e9, 1)}
    ach = nbytes / t / 1e9
    return {"bound": "hbm", "kernel": kernel, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic, "bytes_per_launch": nbytes,
            "avg_launch_us": round(us, 2)}


def col_blocks(R):
    rp = 1 if R == 1 else max(4, 1 << (R - 1).bit_length())
    return min(4, (rp + 15) // 16)


def history_kernel_name(R, precision, mix_group, sched_hist=11, wg=4):
    if R == 1:
        if sched_hist in (11, 22, 24):
            return "k_history_co"
        return "k_history_rows<%d>" % (sched_hist % 10) if sched_hist > 10 else "k_history"
    if precision == 2:
        fl = {64: 16, 16: 4}.get(mix_group, 1)
        return "k_hist_mfma<%d, %d>" % (col_blocks(R), fl)
    return "k_tile_gemm<%s, %d, %d>" % ("double" if precision == 0 else "float", col_blocks(R), wg)


# HIP events bracket every PROFILE_EVERY-th history and Q_0 launch of the timed
# region: an event marker drains the queue, so bracketing every launch would
# slow the march it measures (torus: 3600 instead of 3770 steps/s)
PROFILE_EVERY = 16


def late_time(s, nsteps):
    """Sec. VI-A on the whole kept march: ||w_k|| of every step from the
    device (mot_step_norms); the least-squares slope of log10 ||w_k|| over the
    last min(2000, nsteps/5) steps and the last norm against the peak."""
    import numpy as np
    nr = s.step_norms(0, nsteps)[:, 0]
    m = min(2000, nsteps // 5)
    tail = np.log10(nr[-m:] + 1e-300)
    slope = float(np.polyfit(np.arange(m), tail, 1)[0])
    out = {"steps": nsteps, "window": m, "log10_slope_per_step": slope,
           "last_over_peak": float(nr[-1] / nr.max()), "peak_step": int(np.argmax(nr)) + 1}
    log("late time: %d steps, log10 ||w|| slope %.3e per step over the last %d, last / peak %.2e"
        % (nsteps, slope, m, out["last_over_peak"]))
    return out


def far_field_timing(s, nsteps, n, R, freq):
    """mot_far_field over every kept step of a march: the spectra of the loop
    and star currents at freq and the far field in 181 directions of one
    plane.  Timed on the host around the (synchronous) call; the streaming
    pass over the kept unknowns is its dominant kernel."""
    import numpy as np
    th = np.radians(np.arange(181.0))
    dirs = np.stack([np.sin(th), np.zeros_like(th), np.cos(th)], 1)
    s.far_field(0, min(nsteps, 64), freq, dirs)                 # first call: code objects, pool
    t = time.perf_counter()
    r = s.far_field(0, nsteps, freq, dirs)
    el = time.perf_counter() - t
    nbytes = 8.0 * nsteps * n * R
    mag = np.abs(r["field"]).max(axis=(0, 1, 3))
    log("far field: %d steps, %d directions at f = %g: %.3f ms per call (scratch allocation, kernels, copies to "
        "the host); largest loop / star field %.3e / %.3e" % (nsteps, len(dirs), freq, 1e3 * el, mag[0], mag[1]))
    return {"steps": nsteps, "freq": freq, "directions": len(dirs), "call_ms": round(1e3 * el, 3),
            "spectrum_pass_bytes": nbytes, "max_field_loop": float(mag[0]), "max_field_star": float(mag[1]),
            "note": "host wall time of the whole call; per-kernel times in the rocprofv3 summary"}


def make_solvers(mot, prob, variants, max_steps):
    """One solver per variant (dict of options), all fed by one device
    assembly pass of the problem's retarded blocks; returns the solvers and
    the wall times of create and of assembly + fold (+ preconditioner)."""
    import torch
    from fixture import gpu as fxgpu
    t = time.perf_counter()
    ss = []
    for v in variants:
        kw = dict(profile=PROFILE_EVERY, max_steps=max_steps)
        kw.update(v)
        waves = kw.pop("waves", prob["waves"])          # a variant may march a subset of the waves
        opts = mot.default_options(**kw)
        ss.append(mot.Solver(prob["V"], prob["F"], prob["E"], prob["eps_r"], prob["mu_r"], prob["dt"],
                             prob["T0s"], prob["T0h"], prob["G"], waves, options=opts,
                             stream=torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t
    t = time.perf_counter()
    nl = prob["kmax"] + 2
    fxgpu.load_solvers(ss, prob, on_lag=lambda i: log("  lag %d of %d assembled and folded (%.1f s)"
                                                      % (i, nl - 1, time.perf_counter() - t)))
    torch.cuda.synchronize()
    t_load = time.perf_counter() - t
    return ss, t_create, t_load


def timed(s, prob, name, precision, K, W_, hilo, mix_group, outputs=True, keep_warm=True):
    """W_ warm-up steps (outputs to the host when keep_warm), then K timed
    steps with device-resident outputs (recovery included when outputs)."""
    import torch
    R = len(prob["waves"])
    inf0 = s.info()
    warm = s.run(W_, w=keep_warm, loop=keep_warm, star=keep_warm, device=False)
    torch.cuda.synchronize()
    a = s.info()
    t0 = time.perf_counter()
    s.run(K, w=outputs, loop=outputs, star=outputs, device=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    b = s.info()
    ne, n, L = prob["E"].shape[0], 2 * prob["E"].shape[0], b["nlags"]
    hist_us = 1e3 * (b["hist_ms"] - a["hist_ms"]) / max(1, b["hist_launches"] - a["hist_launches"])
    q0_us = 1e3 * (b["q0_ms"] - a["q0_ms"]) / max(1, b["q0_launches"] - a["q0_launches"])
    hb, hf = history_model(ne, n, L, R, precision, hilo)
    kname = history_kernel_name(R, precision, mix_group, inf0["sched_hist"], inf0["hist_wg"])
    dtype = "f32" if precision == 2 else "f64"
    hist = roofline(kname, hb, hf, hist_us, dtype, R > 1, measured_traffic(kname, name))
    q0b = 8.0 * (3 * ne * ne + 2 * n * R)
    sq = inf0["sched_q0"]
    q0name = (("k_q0_rows<%d>" % (sq % 10) if sq > 10 else "k_q0_matvec") if R == 1
              else "k_tile_gemm<double, %d, %d>" % (col_blocks(R), inf0["q0_wg"]))
    q0 = roofline(q0name, q0b, 2.0 * 4 * ne * ne * R, q0_us, "f64", R > 1,
                  measured_traffic(q0name if R == 1 else q0name + " (Q_0)", name))
    hist_tot = b["hist_ms"] - a["hist_ms"]
    q0_tot = b["q0_ms"] - a["q0_ms"]
    out = dict(steps_s=K / el, el=el, K=K, W=W_, R=R, n=n, L=L, kmax=b["kmax"],
               iters=(b["gmres_iters_total"] - a["gmres_iters_total"]) / K,
               q0_launches=PROFILE_EVERY * (b["q0_launches"] - a["q0_launches"]) / K, hist=hist, q0=q0,
               dominant=hist if hist_tot >= q0_tot else q0, warm=warm, recover_ms=b["recover_ms"],
               device_gb=inf0["device_bytes"] / 1e9, setup_ms=inf0["setup_ms"], fold_ms=inf0["fold_ms"],
               precond_iters=inf0["precond_iters"], precond_resid=inf0["precond_resid"],
               schedule={"history": inf0["sched_hist"], "q0": inf0["sched_q0"], "precond": inf0["sched_pc"],
                         "history_wg": inf0["hist_wg"], "q0_wg": inf0["q0_wg"],
                         "autotuned": bool(inf0["tuned"]), "tune_ms": round(inf0["tune_ms"], 1)})
    log("[%s R=%d %s] timed %d steps in %.3f s: %.2f steps/s (%.1f RHS-steps/s), %.2f GMRES its/step; "
        "history %.1f us (%s %.4g %s, %.3f of peak), Q0 product %.1f us; %.1f GB on device"
        % (name, R, PRECISION[precision], K, el, K / el, R * K / el, out["iters"], hist_us, hist["bound"],
           hist["achieved"], hist["unit"], hist["frac"], q0_us, out["device_gb"]))
    return out


def brief(r):
    return {"steps_s": round(r["steps_s"], 3), "rhs_steps_per_s": round(r["steps_s"] * r["R"], 1),
            "ms_per_step": round(1e3 * r["el"] / r["K"], 4), "gmres_iters_per_step": round(r["iters"], 2),
            "history_kernel": r["hist"], "q0_product": r["q0"], "schedule": r["schedule"],
            "device_gb": round(r["device_gb"], 2)}


def rel(a, b):
    import numpy as np
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def torus_leg(mot, args):
    """The torus, one wave, FP64, 10,000 timed steps after 100: the one-RHS
    step rate, its late-time behaviour over the whole march and the far field
    of every kept step; then the same march replayed from captured graphs."""
    import torch
    from fixture import gpu as fxgpu
    name = "torus_3072"
    t = time.perf_counter()
    prob = fxgpu.build_problem_device(name)
    t_in = time.perf_counter() - t
    W_, K = 100, 10000
    (s,), t_create, t_load = make_solvers(mot, prob, [dict(precond=args.precond)], W_ + K + 8)
    log("[%s] inputs %.1f s, create %.1f s, device assembly and fold %.1f s" % (name, t_in, t_create, t_load))
    m = timed(s, prob, name, 0, K, W_, args.hilo, args.mix_group, keep_warm=False)
    out = dict(brief(m), workload=name + ": " + WORKLOADS[name], steps=K, warmup=W_,
               setup_s=round(t_create + t_load, 2))
    try:
        out["late_time"] = late_time(s, W_ + K)
        out["far_field"] = far_field_timing(s, W_ + K, m["n"], 1, FAR_FIELD_FREQ[name])
    except Exception as e:  # noqa: BLE001
        log("late-time / far-field diagnostics failed: %r" % (e,))
    s.close()
    if not args.no_graph:
        gr = {}
        for g in (0, 1):
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                (sg,), _, _ = make_solvers(mot, prob, [dict(precond=args.precond, graph=g, profile=0)], 5200)
                sg.run(100, w=False, loop=False, star=False, device=True)
                st.synchronize()
                t0 = time.perf_counter()
                sg.run(5000, w=True, loop=True, star=True, device=True)
                st.synchronize()
                el = time.perf_counter() - t0
            gr["graph" if g else "launches"] = {"steps_s": round(5000 / el, 1),
                                                "graph_windows": sg.info()["graph_windows"]}
            sg.close()
        out["graph_replay"] = dict(gr, steps=5000)
        log("window replay: launches %.1f steps/s, graphs %.1f steps/s" % (gr["launches"]["steps_s"],
                                                                          gr["graph"]["steps_s"]))
    return out


def batched_leg(mot, args):
    """The 15,360-unknown sphere with 64 seeded waves: FP64 against the mixed
    path (and, with --mixed32, the FP32 matrix-core path) on the same device
    assembly, recovery inside the timed region; the mixed error against the
    FP64 run over the warm-up steps; and the plain FP64 march of the first wave
    alone (one RHS), the single-excitation rate the batched solves are
    compared with."""
    import numpy as np
    import torch
    from fixture import gpu as fxgpu
    name = "sphere_7680"
    t = time.perf_counter()
    prob = fxgpu.build_problem_device(name)
    t_in = time.perf_counter() - t
    Kb, Wb = args.batched_steps, args.batched_warmup
    variants = [(0, dict(precond=args.precond, precision=0)),
                (1, dict(precond=args.precond, precision=1, hilo_lags=args.hilo))]
    if args.mixed32:
        variants.append((2, dict(precond=args.precond, precision=2, hilo_lags=args.hilo, mix_group=args.mix_group)))
    if not args.no_single_rhs:
        variants.append(("1rhs", dict(precond=args.precond, precision=0, waves=prob["waves"][:1])))
    ss, t_create, t_load = make_solvers(mot, prob, [v for _, v in variants], Wb + Kb + 8)
    log("[%s] inputs %.1f s, create %.1f s, device assembly and fold of %d solvers %.1f s"
        % (name, t_in, t_create, len(ss), t_load))
    res = {}
    for (prec, v), s in zip(variants, ss):
        p_ = dict(prob, waves=v["waves"]) if "waves" in v else prob
        res[prec] = timed(s, p_, name, v["precision"], Kb, Wb, args.hilo, args.mix_group)
        s.close()
    torch.cuda.empty_cache()
    ref = res[0]["warm"]
    out = {"workload": name + ": " + WORKLOADS[name], "steps": Kb, "warmup": Wb,
           "setup_s": round(t_create + t_load, 2), "fp64_64rhs": brief(res[0])}
    if "1rhs" in res:
        one = res["1rhs"]
        out["fp64_1rhs"] = brief(one)
        for prec, key in ((0, "fp64_64rhs"), (1, "mixed_64rhs")):
            if prec in res:
                r = res[prec]
                out.setdefault("vs_fp64_1rhs", {})[key] = {
                    "steps_ratio": round(r["steps_s"] / one["steps_s"], 3),
                    "rhs_steps_ratio": round(r["steps_s"] * r["R"] / one["steps_s"], 2)}
        log("[%s] plain FP64, one wave: %.1f steps/s; 64 waves mixed: %.1f steps/s = %.0f RHS-steps/s (x%.1f)"
            % (name, one["steps_s"], res[1]["steps_s"] if 1 in res else float("nan"),
               res[1]["steps_s"] * 64 if 1 in res else float("nan"),
               res[1]["steps_s"] * 64 / one["steps_s"] if 1 in res else float("nan")))
    for prec, key in ((1, "mixed_64rhs"), (2, "mixed32_64rhs")):
        if prec not in res:
            continue
        e = {k: rel(res[prec]["warm"][k], ref[k]) for k in ("w", "loop", "star")}
        nrm = np.linalg.norm(res[prec]["warm"]["w"].reshape(Wb, -1), axis=1)
        out[key] = dict(brief(res[prec]), precision=PRECISION[prec], hilo_lags=args.hilo,
                        err_vs_fp64={"steps": Wb, **e},
                        speedup_vs_fp64=round(res[prec]["steps_s"] / res[0]["steps_s"], 3))
        log("[%s] %s: %.2f steps/s against FP64 %.2f (x%.3f); error vs FP64 over %d steps: w %.2e loop %.2e "
            "star %.2e" % (name, PRECISION[prec], res[prec]["steps_s"], res[0]["steps_s"],
                           res[prec]["steps_s"] / res[0]["steps_s"], Wb, e["w"], e["loop"], e["star"]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-headline", action="store_true", help="skip the headline solve (profiling the other legs)")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-wave sphere comparison")
    ap.add_argument("--batched-steps", type=int, default=200)
    ap.add_argument("--batched-warmup", type=int, default=40)
    ap.add_argument("--mixed32", action="store_true", help="also time the FP32 matrix-core mixed path")
    ap.add_argument("--no-single-rhs", action="store_true",
                    help="skip the one-wave FP64 march of the 64-wave sphere's mesh")
    ap.add_argument("--no-torus", action="store_true", help="skip the 10,000-step torus march")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay comparison")
    ap.add_argument("--serving", action="store_true",
                    help="also measure continuous batching of a request stream (not run by default)")
    ap.add_argument("--serving-requests", type=int, default=32)
    ap.add_argument("--no-serving-smoke", action="store_true",
                    help="skip the time-boxed 32-request smoke stream (thread-per-solve server)")
    ap.add_argument("--serving-smoke-requests", type=int, default=32)
    ap.add_argument("--serving-smoke-box", type=float, default=60.0, help="seconds before the smoke stream is cut")
    ap.add_argument("--no-serving-c4", action="store_true", help="leave the stream out (the default)")
    ap.add_argument("--serving-c4", action="store_true",
                    help="also serve the time-boxed 256-request stream (batch server; off by default while a stall "
                         "of the batch server with eight concurrent setups is unexplained)")
    ap.add_argument("--serving-c4-requests", type=int, default=256)
    ap.add_argument("--serving-c4-box", type=float, default=120.0, help="seconds before the stream is cut")
    ap.add_argument("--serving-c4-budget-gb", type=float, default=200.0)
    ap.add_argument("--no-step-batch", action="store_true", help="skip the mot_run_batch comparison")
    ap.add_argument("--raw-history", action="store_true",
                    help="also time the history from the raw families (history_form 1) against the folded lags")
    ap.add_argument("--precond", type=int, default=2, help="0 none, 1 FP32, 2 FP64 approximate inverse")
    ap.add_argument("--hilo", type=int, default=2, help="mixed: lags with an FP32 low part (-1: none)")
    ap.add_argument("--mix-group", type=int, default=4, help="precision 2: summation indices per FP32 sum")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the MOT march of one problem runs on one device; "
              "runs on several GPUs are not part of this benchmark.", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    import paper_2510_07989_amd as mot
    from fixture import gpu as fxgpu

    name = "cube_15360"
    W_, K = args.warmup, args.steps
    if args.no_headline:
        result = {"metric": "MOT steps/s (plain FP64, 16 RHS)", "value": None, "unit": "steps/s",
                  "note": "headline solve skipped (--no-headline: a profiling run of the other legs)"}
        run_legs(mot, args, result)
        return
    t = time.perf_counter()
    prob = fxgpu.build_problem_device(name)
    t_in = time.perf_counter() - t
    (s,), t_create, t_load = make_solvers(mot, prob, [dict(precond=args.precond)], W_ + K + 8)
    log("[%s] inputs (mesh, BC basis, Gram, static blocks on the device) %.1f s, create %.1f s, device assembly "
        "and fold %.1f s" % (name, t_in, t_create, t_load))
    m = timed(s, prob, name, 0, K, W_, args.hilo, args.mix_group, keep_warm=False)
    s.close()
    torch.cuda.empty_cache()
    R = m["R"]
    result = {
        "metric": "MOT steps/s (plain FP64, %d RHS)" % R,
        "value": round(m["steps_s"], 3),
        "unit": "steps/s",
        "rhs_steps_per_s": round(m["steps_s"] * R, 2),
        "n_gpus": 1,
        "steps": K,
        "warmup": W_,
        "ms_per_step": round(1e3 * m["el"] / K, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": name + ": " + WORKLOADS[name], "nrhs": R, "unknowns": m["n"], "lags": m["L"],
                   "kmax": m["kmax"], "precision": PRECISION[0],
                   "q0_preconditioner": ["none", "fp32 approximate inverse", "fp64 approximate inverse"][args.precond]},
        "roofline": m["dominant"],
        "history_kernel": m["hist"],
        "q0_product": dict(m["q0"], launches_per_step=round(m["q0_launches"], 2)),
        "gmres_iters_per_step": round(m["iters"], 2),
        "schedule": m["schedule"],
        "setup_s": {"inputs": round(t_in, 1), "create": round(t_create, 1), "assembly_and_fold": round(t_load, 1),
                    "fold_ms": round(m["fold_ms"], 1), "preconditioner_ms": round(m["setup_ms"], 1),
                    "newton_schulz_iters": m["precond_iters"],
                    "newton_schulz_resid": float("%.3e" % m["precond_resid"])},
        "device_gb": round(m["device_gb"], 2),
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline(m["n"], R, m["L"], args.cpu_budget)
        result["cpu_baseline"] = {
            "value": round(cb["steps"] / cb["seconds"], 4), "unit": "steps/s", "cores": blas_threads(),
            "kind": "oracle", "cpu": cpu_model(), "blas": blas_name(),
            "sample": "%d steps of the oracle's march (eq. MOT) at this workload's shape: %d unknowns, %d waves, "
                      "%d history lags all active, Q_0 solved through a given LU factorization; synthetic matrix "
                      "values (one array for every lag); the oracle's O(n^3) setup (lag fold, LU of Q_0) is not "
                      "run" % (cb["steps"], m["n"], R, m["L"] - 1)}
        log("oracle march: %d steps in %.1f s on %d threads" % (cb["steps"], cb["seconds"], blas_threads()))
    run_legs(mot, args, result)


def run_legs(mot, args, result):
    """The legs after the headline solve; prints the JSON line."""
    if not args.no_batched:
        result["batched"] = batched_leg(mot, args)
    if not args.no_torus:
        result["torus"] = torus_leg(mot, args)
    if not args.no_step_batch:
        result["step_batch"] = step_batch(mot)
    if args.raw_history:
        result["raw_history"] = raw_history_leg(mot, args)
    if not args.no_serving_smoke:
        result["serving_smoke"] = guarded(lambda: serving_smoke(args), args.serving_smoke_box + 150.0, result,
                                          "serving_smoke")
    if args.serving_c4 and not args.no_serving_c4:
        try:
            result["serving_c4"] = serving_c4(args)
        except Exception as e:          # the headline line is printed whatever this leg does
            log("[c4] serving stream failed: %s: %s" % (type(e).__name__, e))
            result["serving_c4"] = {"error": "%s: %s" % (type(e).__name__, e)}
    if args.serving:
        result["serving"] = serving(args.serving_requests)
    print(json.dumps(result), flush=True)


def raw_history_bytes(ne, kmax):
    """Algorithmic bytes of one step's history: folded, the three blocks of
    every Q_i, i >= 1; raw, the three blocks of each family present at lag i
    (h to k_max, hat to k_max + 1, tilde to k_max - 1) plus P^Sigma, C1, C2."""
    blk = 8.0 * ne * ne
    fam = sum((i <= kmax) + (i <= kmax + 1) + (i <= kmax - 1) for i in range(1, kmax + 2))
    return 3 * blk * (kmax + 1), 3 * blk * fam + 3 * blk


def raw_history_leg(mot, args, K=1000, W_=20):
    """One wave, FP64: the folded lags (speculative windows, and host-driven
    steps like the raw form) against the raw media-summed families of each lag
    with C1, C2 and the projector applied once per step, on the 3840-unknown
    sphere, the torus and the star pyramid at c dt / D = 0.1 (5184 unknowns,
    k_max 23).  Steps/s, the history's time per step and its algorithmic
    bytes."""
    import torch
    from fixture import gpu as fxgpu
    out = {}
    for name in ("sphere_1920_r16", "torus_3072", "pyramid_2592_fine"):
        prob = fxgpu.build_problem_device(name)
        one = prob["waves"][:1]
        keys = ("folded", "folded_host_driven", "raw")
        variants = [dict(precond=args.precond, waves=one), dict(precond=args.precond, waves=one, spec_window=-1),
                    dict(precond=args.precond, waves=one, history_form=1)]
        ss, t_create, t_load = make_solvers(mot, prob, variants, W_ + K + 8)
        ne, kmax = prob["E"].shape[0], prob["kmax"]
        fb, rb_ = raw_history_bytes(ne, kmax)
        res = {"unknowns": 2 * ne, "kmax": kmax, "setup_s": round(t_create + t_load, 2)}
        ws = []
        for key, s in zip(keys, ss):
            ws.append(s.run(W_, loop=False, star=False)["w"])
            a = s.info()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.run(K, w=False, loop=False, star=False, device=True)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            b = s.info()
            us = 1e3 * (b["hist_ms"] - a["hist_ms"]) / max(1, b["hist_launches"] - a["hist_launches"])
            nb = rb_ if key == "raw" else fb
            res[key] = {"steps_s": round(K / el, 1), "history_us": round(us, 2),
                        "history_bytes": int(nb), "history_gb_s": round(nb / us / 1e3, 1) if us > 0 else None,
                        "device_gb": round(b["device_bytes"] / 1e9, 3)}
            s.close()
        res["raw_vs_folded"] = {"bytes": round(rb_ / fb, 3),
                                "history_time": round(res["raw"]["history_us"] / res["folded_host_driven"]["history_us"], 3),
                                "steps": round(res["raw"]["steps_s"] / res["folded"]["steps_s"], 3)}
        res["warmup_rel_diff_raw_vs_folded"] = rel(ws[2], ws[0])
        torch.cuda.empty_cache()
        log("[%s raw history] folded %.1f steps/s (host-driven %.1f), raw %.1f; history %.1f / %.1f us; bytes x%.2f"
            % (name, res["folded"]["steps_s"], res["folded_host_driven"]["steps_s"], res["raw"]["steps_s"],
               res["folded_host_driven"]["history_us"], res["raw"]["history_us"], rb_ / fb))
        out[name] = res
    out["steps"], out["warmup"] = K, W_
    return out


# a frequency inside the incident pulse's band (sigma = 8 on the torus: up to ~1/(2 pi sigma))
FAR_FIELD_FREQ = {"torus_3072": 0.01}

SERVING_MESHES = ["tiny_torus", "tiny_box", "sphere_480", "sphere_480_r16", "sphere_1920_r16", "torus_3072"]


def step_batch(mot, nsteps=1024, copies=4):
    """Several small solves on one GPU, each on its own stream: marched one
    after another with mot_run, then together with mot_run_batch (windows of
    all solves queued before the host waits on any).  Same kernels, same
    results; the aggregate step rate shows what interleaving recovers on
    meshes too small to fill the device."""
    import numpy as np
    import torch
    from fixture.problem import build_problem
    meshes = ["tiny_torus", "sphere_480"]
    t = time.perf_counter()
    probs = {m: build_problem(m, nsteps=nsteps) for m in meshes}
    log("step-batch inputs assembled in %.1f s" % (time.perf_counter() - t))

    def make():
        out = []
        for m in meshes:
            p = probs[m]
            for _ in range(copies):
                st = torch.cuda.Stream()
                s = mot.Solver(p["V"], p["F"], p["E"], p["eps_r"], p["mu_r"], p["dt"], p["T0s"], p["T0h"],
                               p["G"], p["waves"], options=mot.default_options(precond=2, keep_history=1,
                                                                              max_steps=2 * nsteps + 64),
                               stream=st.cuda_stream)
                s.load_raw(p["raw"], p["kmax"])
                s._keep_stream = st
                out.append(s)
        return out

    res = {"meshes": ["%d x %s" % (copies, m) for m in meshes], "steps_per_solve": nsteps}
    ss = make()
    for s in ss:                                   # warm-up: one window each, alone
        s.run(128, w=False, loop=False, star=False)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for s in ss:
        s.run(nsteps, w=False, loop=False, star=False)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t
    ref = [s.steps(128, nsteps, loop=False, star=False)["w"] for s in ss]
    for s in ss:
        s.close()
    ss = make()
    mot.run_batch(ss, 128)
    torch.cuda.synchronize()
    t = time.perf_counter()
    mot.run_batch(ss, nsteps)
    torch.cuda.synchronize()
    t_bat = time.perf_counter() - t
    same = all(np.array_equal(s.steps(128, nsteps, loop=False, star=False)["w"], r) for s, r in zip(ss, ref))
    for s in ss:
        s.close()
    tot = nsteps * len(ss)
    res.update({"one_after_another_steps_per_s": round(tot / t_seq, 1), "batched_steps_per_s": round(tot / t_bat, 1),
                "speedup": round(t_seq / t_bat, 3), "bitwise_equal": bool(same)})
    log("step batch: %d solves x %d steps: one after another %.1f steps/s, mot_run_batch %.1f steps/s (x%.2f), "
        "identical %s" % (len(ss), nsteps, tot / t_seq, tot / t_bat, t_seq / t_bat, same))
    return res


def c4_requests(nreq, seed=251007991, rate=2.0):
    """The serving stream: nreq seeded requests with Poisson arrivals (rate per
    second), each a random sphere, torus or cube whose unknown count is drawn
    log-uniformly from 500 to 20,000, eps_r uniform in [1.5, 6], mu_r = 1,
    c dt = D / 4 (so k_max = ceil(4 sqrt(eps_r)), 5 to 10), 1 to 32 seeded
    plane waves (sigma = 4 dt), 500 to 5,000 steps.  The mesh is built here;
    the BC basis, Gram matrix, static blocks and every retarded block are
    built in the request's setup (the last two on the device), so setup time
    counts in its end-to-end latency."""
    import math
    import numpy as np
    from fixture import gpu as fxgpu
    from fixture import geometry as geo
    from fixture.problem import make_mesh, make_waves, tmax_kmax
    rng = np.random.Generator(np.random.PCG64(seed))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, nreq))
    out = []
    for i in range(nreq):
        kind = ("sphere", "torus", "cube")[int(rng.integers(3))]
        n_target = math.exp(rng.uniform(math.log(500), math.log(20000)))
        if kind == "sphere":                      # 60 nu^2 unknowns
            spec = ("icosphere", max(3, int(round(math.sqrt(n_target / 60)))))
        elif kind == "torus":                     # 6 nmaj nmin unknowns, nmaj = 4 nmin
            nmin = max(3, int(round(math.sqrt(n_target / 24))))
            spec = ("torus", 1.0, 0.4, 4 * nmin, nmin)
        else:                                     # 36 m^2 unknowns
            spec = ("box", *(3 * [max(2, int(round(math.sqrt(n_target / 36))))]))
        eps_r = float(rng.uniform(1.5, 6.0))
        R = int(rng.integers(1, 33))
        nsteps = int(rng.integers(500, 5001))
        wseed = int(rng.integers(1 << 30))
        V, F, E = make_mesh(spec)
        D = geo.diameter(V)
        dt = D / 4.0
        Tmax, kmax = tmax_kmax(D, dt, eps_r, 1.0)
        ne = E.shape[0]
        waves = make_waves(R, 4.0 * dt, True, seed=wseed)

        def prepare(V=V, F=F, E=E, eps_r=eps_r, dt=dt, kmax=kmax):
            inp = fxgpu.device_inputs(V, F, E)

            def loader(s, V=V, F=F, E=E, eps_r=eps_r, dt=dt, kmax=kmax):
                from paper_2510_07989_amd.serve import stop_if_cancelled
                fxgpu.load_solvers([s], dict(V=V, F=F, E=E, eps_r=eps_r, mu_r=1.0, dt=dt, kmax=kmax, nq=7),
                                   on_lag=lambda i: stop_if_cancelled(s))
            return dict(G=inp["G"], T0s=inp["T0s"], T0h=inp["T0h"], loader=loader)

        prob = dict(name="%s_%d" % (kind, 2 * ne), V=V, F=F, E=E, eps_r=eps_r, mu_r=1.0, dt=dt, kmax=kmax,
                    waves=waves, gnnz=24 * ne, prepare=prepare,
                    # the assembler's rings: three lags of six blocks per medium, while it runs
                    extra_bytes=2 * 3 * 6 * 8 * ne * ne)
        out.append((prob, nsteps, float(arrivals[i])))
    return out


def serving_smoke(args):
    """The serving stream's smoke variant, on by default: the first requests
    of a C4 stream (see c4_requests; its own seed) with a tenth of their steps
    (50 to 500), served by the thread-per-solve server (each request creates,
    loads and marches its solve on its own host thread and stream, in windows
    of mot_run; inputs built on the device in its setup, at most three setups
    at a time), at most 8 at once under a 200 GB budget of peak footprints
    plus the assembler's memory,
    time-boxed: at the box running requests are stopped with mot_cancel (one
    still uploading its lags stops between lags) and requests not yet admitted
    are not served."""
    import numpy as np
    import torch
    from paper_2510_07989_amd.serve import GpuBackend, Request, Server, latency_stats
    t = time.perf_counter()
    stream = c4_requests(args.serving_smoke_requests, seed=251007992)
    log("[smoke] %d requests generated in %.1f s" % (len(stream), time.perf_counter() - t))
    reqs = [Request(i, p, max(1, ns // 10), arr, dict(precond=2, spec_window=32))
            for i, (p, ns, arr) in enumerate(stream)]
    be = GpuBackend(keep_outputs=False, setup_slots=3)
    srv = Server(be, mem_budget=int(200e9), max_active=8, window=128, time_box=args.serving_smoke_box,
                 request_timeout=args.serving_smoke_box, log=log)
    res, summ = srv.run(reqs)
    torch.cuda.empty_cache()
    sizes = sorted(2 * q.problem["E"].shape[0] for q in reqs)
    served = [q for q in reqs if res[q.rid].error is None]
    out = {
        "workload": "C4 smoke stream: %d requests, Poisson arrivals at 2/s, sphere/torus/cube of %d to %d unknowns "
                    "(log-uniform), eps_r U[1.5, 6], 1-32 waves, 50-500 steps (a tenth of C4's), c dt = D/4; inputs "
                    "built in each request's setup (static and retarded blocks on the device)"
                    % (len(reqs), sizes[0], sizes[-1]),
        "server": "thread per solve (mot_run windows of 128 steps, speculative windows of 32, <= 8 at once, "
                  "<= 3 setups at once)",
        "time_box_s": args.serving_smoke_box, "mem_budget_gb": 200.0,
        "completed": summ["completed"], "cancelled_at_box": summ["cancelled"], "not_served": summ["not_served"],
        "errors": summ["errors"], "wall_s": round(summ["wall_s"], 2),
        "steps_marched": summ["steps_marched"], "steps_per_s": round(summ["steps_per_s"], 1),
        "rhs_steps_per_s": round(summ["rhs_steps_per_s"], 1),
        "step_latency_us": {k: round(1e6 * v, 1) if k != "n" else v for k, v in summ["step_latency_s"].items()},
        "end_to_end_s": {k: round(v, 3) if k != "n" else v for k, v in summ["end_to_end_s"].items()},
        "setup_s": {k: round(v, 3) if k != "n" else v
                    for k, v in latency_stats(r.t_ready - r.t_admit for r in res.values()
                                              if r.t_ready > 0).items()},
        "queue_wait_s": {k: round(v, 3) if k != "n" else v for k, v in summ["queue_wait_s"].items()},
        "max_concurrent": summ["max_concurrent"], "peak_budget_gb": round(summ["peak_budget_used"] / 1e9, 2),
        "completed_unknowns": {"max": max((2 * q.problem["E"].shape[0] for q in served), default=0),
                               "median": float(np.median([2 * q.problem["E"].shape[0] for q in served] or [0]))},
    }
    errs = [r.error for r in res.values() if r.error and not r.error.startswith(("CancelledRun", "NotServed"))]
    if errs:
        out["first_errors"] = errs[:3]
    for v in out.values():              # statistics of an empty set are NaN, which JSON does not carry
        if isinstance(v, dict):
            for k in v:
                if isinstance(v[k], float) and v[k] != v[k]:
                    v[k] = None
    log("[smoke] %d completed, %d cancelled at the box, %d not served, %d errors in %.1f s; %.0f steps/s, step p50 "
        "%.0f us p99 %.0f us; end-to-end p50 %.2f s p99 %.2f s"
        % (summ["completed"], summ["cancelled"], summ["not_served"], summ["errors"], summ["wall_s"],
           summ["steps_per_s"], 1e6 * summ["step_latency_s"]["p50"], 1e6 * summ["step_latency_s"]["p99"],
           summ["end_to_end_s"]["p50"], summ["end_to_end_s"]["p99"]))
    return out


def guarded(fn, limit, result, key):
    """Run a leg under a hard wall-clock limit: if it has not returned by then
    (a request stuck inside the runtime), the JSON line is printed with the leg
    marked and the process ends, so the measured legs are not lost."""
    import threading
    box = {}
    done = threading.Event()

    def target():
        try:
            box["out"] = fn()
        except Exception as e:           # the headline line is printed whatever this leg does
            box["out"] = {"error": "%s: %s" % (type(e).__name__, e)}
        finally:
            done.set()

    threading.Thread(target=target, daemon=True).start()
    if not done.wait(limit):
        result[key] = {"error": "did not finish within %.0f s; the process ended there" % limit}
        log("[%s] did not finish within %.0f s" % (key, limit))
        print(json.dumps(result), flush=True)
        sys.stderr.flush()
        os._exit(0)
    return box["out"]


def serving_c4(args):
    """Continuous batching at serving scale (see c4_requests for the stream):
    the batch server (every active solve stepped together through
    mot_run_batch, windows of 128 steps in speculative windows of 32, three
    setup threads beside it), admission by peak footprint plus the assembler's
    memory under a budget, at most 16 solves at once, time-boxed: at the box
    the solves still running are stopped with mot_cancel and requests not yet
    admitted are not served.  Step latency: a batch call's wall time over its
    steps, for every solve in it."""
    import numpy as np
    import torch
    from paper_2510_07989_amd.serve import BatchServer, GpuBackend, Request, latency_stats
    t = time.perf_counter()
    stream = c4_requests(args.serving_c4_requests)
    log("[c4] %d requests generated in %.1f s" % (len(stream), time.perf_counter() - t))
    reqs = [Request(i, p, ns, arr, dict(precond=2, spec_window=32)) for i, (p, ns, arr) in enumerate(stream)]
    be = GpuBackend(keep_outputs=False)
    budget = int(args.serving_c4_budget_gb * 1e9)
    srv = BatchServer(be, mem_budget=budget, max_active=16, window=128, setup_workers=3,
                      time_box=args.serving_c4_box, request_timeout=args.serving_c4_box, log=log)
    res, summ = srv.run(reqs)
    torch.cuda.empty_cache()
    done = [r for r in res.values() if r.error is None]
    sizes = sorted(2 * q.problem["E"].shape[0] for q in reqs)
    out = {
        "workload": "C4 stream: %d requests, Poisson arrivals at 2/s, sphere/torus/cube of %d to %d unknowns "
                    "(log-uniform), eps_r U[1.5, 6], 1-32 waves, 500-5000 steps, c dt = D/4; inputs built in "
                    "each request's setup (static and retarded blocks on the device)"
                    % (len(reqs), sizes[0], sizes[-1]),
        "server": "batch (mot_run_batch, 128-step calls, 32-step windows, 3 setup threads, <= 16 active)",
        "time_box_s": args.serving_c4_box, "mem_budget_gb": args.serving_c4_budget_gb,
        "completed": summ["completed"], "cancelled_at_box": summ["cancelled"], "not_served": summ["not_served"],
        "errors": summ["errors"], "wall_s": round(summ["wall_s"], 2),
        "steps_marched": summ["steps_marched"], "steps_per_s": round(summ["steps_per_s"], 1),
        "rhs_steps_per_s": round(summ["rhs_steps_per_s"], 1),
        "step_latency_us": {k: round(1e6 * v, 1) if k != "n" else v for k, v in summ["step_latency_s"].items()},
        "end_to_end_s": {k: round(v, 3) if k != "n" else v for k, v in summ["end_to_end_s"].items()},
        "setup_s": {k: round(v, 3) if k != "n" else v
                    for k, v in latency_stats(r.t_ready - r.t_admit for r in res.values()
                                              if r.t_ready > 0).items()},
        "queue_wait_s": {k: round(v, 3) if k != "n" else v for k, v in summ["queue_wait_s"].items()},
        "max_concurrent": summ["max_concurrent"], "peak_budget_gb": round(summ["peak_budget_used"] / 1e9, 2),
        "completed_unknowns": {"max": max((2 * q.problem["E"].shape[0] for q in reqs
                                           if res[q.rid].error is None), default=0),
                               "median": float(np.median([2 * q.problem["E"].shape[0] for q in reqs
                                                          if res[q.rid].error is None] or [0]))},
    }
    errs = [r.error for r in res.values() if r.error and not r.error.startswith(("CancelledRun", "NotServed"))]
    if errs:
        out["first_errors"] = errs[:3]
    log("[c4] %d completed, %d cancelled at the box, %d not served, %d errors in %.1f s; %.0f steps/s, step p50 "
        "%.0f us p99 %.0f us; end-to-end p50 %.2f s p99 %.2f s"
        % (summ["completed"], summ["cancelled"], summ["not_served"], summ["errors"], summ["wall_s"],
           summ["steps_per_s"], 1e6 * summ["step_latency_s"]["p50"], 1e6 * summ["step_latency_s"]["p99"],
           summ["end_to_end_s"]["p50"], summ["end_to_end_s"]["p99"]))
    return out


def serving(nreq, have=None, seed=251007990):
    """Continuous batching on one GPU: a seeded Poisson stream of requests,
    each a random scatterer among the assembled ones (torus, box and sphere
    meshes of 432 to 6144 unknowns), 1 to 16 of its plane waves, 500 to 2000
    steps; admission by peak device footprint under a budget, at most 8 solves
    at once, windows of 128 steps, every request from mot_create on (setup, the
    upload and fold of its lag blocks, the march, outputs on the host); the
    same stream once with launches and once with graph replay."""
    import numpy as np
    from fixture.problem import build_problem
    from paper_2510_07989_amd.serve import GpuBackend, Request, Server, latency_stats
    t = time.perf_counter()
    have = dict(have or {})
    probs = {m: have[m] if m in have else build_problem(m) for m in SERVING_MESHES}
    log("serving inputs assembled in %.1f s" % (time.perf_counter() - t))
    rng = np.random.Generator(np.random.PCG64(seed))
    rate = 8.0                                    # requests per second
    arrivals = np.cumsum(rng.exponential(1.0 / rate, nreq))
    reqs = []
    for i in range(nreq):
        m = SERVING_MESHES[int(rng.integers(len(SERVING_MESHES)))]
        p = probs[m]
        nw = len(p["waves"])
        R = 1 if nw == 1 else int(rng.integers(1, nw + 1))
        nsteps = int(rng.integers(500, 2001))
        pr = dict(p, waves=p["waves"][:R])
        reqs.append(Request(i, pr, nsteps, float(arrivals[i]), dict(precond=2)))
        log("[serve] request %d: %s, %d waves, %d steps, arrives at %.3f s" % (i, m, R, nsteps, arrivals[i]))
    out = {"requests": nreq, "arrival_rate_per_s": rate, "seed": seed, "meshes": SERVING_MESHES,
           "max_active": 8, "window_steps": 128}
    fps = sorted(GpuBackend().footprint(r) for r in reqs)
    budget = 3 * fps[-1]
    out["mem_budget_bytes"] = budget
    # the same stream twice: windows queued launch by launch, then replayed from
    # captured graphs (128-step windows: one RHS batch, so every full window replays)
    for label, graph in (("launches", 0), ("graphs", 1)):
        be = GpuBackend(options={"graph": graph}, keep_outputs=True)
        srv = Server(be, mem_budget=budget, max_active=8, window=128, request_timeout=60.0, log=log)
        res, summ = srv.run(reqs)
        log("serving (%s): %d requests in %.2f s, %.1f steps/s, step p50 %.1f us p99 %.1f us, end-to-end p50 "
            "%.3f s p99 %.3f s" % (label, nreq, summ["wall_s"], summ["steps_per_s"],
                                   1e6 * summ["step_latency_s"]["p50"], 1e6 * summ["step_latency_s"]["p99"],
                                   summ["end_to_end_s"]["p50"], summ["end_to_end_s"]["p99"]))
        mix = {}
        for r in reqs:
            mix[r.problem["name"]] = mix.get(r.problem["name"], 0) + 1
        out[label] = {
            "wall_s": round(summ["wall_s"], 3), "steps_per_s": round(summ["steps_per_s"], 1),
            "rhs_steps_per_s": round(summ["rhs_steps_per_s"], 1),
            "step_latency_us": {k: round(1e6 * v, 2) if k != "n" else v for k, v in summ["step_latency_s"].items()},
            "end_to_end_s": {k: round(v, 4) if k != "n" else v for k, v in summ["end_to_end_s"].items()},
            "queue_wait_s": {k: round(v, 4) if k != "n" else v for k, v in summ["queue_wait_s"].items()},
            "setup_s": {k: round(v, 4) if k != "n" else v
                        for k, v in latency_stats(r.t_ready - r.t_admit for r in res.values()
                                                  if r.error is None).items()},
            "mix": mix,
            "max_concurrent": summ["max_concurrent"], "errors": summ["errors"]}
    out["note"] = ("requests reuse the scatterers assembled for this run (host-side assembly of hundreds of "
                   "distinct large meshes is out of reach of a bench run); each request still builds its "
                   "solver, uploads and folds its lags on the device")
    return out


if __name__ == "__main__":
    main()
