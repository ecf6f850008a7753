#!/usr/bin/env python3
"""MOT throughput on one MI355X: steps/s of the qHP TD-PMCHWT march.

Headline workload: torus R = 1, r = 0.4, 2048 triangles / 3072 edges -> 6144
unknowns, eps_r = 4, mu_r = 1, dt = 2.0 (c dt comparable to the diameter),
one Gaussian plane wave, plain FP64, 10,000 steps.  A step is the whole hot
path: tested incident fields, preconditioned RHS, history convolution over
Q_1..Q_{L-1}, GMRES on Q_0, ring update, and the loop/star current recovery
of the timed steps.  Inputs are assembled on the host and resident on the
device before the timed region.

The `batched` object compares, on one sphere mesh (1280 triangles / 1920
edges -> 3840 unknowns, eps_r = 2, dt = 0.15): plain FP64 with one wave, FP64
with 16 seeded waves marched together, and the mixed path (FP32-stored lags,
FP64 MFMA products) with the same 16 waves, whose error is stated against the
FP64 run.

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
    "torus_3072": "torus R=1 r=0.4, 2048 triangles / 3072 edges -> 6144 unknowns, eps_r=4, mu_r=1, "
                  "dt=2.0, 1 Gaussian plane wave",
    "sphere_480": "sphere r=1, 320 triangles / 480 edges -> 960 unknowns, eps_r=2, dt=0.25, "
                  "1 Gaussian plane wave",
    "sphere_1920_r16": "sphere r=1, 1280 triangles / 1920 edges -> 3840 unknowns, eps_r=2, dt=0.15, "
                       "16 seeded Gaussian plane waves marched together",
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


def cpu_baseline(prob, budget_s, nmax):
    """The oracle, as it stands, on the first steps of the same problem."""
    from oracle.mot_oracle import Oracle, march, recover
    t = time.perf_counter()
    O = Oracle(prob)
    prep = time.perf_counter() - t
    t = time.perf_counter()
    r1 = O.rhs_all(1)
    march(O.Q, r1)
    one = time.perf_counter() - t
    ns = int(max(3, min(nmax, budget_s / max(one, 1e-6))))
    t = time.perf_counter()
    r = O.rhs_all(ns)
    W = march(O.Q, r)
    loop, star = recover(O.P, O.Tmax, prob["dt"], W)
    el = time.perf_counter() - t
    return dict(steps=ns, seconds=el, prep_s=prep, W=W, loop=loop, star=star)


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


def history_kernel_name(R, precision, mix_group, sched_hist=11):
    if R == 1:
        if sched_hist in (11, 22, 24):
            return "k_history_co"
        return "k_history_rows<%d>" % (sched_hist % 10) if sched_hist > 10 else "k_history"
    if precision == 2:
        fl = {64: 16, 16: 4}.get(mix_group, 1)
        return "k_hist_mfma<%d, %d>" % (col_blocks(R), fl)
    return "k_tile_gemm<%s, %d>" % ("double" if precision == 0 else "float", col_blocks(R))


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


def measure(mot, prob, name, precision, K, W_, precond, split, hilo, mix_group, outputs=True, far=None):
    """Set up one problem on the device, march W_ warm-up steps (kept as the
    parity sample), then time K steps with device-resident outputs."""
    import torch
    R = len(prob["waves"])
    opts = mot.default_options(profile=PROFILE_EVERY, max_steps=W_ + K + 8, precond=precond, stream_split=split,
                               precision=precision, hilo_lags=hilo, mix_group=mix_group)
    t = time.perf_counter()
    s = mot.Solver(prob["V"], prob["F"], prob["E"], prob["eps_r"], prob["mu_r"], prob["dt"],
                   prob["T0s"], prob["T0h"], prob["G"], prob["waves"], options=opts,
                   stream=torch.cuda.current_stream().cuda_stream)
    s.load_raw(prob["raw"], prob["kmax"])
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t
    inf0 = s.info()
    log("[%s R=%d %s] device setup %.2f s (preconditioner %.0f ms, fold %.0f ms), %d lags, %.2f GB on device; "
        "schedules history %d, Q0 %d, preconditioner %d (tuned in %.1f ms)"
        % (name, R, PRECISION[precision], t_setup, inf0["setup_ms"], inf0["fold_ms"], inf0["nlags"],
           inf0["device_bytes"] / 1e9, inf0["sched_hist"], inf0["sched_q0"], inf0["sched_pc"], inf0["tune_ms"]))
    warm = s.run(W_, w=True, loop=True, star=True, device=False)
    torch.cuda.synchronize()
    a = s.info()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.run(K, w=outputs, loop=outputs, star=outputs, device=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    b = s.info()
    ff = late = None
    if far is not None:
        # diagnostics after the timed march: a failure here must not cost the step-rate line
        try:
            ff = far_field_timing(s, W_ + K, 2 * prob["E"].shape[0], R, far)
            late = late_time(s, W_ + K)
        except Exception as e:  # noqa: BLE001
            log("far-field / late-time diagnostics failed: %r" % (e,))
    s.close()
    ne, n, L = prob["E"].shape[0], 2 * prob["E"].shape[0], b["nlags"]
    hist_us = 1e3 * (b["hist_ms"] - a["hist_ms"]) / max(1, b["hist_launches"] - a["hist_launches"])
    q0_us = 1e3 * (b["q0_ms"] - a["q0_ms"]) / max(1, b["q0_launches"] - a["q0_launches"])
    hb, hf = history_model(ne, n, L, R, precision, hilo)
    kname = history_kernel_name(R, precision, mix_group, inf0["sched_hist"])
    dtype = "f32" if precision == 2 else "f64"
    hist = roofline(kname, hb, hf, hist_us, dtype, R > 1, measured_traffic(kname, name))
    q0b = 8.0 * (3 * ne * ne + 2 * n * R)
    sq = inf0["sched_q0"]
    q0name = (("k_q0_rows<%d>" % (sq % 10) if sq > 10 else "k_q0_matvec") if R == 1
              else "k_tile_gemm<double, %d>" % col_blocks(R))
    q0 = roofline(q0name, q0b, 2.0 * 4 * ne * ne * R, q0_us, "f64", R > 1,
                  measured_traffic(q0name if R == 1 else q0name + " (Q_0)", name))
    hist_tot = b["hist_ms"] - a["hist_ms"]
    q0_tot = b["q0_ms"] - a["q0_ms"]
    out = dict(steps_s=K / el, el=el, K=K, W=W_, R=R, n=n, L=L, kmax=b["kmax"], setup_s=t_setup,
               iters=(b["gmres_iters_total"] - a["gmres_iters_total"]) / K,
               q0_launches=PROFILE_EVERY * (b["q0_launches"] - a["q0_launches"]) / K, hist=hist, q0=q0,
               dominant=hist if hist_tot >= q0_tot else q0, warm=warm, recover_ms=b["recover_ms"],
               device_gb=inf0["device_bytes"] / 1e9, far_field=ff, late_time=late,
               schedule={"history": inf0["sched_hist"], "q0": inf0["sched_q0"], "precond": inf0["sched_pc"],
                         "autotuned": bool(inf0["tuned"] and opts.autotune), "tune_ms": round(inf0["tune_ms"], 1)})
    log("[%s R=%d] timed %d steps in %.3f s: %.1f steps/s (%.1f RHS-steps/s), %.2f GMRES its/step; "
        "history %.1f us (%s %.4g %s), Q0 product %.1f us"
        % (name, R, K, el, K / el, R * K / el, out["iters"], hist_us, hist["bound"], hist["achieved"],
           hist["unit"], q0_us))
    return out


def graph_compare(mot, prob, K, W_, precond):
    """The same march with its speculative windows queued launch by launch and
    replayed from captured HIP graphs, on a stream of its own, no events."""
    import torch
    out = {}
    for g in (0, 1):
        st = torch.cuda.Stream()
        opts = mot.default_options(max_steps=W_ + K + 8, precond=precond, graph=g)
        s = mot.Solver(prob["V"], prob["F"], prob["E"], prob["eps_r"], prob["mu_r"], prob["dt"], prob["T0s"],
                       prob["T0h"], prob["G"], prob["waves"], options=opts, stream=st.cuda_stream)
        s.load_raw(prob["raw"], prob["kmax"])
        with torch.cuda.stream(st):
            s.run(W_, w=False, loop=False, star=False, device=True)
            st.synchronize()
            t0 = time.perf_counter()
            s.run(K, w=True, loop=True, star=True, device=True)
            st.synchronize()
            el = time.perf_counter() - t0
        inf = s.info()
        s.close()
        out["graph" if g else "launches"] = {"steps_s": round(K / el, 1), "graph_windows": inf["graph_windows"]}
    log("window replay: launches %.1f steps/s, graphs %.1f steps/s (%d windows)"
        % (out["launches"]["steps_s"], out["graph"]["steps_s"], out["graph"]["graph_windows"]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="torus_3072", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched/mixed comparison")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay comparison")
    ap.add_argument("--no-wide", action="store_true", help="skip the 64-wave batched runs")
    ap.add_argument("--batched-steps", type=int, default=1000)
    ap.add_argument("--serving", action="store_true",
                    help="also measure continuous batching of a request stream (not run by default)")
    ap.add_argument("--serving-requests", type=int, default=32)
    ap.add_argument("--no-step-batch", action="store_true", help="skip the mot_run_batch comparison")
    ap.add_argument("--no-far-field", action="store_true", help="skip the far-field timing")
    ap.add_argument("--precond", type=int, default=2, help="0 none, 1 FP32, 2 FP64 approximate inverse")
    ap.add_argument("--split", type=int, default=0, help="wavefronts per matrix row (0: by size)")
    ap.add_argument("--precision", type=int, default=0, help="0 FP64, 1 mixed (FP64 MFMA), 2 mixed (FP32 MFMA)")
    ap.add_argument("--hilo", type=int, default=2, help="mixed: lags with an FP32 low part (-1: none)")
    ap.add_argument("--mix-group", type=int, default=4, help="precision 2: summation indices per FP32 sum")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the MOT march of one problem runs on one device; "
              "runs on several GPUs are not part of this benchmark.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    import paper_2510_07989_amd as mot
    from fixture.problem import build_problem

    W_, K = args.warmup, args.steps
    t = time.perf_counter()
    prob = build_problem(args.workload, nsteps=W_ + K, verbose=True)
    t_fixture = time.perf_counter() - t
    log("inputs assembled on the host in %.1f s" % t_fixture)
    m = measure(mot, prob, args.workload, args.precision, K, W_, args.precond, args.split, args.hilo,
                args.mix_group, far=None if args.no_far_field else FAR_FIELD_FREQ.get(args.workload, 0.01))
    R = m["R"]
    result = {
        "metric": "MOT steps/s (%s, %d RHS)" % ("plain FP64" if args.precision == 0 else "mixed precision", R),
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
        "dtype": "f64" if args.precision == 0 else "f32 storage, f64 arithmetic" if args.precision == 1 else "f32",
        "data": "synthetic",
        "config": {"workload": args.workload + ": " + WORKLOADS[args.workload], "nrhs": R,
                   "unknowns": m["n"], "lags": m["L"], "kmax": m["kmax"], "precision": PRECISION[args.precision],
                   "q0_preconditioner": ["none", "fp32 approximate inverse", "fp64 approximate inverse"][args.precond]},
        "roofline": m["dominant"],
        "history_kernel": m["hist"],
        "q0_product": dict(m["q0"], launches_per_step=round(m["q0_launches"], 2)),
        "gmres_iters_per_step": round(m["iters"], 2),
        "schedule": m["schedule"],
        "setup_s": round(m["setup_s"], 3),
        "fixture_s": round(t_fixture, 1),
        "device_gb": round(m["device_gb"], 2),
    }
    if m["far_field"] is not None:
        result["far_field"] = m["far_field"]
    if m["late_time"] is not None:
        result["late_time"] = m["late_time"]

    if not args.no_cpu_baseline:
        cb = cpu_baseline(prob, args.cpu_budget, min(W_, 400))
        ns = cb["steps"]
        warm = m["warm"]
        e_w = float(np.linalg.norm(warm["w"][:ns] - cb["W"]) / np.linalg.norm(cb["W"]))
        e_l = float(np.linalg.norm(warm["loop"][:ns] - cb["loop"]) / np.linalg.norm(cb["loop"]))
        e_s = float(np.linalg.norm(warm["star"][:ns] - cb["star"]) / max(np.linalg.norm(cb["star"]), 1e-300))
        result["cpu_baseline"] = {"value": round(ns / cb["seconds"], 4), "unit": "steps/s",
                                  "cores": blas_threads(), "kind": "oracle",
                                  "sample": "first %d steps of the same workload (RHS, march with LU of Q_0, "
                                            "recovery), oracle setup %.1f s not timed" % (ns, cb["prep_s"])}
        result["err_vs_oracle"] = {"steps": ns, "w": e_w, "loop": e_l, "star": e_s}
        log("oracle: %d steps in %.1f s; GPU vs oracle: w %.2e loop %.2e star %.2e" % (ns, cb["seconds"], e_w, e_l, e_s))

    if not args.no_graph:
        result["graph_replay"] = dict(graph_compare(mot, prob, min(K, 5000), W_, args.precond),
                                      steps=min(K, 5000), workload=args.workload)

    if not args.no_batched:
        name = "sphere_1920_r16"
        Kb, Wb = args.batched_steps, 300
        t = time.perf_counter()
        pb = build_problem(name, nsteps=Wb + Kb, verbose=True)
        log("batched inputs assembled on the host in %.1f s" % (time.perf_counter() - t))
        one = dict(pb, waves=pb["waves"][:1])
        r1 = measure(mot, one, name, 0, Kb, Wb, args.precond, args.split, args.hilo, args.mix_group, outputs=False)
        r16 = measure(mot, pb, name, 0, Kb, Wb, args.precond, args.split, args.hilo, args.mix_group, outputs=False)
        rmx = measure(mot, pb, name, 1, Kb, Wb, args.precond, args.split, args.hilo, args.mix_group, outputs=False)

        def rel(a, b):
            return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))

        err = {k: rel(rmx["warm"][k], r16["warm"][k]) for k in ("w", "loop", "star")}
        nrm = np.linalg.norm(rmx["warm"]["w"].reshape(Wb, -1), axis=1)
        tail = np.log10(nrm[-Wb // 4:] + 1e-300)
        growth = float(np.polyfit(np.arange(tail.size), tail, 1)[0])

        def brief(r):
            return {"steps_s": round(r["steps_s"], 2), "rhs_steps_per_s": round(r["steps_s"] * r["R"], 1),
                    "ms_per_step": round(1e3 * r["el"] / r["K"], 4), "gmres_iters_per_step": round(r["iters"], 2),
                    "history_kernel": r["hist"], "schedule": r["schedule"], "device_gb": round(r["device_gb"], 2)}

        result["batched"] = {
            "workload": name + ": " + WORKLOADS[name],
            "steps": Kb, "warmup": Wb,
            "fp64_1rhs": brief(r1),
            "fp64_16rhs": brief(r16),
            "mixed_16rhs": dict(brief(rmx), precision=PRECISION[1], hilo_lags=args.hilo,
                                err_vs_fp64_16rhs={"steps": Wb, **err},
                                late_log10_growth_per_step=growth),
            "mixed_vs_fp64_1rhs_steps_ratio": round(rmx["steps_s"] / r1["steps_s"], 3),
            "mixed_vs_fp64_1rhs_rhs_steps_ratio": round(rmx["steps_s"] * rmx["R"] / r1["steps_s"], 2),
        }
        log("batched: FP64 1 RHS %.1f steps/s; FP64 16 RHS %.1f; mixed 16 RHS %.1f (err w %.2e star %.2e vs FP64)"
            % (r1["steps_s"], r16["steps_s"], rmx["steps_s"], err["w"], err["star"]))
        if not args.no_wide:
            # 64 waves on the same mesh (the lag blocks do not depend on the
            # waves): the history products become MFMA-bound
            from fixture.problem import CONFIGS, make_waves
            cfg = CONFIGS[name]
            p64 = dict(pb, waves=make_waves(64, cfg["sigma"], True))
            K64, W64 = 300, 100
            w64 = {}
            for key, prec in (("fp64_64rhs", 0), ("mixed_64rhs", 1), ("mixed32_64rhs", 2)):
                w64[key] = measure(mot, p64, name, prec, K64, W64, args.precond, args.split, args.hilo,
                                   args.mix_group, outputs=False)
            ref = w64["fp64_64rhs"]["warm"]
            wide = {"workload": name + " with 64 seeded waves", "steps": K64, "warmup": W64}
            for key, prec in (("fp64_64rhs", 0), ("mixed_64rhs", 1), ("mixed32_64rhs", 2)):
                e = dict(brief(w64[key]), precision=PRECISION[prec])
                if prec:
                    e["err_vs_fp64_64rhs"] = {"steps": W64, **{k: rel(w64[key]["warm"][k], ref[k])
                                                               for k in ("w", "loop", "star")}}
                    if prec == 2:
                        e["mix_group"] = args.mix_group
                wide[key] = e
            result["batched"]["wide"] = wide
            log("batched, 64 waves: FP64 %.1f steps/s, mixed %.1f (err w %.2e), mixed32 %.1f (err w %.2e)"
                % (w64["fp64_64rhs"]["steps_s"], w64["mixed_64rhs"]["steps_s"],
                   wide["mixed_64rhs"]["err_vs_fp64_64rhs"]["w"], w64["mixed32_64rhs"]["steps_s"],
                   wide["mixed32_64rhs"]["err_vs_fp64_64rhs"]["w"]))
    if not args.no_step_batch:
        result["step_batch"] = step_batch(mot)
    if args.serving:
        have = {args.workload: prob}
        if not args.no_batched:
            have["sphere_1920_r16"] = pb
        result["serving"] = serving(args.serving_requests, have)
    print(json.dumps(result), flush=True)


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
