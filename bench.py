#!/usr/bin/env python3
"""MOT throughput on one MI355X: steps/s of the qHP TD-PMCHWT march.

Workload (default): torus R = 1, r = 0.4, 2048 triangles / 3072 edges ->
6144 unknowns, eps_r = 4, mu_r = 1, dt = 2.0 (c dt comparable to the
diameter), one Gaussian plane wave, plain FP64.  A step is the whole hot
path: tested incident fields, preconditioned RHS, history convolution over
Q_1..Q_{L-1}, GMRES on Q_0, ring update, and the loop/star current recovery
of the timed steps.  Inputs are assembled on the host and resident on the
device before the timed region.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "torus_3072": "torus R=1 r=0.4, 2048 triangles / 3072 edges -> 6144 unknowns, eps_r=4, mu_r=1, "
                  "dt=2.0, 1 Gaussian plane wave, plain FP64",
    "sphere_480": "sphere r=1, 320 triangles / 480 edges -> 960 unknowns, eps_r=2, dt=0.25, "
                  "1 Gaussian plane wave, plain FP64",
    "sphere_1920_r16": "sphere r=1, 1280 triangles / 1920 edges -> 3840 unknowns, eps_r=2, dt=0.15, "
                       "16 seeded Gaussian plane waves marched together",
}


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


def cpu_baseline(prob, budget_s, nmax):
    """The oracle, as it stands, on the first steps of the same problem."""
    import numpy as np
    from oracle.mot_oracle import Oracle, march, recover
    t = time.perf_counter()
    O = Oracle(prob)
    prep = time.perf_counter() - t
    # one step to size the sample
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--warmup", type=int, default=60)
    ap.add_argument("--workload", default="torus_3072", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precond", type=int, default=2, help="0 none, 1 FP32, 2 FP64 approximate inverse")
    ap.add_argument("--split", type=int, default=0, help="wavefronts per matrix row (0: by size)")
    ap.add_argument("--precision", type=int, default=0, help="0 FP64 history, 1 mixed FP32/MFMA history")
    ap.add_argument("--hilo", type=int, default=2, help="mixed: lags with split hi/lo products (-1: none)")
    ap.add_argument("--mix-group", type=int, default=4, help="mixed: summation indices per FP32 accumulator (4, 16, 64)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the MOT march of one problem runs on one device "
              "(multi-GPU sharding is described in DESIGN.md, not run).", file=sys.stderr)
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

    opts = mot.default_options(profile=1, max_steps=W_ + K + 8, precond=args.precond, stream_split=args.split,
                               precision=args.precision, hilo_lags=args.hilo, mix_group=args.mix_group)
    t = time.perf_counter()
    s = mot.Solver(prob["V"], prob["F"], prob["E"], prob["eps_r"], prob["mu_r"], prob["dt"],
                   prob["T0s"], prob["T0h"], prob["G"], prob["waves"], options=opts,
                   stream=torch.cuda.current_stream().cuda_stream)
    s.load_raw(prob["raw"], prob["kmax"])
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t
    inf0 = s.info()
    log("device setup %.2f s (preconditioner %.0f ms, fold %.0f ms), %d lags, %.2f GB on device"
        % (t_setup, inf0["setup_ms"], inf0["fold_ms"], inf0["nlags"], inf0["device_bytes"] / 1e9))

    # warm-up steps (their outputs are also the parity sample)
    warm = s.run(W_, w=True, loop=True, star=True, device=False)
    torch.cuda.synchronize()
    a = s.info()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = s.run(K, w=True, loop=True, star=True, device=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    b = s.info()
    el = t1 - t0
    steps_s = K / el
    ne, n = s.ne, s.n
    R = s.nrhs
    L = b["nlags"]
    qb = 4 if args.precision == 1 else 8
    iters = (b["gmres_iters_total"] - a["gmres_iters_total"]) / K
    # algorithmic bytes (FP64): the Q_0 product reads q1, qk, q2 (3 ne^2) and the
    # input vector, writes n; the history kernel reads the (L-1) 3 ne^2 entries
    # of Q_1..Q_{L-1}, the L-1 history vectors and r_k, writes n.
    q0_bytes = 8.0 * (3 * ne * ne + 2 * n * R)
    hist_bytes = qb * (L - 1) * 3 * ne * ne + 8.0 * ((L - 1) * n * R + 2 * n * R)
    q0_ms = (b["q0_ms"] - a["q0_ms"]) / max(1, b["q0_launches"] - a["q0_launches"])
    hist_ms = (b["hist_ms"] - a["hist_ms"]) / max(1, b["hist_launches"] - a["hist_launches"])
    q0_tot = b["q0_ms"] - a["q0_ms"]
    hist_tot = b["hist_ms"] - a["hist_ms"]
    q0_gbs = q0_bytes / (q0_ms * 1e-3) / 1e9
    hist_gbs = hist_bytes / (hist_ms * 1e-3) / 1e9
    if q0_tot >= hist_tot:
        dom = dict(kernel="k_q0_matvec (GMRES Q_0 product)", bytes=q0_bytes, ms=q0_ms, gbs=q0_gbs)
    else:
        dom = dict(kernel="k_history (history convolution)", bytes=hist_bytes, ms=hist_ms, gbs=hist_gbs)
    log("timed %d steps in %.3f s: %.1f steps/s, %.2f GMRES its/step; Q0 product %.1f us (%.0f GB/s), "
        "history %.1f us (%.0f GB/s); recovery %.1f ms"
        % (K, el, steps_s, iters, q0_ms * 1e3, q0_gbs, hist_ms * 1e3, hist_gbs, b["recover_ms"]))

    prec = "fp64" if args.precision == 0 else "mixed fp32-mfma history"
    result = {
        "metric": "MOT steps/s (%s, %d RHS)" % ("plain FP64" if args.precision == 0 else "mixed precision", R),
        "value": round(steps_s, 3),
        "unit": "steps/s",
        "rhs_steps_per_s": round(steps_s * R, 2),
        "n_gpus": 1,
        "steps": K,
        "warmup": W_,
        "ms_per_step": round(1e3 * el / K, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload + ": " + WORKLOADS[args.workload], "nrhs": R,
                   "unknowns": n, "lags": L, "kmax": b["kmax"], "precision": prec,
                   "q0_preconditioner": ["none", "fp32 approximate inverse", "fp64 approximate inverse"][args.precond]},
        "roofline": {"bound": "hbm", "kernel": dom["kernel"], "achieved": round(dom["gbs"], 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(dom["gbs"] / HBM_PEAK_GBS, 4),
                     "traffic": None, "bytes_per_launch": dom["bytes"], "avg_launch_us": round(dom["ms"] * 1e3, 2)},
        "history_kernel": {"achieved_gbs": round(hist_gbs, 1), "avg_launch_us": round(hist_ms * 1e3, 2),
                           "bytes_per_launch": hist_bytes},
        "q0_product": {"achieved_gbs": round(q0_gbs, 1), "avg_launch_us": round(q0_ms * 1e3, 2),
                       "bytes_per_launch": q0_bytes, "launches_per_step": round((b["q0_launches"] - a["q0_launches"]) / K, 2)},
        "gmres_iters_per_step": round(iters, 2),
        "setup_s": round(t_setup, 3),
        "fixture_s": round(t_fixture, 1),
    }

    if not args.no_cpu_baseline:
        cb = cpu_baseline(prob, args.cpu_budget, min(W_, 400))
        ns = cb["steps"]
        e_w = float(np.linalg.norm(warm["w"][:ns] - cb["W"]) / np.linalg.norm(cb["W"]))
        e_l = float(np.linalg.norm(warm["loop"][:ns] - cb["loop"]) / np.linalg.norm(cb["loop"]))
        e_s = float(np.linalg.norm(warm["star"][:ns] - cb["star"]) / max(np.linalg.norm(cb["star"]), 1e-300))
        result["cpu_baseline"] = {"value": round(ns / cb["seconds"], 4), "unit": "steps/s",
                                  "cores": blas_threads(), "kind": "oracle",
                                  "sample": "first %d steps of the same workload (RHS, march with LU of Q_0, "
                                            "recovery), oracle setup %.1f s not timed" % (ns, cb["prep_s"])}
        result["err_vs_oracle"] = {"steps": ns, "w": e_w, "loop": e_l, "star": e_s}
        log("oracle: %d steps in %.1f s; GPU vs oracle: w %.2e loop %.2e star %.2e" % (ns, cb["seconds"], e_w, e_l, e_s))
    s.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
