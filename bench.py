#!/usr/bin/env python3
"""Throughput of the additive-kernel matvec and its l-derivative products on one MI355X.

Workload (the large configuration): N = 1e6 points, D = 15 i.i.d. N(0,1)
features min-max scaled to [-1/4, 1/4], 5 consecutive d = 3 windows, Gaussian
kernel l_w = 0.1, sigma_w = 1, R = 16 right-hand sides, n = 64, m = 6,
oversampling 2; FP32 spreading/FFT/interpolation, FP64 multipliers and window
sums (``--precision fp64``: every step in FP64, against the FP64 vector peak).
Synthetic data (seeded); inputs resident in HBM before timing.

One step = one ``addk_dmatvec`` call producing K V and (dK/dl_w) V for all five
windows for the 16 right-hand sides.  ``value`` = right-hand-side vectors per
second for which both products (K v and all dK/dl_w v) are delivered.

Printed as one JSON line, with
  roofline     : the dominant kernel's algorithmic FLOP rate (HIP events over
                 the timed region) against the FP32 vector peak,
  cpu_baseline : the FP64 CPU oracle timed on a bounded sample of output rows,
  accuracy     : FP32 result vs the FP64 GPU path and vs the oracle rows.

Also in the line: ``rates`` (the joint rate and the K-only ``addk_matvec`` rate
over the same steps) and ``stage_hbm`` (algorithmic bytes and HBM rate of the
spread, interpolation and window-sum kernels).

``--workload d1``: the same points with each of the 15 features its own d = 1
window (12 taps per point and window), where spreading and interpolation move
more bytes than they compute on; its roofline is the dominant kernel's
algorithmic HBM rate against the 8 TB/s peak.

``--workload batched``: 64 uneven problems (N log-uniform in [5e3, 2e5], 1-5
windows of d in {1, 2, 3}, 8 RHS, FP32, m = 4) replayed as one autotuned
hipGraph.

``--workload matern-near-field`` measures the near-field corrected Matern-1/2
product instead: the derivative workload's shape (N = 1e5 points, D = 9 N(0,1)
features min-max scaled, 3 windows d = 3, l = (0.05, 0.1, 0.2), R = 1, n = 64,
m = 6), one ``addk_dmatvec`` (K v, dK/dl_w v, dK/dsigma_w v) per step; its
roofline is the close-pair kernel's, with the close pairs counted by brute
force (FP64 distances on the device): 47 flop per unordered pair for the two
kernel values (distance, square root, exponential, two degree-8 polynomials in
r^2; the kernels are symmetric) and 4R per ordered pair (2R multiply-adds).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "kernel matvecs/s and ∂K/∂ℓ matvecs/s at N=1e6, 5×d=3 windows, at rel err ≤1e-5"
METRIC_D1 = "kernel matvecs/s and ∂K/∂ℓ matvecs/s at N=1e6, 15×d=1 windows, at rel err ≤1e-5"
METRIC_MATERN = "Matérn-1/2 kernel matvecs/s and ∂K/∂ℓ, ∂K/∂σ matvecs/s at N=1e5, 3×d=3 windows, at rel err ≤1e-5"
FP32_VECTOR_PEAK_TFLOPS = 157.3
FP64_VECTOR_PEAK_TFLOPS = 78.6
HBM_PEAK_BPS = 8.0e12


def relerr_cols(a: np.ndarray, b: np.ndarray) -> float:
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return float(max(np.linalg.norm(a[:, r] - b[:, r]) / np.linalg.norm(b[:, r]) for r in range(b.shape[1])))


def source_digest() -> str:
    """SHA-256 over the library's device sources (every .hip and .h under csrc/)."""
    csrc = os.path.join(ROOT, "paper_2404_17344_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(stage: str, fname: str = "c5_dmatvec_hbm_traffic.txt"):
    """HBM bytes per launch of a stage's kernel, from a committed rocprofv3 counter
    summary under profiles/ (FETCH_SIZE and WRITE_SIZE, each scaled by a plain copy's
    reading), or None when the summary is missing or the device sources changed
    since it was taken."""
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return None
    digest, table = None, {}
    with open(path) as f:
        for line in f:
            parts = line.split()
            if len(parts) == 2 and parts[0] == "source_sha256:":
                digest = parts[1]
            elif len(parts) == 4 and parts[0] == "traffic_bytes:":
                table[parts[1]] = (float(parts[2]), float(parts[3]))
    if digest != source_digest() or stage not in table:
        return None
    rd, wr = table[stage]
    return {"bytes": rd + wr, "read": rd, "written": wr}


def log(msg: str):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--N", type=int, default=1000000, help="points (default: the full 1e6 workload)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuned leg of the d = 3 and d = 1 workloads")
    ap.add_argument("--no-k-only", action="store_true",
                    help="skip the separate K-only (addk_matvec) measurement, so that a profiled run holds "
                         "only the timed dmatvec steps")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (HBM counter calibration) and exit")
    ap.add_argument("--workload", choices=["large", "d1", "batched", "matern-near-field"], default="large")
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32",
                    help="engine precision (FP32: FP32 grids with FP64 multipliers and sums; FP64: every step)")
    ap.add_argument("--n", type=int, default=64, help="bandwidth of the matern-near-field workload")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested; run with --gpus 1)" % args.gpus, flush=True)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        # A plain copy kernel of known size: its FETCH_SIZE / WRITE_SIZE counters
        # calibrate the ones read for the path's own kernels.
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 5}), flush=True)
        return

    import paper_2404_17344_amd as A
    import workloads as WL

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "matern-near-field":
        return matern_main(args, A, WL, torch)
    if args.workload == "batched":
        return batched_main(args, A, WL, torch)
    return additive_main(args, A, WL, torch)


def stage_hbm(stages, q, d, R, P, N, rs, nout, traffic_file):
    """Per-stage HBM rates of the spread, interpolation and window-sum kernels.

    Algorithmic bytes per launch (the point side; the grid boxes, at most a few
    percent at these sizes, are left out, so these are lower bounds):
      spread (tile or dense-cell):  pairs x (d coordinates + R RHS values) x rs
      interp (tile or dense-cell):  pairs x (d + nout x R) x rs (coordinates read,
                                    per-window products written in the engine's precision)
      combine:                      nout P N R x rs read + (1 + P) N R x 8 written (FP64);
                                    all-d = 1 plans, whose window sum also interpolates
                                    (no per-window products): P N x rs coordinates read
                                    + (1 + P) N R x 8 written
    with rs the engine's real size and pairs the point-window pairs each kernel
    handles.  "measured" is the counter-based traffic where a summary exists."""
    pairs = {"spread": q["tile_points"], "spread_dense": q["dense_points"], "interp": q["tile_points"],
             "interp_dense": q["dense_points"]}
    alg = {k: pairs[k] * (d + R) * rs for k in ("spread", "spread_dense")}
    alg.update({k: pairs[k] * (d + nout * R) * rs for k in ("interp", "interp_dense")})
    fused = d == 1 and stages.get("interp", (0, 0))[1] == 0 and stages.get("interp_dense", (0, 0))[1] == 0
    alg["combine"] = (P * N * rs if fused else nout * P * N * R * rs) + (1 + P) * N * R * 8
    out = {}
    for k, b in alg.items():
        if stages.get(k, (0, 0))[1] == 0:
            continue
        ms = stages[k][0] / stages[k][1]
        e = {"algorithmic_bytes": int(b), "avg_launch_ms": round(ms, 4),
             "GBps": round(b / (ms * 1e-3) / 1e9, 1), "frac_of_hbm_peak": round(b / (ms * 1e-3) / HBM_PEAK_BPS, 4)}
        t = measured_traffic(k, traffic_file)
        if t is not None:
            e["measured_bytes"] = int(t["bytes"])
            e["measured_GBps"] = round(t["bytes"] / (ms * 1e-3) / 1e9, 1)
        out[k] = e
    return out


def additive_main(args, A, WL, torch):
    """The large workloads: five d = 3 windows (default) or fifteen d = 1 windows."""
    dev = torch.device("cuda:0")
    d1 = args.workload == "d1"
    log("generating inputs")
    p = WL.large_d1(N=args.N) if d1 else WL.large_c5(N=args.N)
    N, R, P, W = p.N, p.R, p.P, 2 * p.m
    d = len(p.windows[0])
    # column-major N x R, the layout the library takes: no copy inside the step
    V = torch.from_numpy(np.ascontiguousarray(p.V.T)).to(dev).t()
    torch.cuda.synchronize()

    fp64 = args.precision == "fp64"
    rs = 8 if fp64 else 4
    log("plan (%s)" % args.precision)
    t0 = time.perf_counter()
    plan = A.Plan(p.X, p.windows, p.ell, p.sigma, n=p.n, m=p.m, oversampling=p.oversampling, precision=args.precision)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t0) * 1e3

    def step():
        return plan.dmatvec(V, want_y=True, want_dell=True, want_dsigma=False)

    log("warmup %d" % args.warmup)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    plan.profile(True)
    plan.profile_read()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    log("timing %d steps" % args.steps)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(args.steps):
        out = step()
    ev1.record()
    torch.cuda.synchronize()
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    stages = plan.profile_read()
    plan.profile(False)
    value = R / (ms_per_step * 1e-3)

    # K V alone (addk_matvec): the same number of steps after the derivative run
    ms_k, Yk = None, None
    if not args.no_k_only:
        log("timing %d K-only steps" % args.steps)
        Yk = torch.empty((R, N), dtype=torch.float64, device=dev)
        for _ in range(args.warmup):
            plan.matvec(V, out=Yk)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(args.steps):
            plan.matvec(V, out=Yk)
        ev1.record()
        torch.cuda.synchronize()
        ms_k = ev0.elapsed_time(ev1) / args.steps

    # The autotuned kernel choice (a plan-time measurement; the lines above use the
    # hard-coded defaults): the same steps again with the knobs it keeps.
    q = plan.query()  # the default knobs, as timed above
    tuned = {}
    if not args.no_tune:
        log("autotune")
        knobs = plan.autotune(R=R, nout=2, reps=2)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(args.steps):
            step()
        ev1.record()
        torch.cuda.synchronize()
        ms_t = ev0.elapsed_time(ev1) / args.steps
        tuned = {"tuned_knobs": knobs, "tuned_K_and_dK_dl_matvecs_per_s": round(R / (ms_t * 1e-3), 3),
                 "tuned_ms_per_step": round(ms_t, 4)}

    # Algorithmic FLOPs per launch: one FMA (2 flop) per tap, point-window pair and
    # RHS; interpolation launches produce two outputs (kernel and derivative kernel).
    # Dense-cell and tile kernels split the point-window pairs between them.
    taps = W ** d
    pts = {"spread_dense": q["dense_points"], "spread": q["tile_points"],
           "interp_dense": q["dense_points"], "interp": q["tile_points"]}
    outs = {"spread_dense": 1, "spread": 1, "interp_dense": 2, "interp": 2}
    flops = {k: 2.0 * taps * pts[k] * R * outs[k] for k in pts}
    traffic_file = "d1_dmatvec_hbm_traffic.txt" if d1 else "c5_dmatvec_hbm_traffic.txt"
    hbm = stage_hbm(stages, q, d, R, P, N, rs, 2, traffic_file)
    peak = FP64_VECTOR_PEAK_TFLOPS if fp64 else FP32_VECTOR_PEAK_TFLOPS
    full = N == 1000000 and not fp64
    if d1:
        # 12 taps per point and window: the spread and interpolation kernels are
        # bound by the bytes they move; the dominant one by time is reported
        # against the HBM peak (the interpolation of an all-d = 1 plan runs in the
        # window sum, stage "combine")
        cand = list(hbm)
        dom = max(cand, key=lambda s: stages[s][0])
        e = hbm[dom]
        roofline = {"bound": "hbm", "kernel": dom, "achieved": e["GBps"], "peak": HBM_PEAK_BPS / 1e9,
                    "unit": "GB/s", "frac": e["frac_of_hbm_peak"],
                    "traffic": measured_traffic(dom, traffic_file) if full else None,
                    "avg_launch_ms": e["avg_launch_ms"], "algorithmic_bytes_per_launch": e["algorithmic_bytes"],
                    # the fused window sum interpolates every point-window pair
                    "point_window_pairs": pts.get(dom, q["dense_points"] + q["tile_points"])}
    else:
        cand = [k for k in flops if stages[k][1] > 0]
        dom = max(cand, key=lambda s: stages[s][0])
        tot_ms, launches = stages[dom]
        avg_ms = tot_ms / max(launches, 1)
        achieved = flops[dom] / (avg_ms * 1e-3) / 1e12
        # the d = 3 dense-cell kernels run on the matrix cores (v_mfma_f32_16x16x4f32 /
        # v_mfma_f64_16x16x4f64) unless the knobs turn them off; MI355X's dense FP32 and
        # FP64 matrix peaks equal its vector peaks (157.3 and 78.6 TFLOP/s)
        knob = {"spread_dense": 1, "interp_dense": 2, "interp": 4}.get(dom, 0)
        on_mfma = bool(knob and (q["knobs"] & knob) and (not fp64 or R >= 2))
        roofline = {"bound": "mfma" if on_mfma else "alu", "kernel": dom, "achieved": round(achieved, 3),
                    "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                    "traffic": measured_traffic(dom, traffic_file) if full else None,
                    "avg_launch_ms": round(avg_ms, 4), "algorithmic_flop_per_launch": flops[dom],
                    "point_window_pairs": pts[dom]}
    stage_ms = {k: round(v[0] / max(v[1], 1), 4) for k, v in stages.items() if v[1]}

    accuracy = {}
    Y32 = out[0].cpu().numpy()   # the timed path's outputs (FP64 values in either mode)
    dl32 = out[1].cpu().numpy()
    if Yk is not None:
        accuracy["rel_err_K_only_vs_dmatvec_Y"] = relerr_cols(Yk.t().cpu().numpy(), Y32)
    if not args.no_accuracy and not fp64:
        log("fp64 reference run")
        del out
        plan64 = A.Plan(p.X, p.windows, p.ell, p.sigma, n=p.n, m=p.m, oversampling=p.oversampling, precision="fp64")
        Y64, dl64, _ = plan64.dmatvec(V, want_dsigma=False)
        Y64 = Y64.cpu().numpy()
        dl64 = dl64.cpu().numpy()
        accuracy["rel_err_Y_vs_fp64_gpu"] = relerr_cols(Y32, Y64)
        accuracy["rel_err_dY_dell_vs_fp64_gpu"] = max(relerr_cols(dl32[w], dl64[w]) for w in range(P))
        plan64.close()
        del plan64

    cpu = None
    if not args.no_cpu_baseline:
        from oracle.direct import oracle_direct, oracle_threads
        rng = np.random.default_rng(17347 if d1 else 17345)
        log("cpu baseline (oracle)")
        probe = rng.choice(N, 64, replace=False)
        oracle_direct(p.X, p.windows, p.kernel, p.ell, p.sigma, p.V, rows=probe[:8], want_derivs=True)  # threads up
        t0 = time.perf_counter()
        oracle_direct(p.X, p.windows, p.kernel, p.ell, p.sigma, p.V, rows=probe, want_derivs=True)
        t_probe = time.perf_counter() - t0
        nrows = int(min(max(64, 64 * args.cpu_seconds / max(t_probe, 1e-3)), 8192))
        rows = rng.choice(N, nrows, replace=False)
        t0 = time.perf_counter()
        Yo, dlo, _ = oracle_direct(p.X, p.windows, p.kernel, p.ell, p.sigma, p.V, rows=rows, want_derivs=True)
        t_cpu = time.perf_counter() - t0
        cpu = {"value": round(R * (nrows / N) / t_cpu, 6), "unit": "matvecs/s", "cores": oracle_threads(),
               "kind": "oracle",
               "sample": "%d of %d output rows, all %d windows, %d RHS, K v and dK/dl_w v, FP64 direct sums; "
                         "%.1f s; rate scaled by N/rows" % (nrows, N, P, R, t_cpu)}
        if not args.no_accuracy:
            accuracy["rel_err_Y_vs_oracle_rows"] = relerr_cols(Y32[rows], Yo)
            accuracy["rel_err_dY_dell_vs_oracle_rows"] = max(relerr_cols(dl32[w][rows], dlo[w]) for w in range(P))
            accuracy["oracle_rows"] = nrows

    if d1:
        metric = METRIC_D1
        wl = ("large additive Gaussian, d=1 windows: N=%d, D=15 N(0,1) features min-max scaled, 15 windows d=1, "
              "l=0.1, sigma=1, R=16, n=64, m=6, oversampling 2" % N)
    else:
        metric = METRIC
        wl = ("large additive Gaussian: N=%d, D=15 N(0,1) features min-max scaled, 5 windows d=3, "
              "l=0.1, sigma=1, R=16, n=64, m=6, oversampling 2" % N)
    result = {
        "metric": metric,
        "value": round(value, 3),
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if fp64 else "f32",
        "data": "synthetic",
        "config": {"workload": wl, "N": N, "R": R, "P": P, "n": p.n, "m": p.m, "oversampling": p.oversampling,
                   "step": "addk_dmatvec: K V and dK/dl_w V, all windows",
                   "precision": "FP64 every step" if fp64 else
                                "FP32 spread/FFT/interp with FP64-computed multipliers applied in FP32; "
                                "FP64 window sums and outputs"},
        "rates": {"K_and_dK_dl_matvecs_per_s": round(value, 3),
                  "K_only_matvecs_per_s": round(R / (ms_k * 1e-3), 3) if ms_k else None,
                  "K_only_ms_per_step": round(ms_k, 4) if ms_k else None, **tuned},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "accuracy": accuracy,
        "stage_avg_ms": stage_ms,
        "stage_hbm": hbm,
        "plan_ms": round(plan_ms, 2),
    }
    print(json.dumps(result), flush=True)


def batched_main(args, A, WL, torch):
    """The batched workload: 64 independent problems (N log-uniform in [5e3, 2e5],
    1-5 windows of d in {1, 2, 3}, Gaussian l ~ U(0.05, 0.3), 8 RHS each, FP32,
    m = 4, n per problem from the error model at 1e-5) replayed as one autotuned
    hipGraph.  value = problem right-hand sides delivered per second (one
    matvec = one RHS of one problem through all its windows)."""
    probs = WL.batched_c4()
    R = probs[0].R
    log("batched: %d problems, %d points" % (len(probs), sum(p.N for p in probs)))
    plans = []
    t0 = time.perf_counter()
    for p in probs:
        n = A.choose_n_for(p.X, p.windows, p.ell, m=4, oversampling=2.0, tol=1e-5)
        plans.append(A.Plan(p.X, p.windows, p.ell, p.sigma, n=n, m=4, precision="fp32"))
    B = A.Batch(plans, R=R)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t0) * 1e3
    B.set_inputs([torch.from_numpy(np.ascontiguousarray(p.V)).cuda() for p in probs])
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    # the graph of the hard-coded kernel choices first, then the autotuned one
    for _ in range(args.warmup):
        B.launch()
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(args.steps):
        B.launch()
    ev1.record()
    torch.cuda.synchronize()
    ms_default = ev0.elapsed_time(ev1) / args.steps
    knobs = B.autotune(reps=3)
    for _ in range(args.warmup):
        B.launch()
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(args.steps):
        B.launch()
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    ev0.record()
    for _ in range(args.steps):
        B.run_eager()
    ev1.record()
    torch.cuda.synchronize()
    ms_eager = ev0.elapsed_time(ev1) / args.steps
    nmat = len(probs) * R
    result = {
        "metric": "batched problem matvecs/s (64 uneven problems, 8 RHS, one hipGraph replay)",
        "value": round(nmat / (ms * 1e-3), 3), "unit": "matvecs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched: 64 problems, N log-uniform in [5e3, 2e5], 1-5 windows of d in {1,2,3}, "
                               "l ~ U(0.05, 0.3), R=8, m=4, n per problem at 1e-5, FP32",
                   "problems": len(probs), "points": int(sum(p.N for p in probs)),
                   "windows": int(sum(p.P for p in probs)), "R": R, "knobs": knobs},
        "eager_ms_per_step": round(ms_eager, 4),
        "untuned_ms_per_step": round(ms_default, 4),
        "plan_ms": round(plan_ms, 2),
    }
    print(json.dumps(result), flush=True)


def matern_main(args, A, WL, torch):
    """The near-field corrected Matern-1/2 product on the derivative workload's shape."""
    dev = torch.device("cuda:0")
    N = args.N if args.N != 1000000 else 100000
    log("generating inputs (matern, N=%d)" % N)
    p = WL.derivative_c3(N=N, kernel=WL.MATERN12)
    R, P = p.R, p.P
    V = torch.from_numpy(np.ascontiguousarray(p.V.T)).to(dev).t()
    torch.cuda.synchronize()
    log("plan (%s, near field)" % args.precision)
    t0 = time.perf_counter()
    n = args.n
    plan = A.Plan(p.X, p.windows, p.ell, p.sigma, kernel="matern12", n=n, m=p.m, oversampling=p.oversampling,
                  precision=args.precision, near_field=True)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t0) * 1e3

    def step():
        return plan.dmatvec(V, want_y=True, want_dell=True, want_dsigma=True)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.profile(True)
    plan.profile_read()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    log("timing %d steps" % args.steps)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(args.steps):
        out = step()
    ev1.record()
    torch.cuda.synchronize()
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    stages = plan.profile_read()
    plan.profile(False)
    stage_ms = {k: round(v[0] / max(v[1], 1), 4) for k, v in stages.items() if v[1]}

    # close pairs (ordered, the diagonal included) within each window's radius
    # 5 T_w / n, counted with plain FP64 distances in row blocks
    log("counting close pairs")
    T = plan.query()["T"]
    pairs = 0
    for w, feats in enumerate(p.windows):
        Xw = torch.from_numpy(np.ascontiguousarray(p.X[:, feats])).to(dev)
        r2 = (5.0 * T[w] / n) ** 2
        for s in range(0, N, 2048):
            D2 = ((Xw[s:s + 2048, None, :] - Xw[None, :, :]) ** 2).sum(-1)
            pairs += int((D2 < r2).sum().item())
            del D2
    # kernel values once per unordered pair (the diagonal's N per window once),
    # multiply-adds per ordered pair
    unordered = (pairs + N * len(p.windows)) // 2
    flop = 47 * unordered + 4 * R * pairs
    tot_ms, launches = stages["near"]
    avg_ms = tot_ms / max(launches, 1)
    achieved = flop / (avg_ms * 1e-3) / 1e12
    peak = FP32_VECTOR_PEAK_TFLOPS if args.precision == "fp32" else FP64_VECTOR_PEAK_TFLOPS
    roofline = {"bound": "alu", "kernel": "near", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": None, "avg_launch_ms": round(avg_ms, 4),
                "algorithmic_flop_per_launch": flop, "close_pairs": pairs, "unordered_pairs": unordered}

    Y = out[0].cpu().numpy()
    dl = out[1].cpu().numpy()
    ds = out[2].cpu().numpy()
    cpu, accuracy = None, {}
    if not args.no_cpu_baseline:
        from oracle.direct import oracle_direct, oracle_threads
        rng = np.random.default_rng(17343)
        probe = rng.choice(N, 64, replace=False)
        oracle_direct(p.X, p.windows, p.kernel, p.ell, p.sigma, p.V, rows=probe[:8], want_derivs=True)
        t0 = time.perf_counter()
        oracle_direct(p.X, p.windows, p.kernel, p.ell, p.sigma, p.V, rows=probe, want_derivs=True)
        t_probe = time.perf_counter() - t0
        nrows = int(min(max(64, 64 * args.cpu_seconds / max(t_probe, 1e-3)), N))
        rows = rng.choice(N, nrows, replace=False)
        t0 = time.perf_counter()
        Yo, dlo, dso = oracle_direct(p.X, p.windows, p.kernel, p.ell, p.sigma, p.V, rows=rows, want_derivs=True)
        t_cpu = time.perf_counter() - t0
        cpu = {"value": round(R * (nrows / N) / t_cpu, 6), "unit": "matvecs/s", "cores": oracle_threads(),
               "kind": "oracle",
               "sample": "%d of %d output rows, all 3 windows, 1 RHS, K v, dK/dl_w v and dK/dsigma_w v, FP64 "
                         "direct sums; %.1f s; rate scaled by N/rows" % (nrows, N, t_cpu)}
        if not args.no_accuracy:
            accuracy["rel_err_Y_vs_oracle_rows"] = relerr_cols(Y[rows], Yo)
            accuracy["rel_err_dY_dell_vs_oracle_rows"] = max(relerr_cols(dl[w][rows], dlo[w]) for w in range(P))
            accuracy["rel_err_dY_dsigma_vs_oracle_rows"] = max(relerr_cols(ds[w][rows], dso[w]) for w in range(P))
            accuracy["oracle_rows"] = nrows
    result = {
        "metric": METRIC_MATERN,
        "value": round(R / (ms_per_step * 1e-3), 3),
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "derivative Matern-1/2, near-field corrected: N=%d, D=9 N(0,1) features min-max "
                               "scaled, 3 windows d=3, l=(0.05, 0.1, 0.2), sigma=1, R=1, n=%d, m=6, oversampling 2"
                               % (N, n),
                   "N": N, "R": R, "P": P, "n": n, "m": p.m, "step": "addk_dmatvec: K v, dK/dl_w v, dK/dsigma_w v",
                   "precision": args.precision},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "accuracy": accuracy,
        "stage_avg_ms": stage_ms,
        "plan_ms": round(plan_ms, 2),
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
