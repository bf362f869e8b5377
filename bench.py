"""Benchmark: NLL + gradient of the fourteen-chain D0 -> K+ pi- pi+ pi- model
on 50,000 data events and 4,000,000 phase-space MC events on one MI355X.

One step is one full evaluation (mxa_nll_grad): every lineshape recomputed,
data pass, MC normalisation pass, reductions, finalisation and the copy of
the NLL and its 36-component gradient to the host. Inputs are resident in HBM
(the parameter-independent per-event cache is built once, before timing).

Prints one JSON line. The headline value is the FP32-amplitude path; the
FP64 path and the NLL-only forms are reported beside it, with the error of the
FP32-amplitude result against the FP64 one.
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
sys.path.insert(0, ROOT)

from paper_1702_06735_amd import inputs as I  # noqa: E402

METRIC = ("NLL+grad events/s (FP32-amp vs FP64) at stated error; "
          "toy-fit p50/p99 latency")
HBM_PEAK_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_1702_06735_amd", "csrc", "kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_eval_fp32amp_grad_full.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def gpu_terms_fn(M, model, theta):
    """Per-event |A|^2, |Abar|^2, A Abar*, rate from the library (for the
    accept-reject draw of pseudo-data)."""
    ctx = M.Context(model, device=0)

    def fn(p4, t):
        kind = M.MXA_MC if t is None else M.MXA_DATA
        ctx.load_events(kind, p4, t)
        ctx.set_params(theta)
        return ctx.event_terms(kind, "fp64")

    return ctx, fn


def algorithmic_bytes(n_data, n_mc, word):
    # 25 tier-0 columns per event; data events also read their decay time (FP64)
    return n_mc * 25 * word + n_data * (25 * word + 8)


def kernel_sha():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def read_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_sha():
        return None
    return t.get("bytes_per_launch")


def timed_steps(ctx, fn, steps, warmup, sync):
    """Seconds per step (API call to host values), then the MC pass's average
    kernel duration [ms] from HIP events, taken in a second loop so that the
    events do not perturb the step time."""
    ctx.set_timing(False)
    for _ in range(warmup):
        fn()
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    sync()
    dt = time.perf_counter() - t0
    ctx.set_timing(True)
    ctx.kernel_time(reset=True)
    for _ in range(steps):
        fn()
    sync()
    kms, nk = ctx.kernel_time(reset=True)
    ctx.set_timing(False)
    return dt / steps, kms / max(nk, 1)


def cpu_baseline(model, theta, pd, td, mc):
    import oracle
    n_d, n_m = len(td), len(mc)
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    oracle.nll_grad(model, theta, pd[:n_d], td[:n_d], mc[:n_m])
    dt = time.perf_counter() - t0
    return {"value": (n_d + n_m) / dt, "unit": "events/s", "cores": threads, "kind": "oracle",
            "sample": f"one NLL+gradient evaluation (dual numbers) on {n_d} data + {n_m} MC "
                      f"events of the same workload; {dt:.1f} s on {threads} threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="full", choices=["full", "gradient", "small"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-fraction", type=float, default=0.25,
                    help="fraction of the workload the oracle evaluates")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; run with --gpus 1"}))
        sys.exit(2)

    import torch
    from paper_1702_06735_amd import mixamp as M
    M.load_library()

    W = I.WORKLOADS[args.workload]
    model = W.model
    theta = I.make_theta(model, I.draw_coefficients(model, W.seed_coeff))
    t0 = time.perf_counter()
    mc = I.phase_space(W.n_mc, W.seed_mc)
    log(f"[bench] {W.n_mc} MC events in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    gctx, fn = gpu_terms_fn(M, model, theta)
    data = I.draw_data(fn, W.n_data, W.seed_data, model, theta)
    gctx.close()
    log(f"[bench] {W.n_data} data events from {data.n_candidates} candidates in "
        f"{time.perf_counter() - t0:.1f} s")

    ctx = M.Context(model, device=0)
    ctx.load_events(M.MXA_MC, mc)
    ctx.load_events(M.MXA_DATA, data.p4, data.t)
    ctx.set_params(theta)
    sync = torch.cuda.synchronize
    n_ev = W.n_data + W.n_mc

    results = {}
    for name, f in (("fp32amp_grad", lambda: ctx.nll_grad("fp32amp")),
                    ("fp64_grad", lambda: ctx.nll_grad("fp64")),
                    ("fp32amp_nll", lambda: ctx.nll("fp32amp")),
                    ("fp64_nll", lambda: ctx.nll("fp64"))):
        step_s, kern_ms = timed_steps(ctx, f, args.steps, args.warmup, sync)
        results[name] = (step_s, kern_ms)
        log(f"[bench] {name}: {step_s * 1e6:.1f} us/step, kernel {kern_ms * 1e3:.1f} us, "
            f"{n_ev / step_s:.3e} events/s")

    v64, g64, d64 = ctx.nll_grad("fp64", diag=True)
    v32, g32 = ctx.nll_grad("fp32amp")
    scale = d64[2]
    err = {"fp32amp_vs_fp64_nll_abs": abs(v32 - v64),
           "fp32amp_vs_fp64_nll_over_scale": abs(v32 - v64) / scale,
           "fp32amp_vs_fp64_grad_over_max": float(np.max(np.abs(g32 - g64)) / np.max(np.abs(g64)))}

    if args.copy_probe:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        sync()
        log("[bench] copy probe: 5 x 1 GiB device copies")

    step_s, kern_ms = results["fp32amp_grad"]
    alg = algorithmic_bytes(0, W.n_mc, 4)   # the MC pass: 25 FP32 columns per event
    achieved = alg / (kern_ms * 1e-3) / 1e9
    traffic = read_traffic()
    out = {
        "metric": METRIC,
        "value": n_ev / step_s,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 amplitudes + f64 mixing/logs/sums",
        "data": "synthetic (seeded GENBOD phase space; pseudo-data by accept-reject from the model)",
        "config": {"workload": f"{W.name}: fourteen-chain model, NLL+gradient (36 parameters), "
                               f"{W.n_data} data + {W.n_mc} MC events",
                   "n_data": W.n_data, "n_mc": W.n_mc, "precision": "fp32amp"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic},
        "kernel_us": kern_ms * 1e3,
        "forms": {k: {"events_per_s": n_ev / s, "us_per_step": s * 1e6, "kernel_us": km * 1e3}
                  for k, (s, km) in results.items()},
        "error": err,
    }
    if not args.no_cpu_baseline:
        nd = int(W.n_data * args.cpu_fraction)
        nm = int(W.n_mc * args.cpu_fraction)
        out["cpu_baseline"] = cpu_baseline(model, theta, data.p4[:nd], data.t[:nd], mc[:nm])
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
