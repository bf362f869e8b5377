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
import math
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
UTIL_FILE = os.path.join(ROOT, "profiles", "utilisation_eval_full_50k_4M.json")
HEADLINE_KERNEL = "eval_both_kernel<float, 207, 255, true>"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes(n_data, n_mc, word):
    """Bytes one evaluation must read: the 21-value tier-0 record per event (7
    invariant masses and 14 spin factors with their D-vertex factors), plus
    the decay time of a data event, in the amplitude precision: 84 / 88 B per
    MC / data event in FP32, 168 / 176 B in FP64."""
    return n_mc * 21 * word + n_data * 22 * word


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


def read_utilisation(kernel):
    """VALU busy share [%] and active-lane share of the kernel from the
    committed rocprofv3 counter summary, if taken on the current source."""
    try:
        with open(UTIL_FILE) as f:
            u = json.load(f)
    except (OSError, ValueError):
        return None
    if u.get("kernel_sha") != kernel_sha() or kernel not in u.get("kernels", {}):
        return None
    k = u["kernels"][kernel]
    return {"valu_busy_pct": k["valu_busy_pct"], "valu_lane_util_pct": k["valu_lane_util_pct"]}


class Steps:
    """Per-step wall times [s] (API call to host values) and per-launch
    durations [ms] of the dominant kernel from HIP events."""

    def __init__(self, wall, kern):
        self.wall = np.asarray(wall)
        self.kern = np.asarray(kern)

    @property
    def mean_s(self):
        return float(self.wall.mean())

    @property
    def median_s(self):
        return float(np.median(self.wall))

    @property
    def p99_s(self):
        return float(np.percentile(self.wall, 99))

    @property
    def kernel_ms(self):
        return float(np.median(self.kern))

    def summary(self, n_ev):
        return {"events_per_s": n_ev / self.mean_s, "us_per_step": self.mean_s * 1e6,
                "us_per_step_median": self.median_s * 1e6, "us_per_step_p99": self.p99_s * 1e6,
                "kernel_us": self.kernel_ms * 1e3,
                "kernel_us_mean": float(self.kern.mean()) * 1e3}


def timed_steps(ctx, fn, steps, sync):
    """Each step's wall time (API call to host values: every call returns host
    values, so it has synchronised), then, in a second loop so that the events
    do not perturb the step times, each launch's duration of the dominant
    kernel from HIP events recorded on the context's stream."""
    ctx.set_timing(False)
    sync()
    wall = np.empty(steps)
    for i in range(steps):
        t0 = time.perf_counter()
        fn()
        wall[i] = time.perf_counter() - t0
    sync()
    ctx.set_timing(True)
    ctx.kernel_time(reset=True)
    kern = np.empty(steps)
    for i in range(steps):
        fn()
        kms, nk = ctx.kernel_time(reset=True)
        kern[i] = kms / max(nk, 1)
    sync()
    ctx.set_timing(False)
    return Steps(wall, kern)


def cpu_baseline(model, theta, pd, td, mc, min_seconds=10.0, max_passes=8):
    """The oracle's NLL+gradient (FP64, forward-mode dual numbers, OpenMP over
    events) on the whole workload, repeated until at least ``min_seconds`` of
    CPU work have been timed."""
    import oracle
    n_d, n_m = len(td), len(mc)
    threads = oracle.max_threads()
    passes, dt, ref = 0, 0.0, None
    while passes < max_passes and (passes == 0 or dt < min_seconds):
        t0 = time.perf_counter()
        ref = oracle.nll_grad(model, theta, pd, td, mc)
        dt += time.perf_counter() - t0
        passes += 1
    _, _, _, S = oracle.nll(model, theta, pd, td, mc, diag=True)
    return {"value": passes * (n_d + n_m) / dt, "unit": "events/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{passes} NLL+gradient evaluations of the whole workload ({n_d} data + "
                      f"{n_m} MC events); {dt:.1f} s on {threads} threads"}, (ref[0], ref[1], S)


def errors_vs_oracle(ref, gpu):
    """Error of each GPU form against the oracle's FP64 NLL and gradient on the
    same workload: |dNLL| / |NLL|, |dNLL| / S (S = sum |Gamma t - ln B| +
    n |ln Nhat|) and max |dg| / max |g|."""
    v0, g0, S = ref
    out = {"oracle_nll": v0, "oracle_scale_S": S}
    for name, (v, g) in gpu.items():
        out[name] = {"nll_rel": abs(v - v0) / abs(v0), "nll_over_S": abs(v - v0) / S,
                     "nll_abs": abs(v - v0),
                     "grad_over_max": float(np.max(np.abs(g - g0)) / np.max(np.abs(g0)))}
    return out


def _latency_stats(res):
    """Latency (submission to result), queueing (submission to admission),
    throughput over the whole run, and the same latency percentiles over the
    converged fits alone."""
    lat = np.array([(r["t_done_ns"] - r["t_submit_ns"]) * 1e-6 for r in res])
    wait = np.array([(r["t_start_ns"] - r["t_submit_ns"]) * 1e-6 for r in res])
    conv = np.array([r["status"] == "converged" for r in res])
    span = (max(r["t_done_ns"] for r in res) - min(r["t_submit_ns"] for r in res)) * 1e-9
    ev = sum(r["n_evals"] * r["n"] for r in res)
    out = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "events_per_s": ev / span,
           "mean_ms": float(lat.mean()), "queue_p50_ms": float(np.percentile(wait, 50)),
           "queue_p99_ms": float(np.percentile(wait, 99)),
           "wall_s": span, "fits_per_s": len(res) / span,
           "evals_mean": float(np.mean([r["n_evals"] for r in res])),
           "converged": int(conv.sum()),
           "max_evals": int(sum(r["status"] == "max_evals" for r in res)),
           "failed": int(sum(r["status"] not in ("converged", "max_evals") for r in res))}
    if conv.any():
        out["converged_p50_ms"] = float(np.percentile(lat[conv], 50))
        out["converged_p99_ms"] = float(np.percentile(lat[conv], 99))
    return out


def serving(M, model, theta, mc_host, args):
    """Toy-fit serving (the sensitivity studies of Sec. 4 as a service): fits
    of n ~ log-uniform[5e3, 5e5] events arrive as a Poisson stream of 200/s;
    each toy's x, y are the nominal ones jittered by U[-0.002, 0.002]; every
    fit starts at the nominal point, floats the coefficients (one Abar_f
    coefficient fixed) and x, y, stops at an estimated distance to the
    minimum below 1e-4, and shares one 4M-event MC sample through its Gram
    matrix (fixed masses and widths). Latency = submission to result. These
    fits keep their bases in FP64, with a cap of 500 evaluations: with every
    coefficient free the NLL is nearly flat along the Abar_f coefficients and
    x, y, and the minimiser needs ~85 evaluations (median; 99% within ~240)
    with a smooth NLL. The server with FP32 bases (evaluated in FP64 as well)
    is reported beside, with a cap of 1000.
    Batched (64 slots), under a 256 MB HBM budget, and one fit at a time;
    then the same fits submitted all at once (the server's capacity: events/s
    of a saturated server, batched against one fit at a time, and the
    256 MB budget binding admission).
    Then the same fits with the masses and widths floating too (36
    parameters, 34 free): the streamed server evaluates every active fit's MC
    sums over the shared sample in one walk per tick (batched), against the
    same server one fit at a time. The toys are generated on the device and
    stay there: each is submitted in place (events_on_device), so submission
    copies nothing (host arrays would be copied twice, to the host and back,
    which at ~1 ms per toy was what limited the all-at-once runs)."""
    rng = np.random.default_rng(501)
    nf = args.fits
    sizes = np.rint(np.exp(rng.uniform(math.log(5e3), math.log(5e5), nf))).astype(np.int64)
    arrivals = np.cumsum(rng.exponential(1.0 / 200.0, nf))
    jit = rng.uniform(-0.002, 0.002, (nf, 2))
    ix, iy = I.theta_index(model, "x"), I.theta_index(model, "y")
    nc = len(model["comp_a"]) + len(model["comp_ab"])
    scale = np.zeros(I.n_theta(model))
    scale[:2 * nc] = 0.05
    j = len(model["comp_a"]) + model["comp_ab"].index(5)
    scale[2 * j:2 * j + 2] = 0.0
    scale[ix] = scale[iy] = 1e-3
    shape = [model[k] for k in ("m_ks", "g_ks", "m_rho", "g_rho", "m_a1", "g_a1")]
    # toy data from the generator; |A|^2 + |Abar|^2 does not depend on x, y,
    # so one envelope serves every toy
    t0 = time.perf_counter()
    gen = M.Context(model, device=0)
    _, _, st0 = gen.draw_data(theta, 1000, seed=500)
    env = st0["envelope"]
    toys = []
    for i in range(nf):
        th = theta.copy()
        th[ix] += jit[i, 0]
        th[iy] += jit[i, 1]
        gen.set_params(th)
        p4, t, _, st = gen.generate(M.MXA_DATA, int(sizes[i]), seed=10_000 + i, envelope=env)
        if st["n_exceed"]:
            raise RuntimeError("toy envelope exceeded")
        toys.append((p4, t))  # left on the device: submitted in place
    gen.close()
    t_gen = time.perf_counter() - t0
    log(f"[bench] {nf} toys, {int(sizes.sum())} data events generated in {t_gen:.1f} s")

    xy_only = np.zeros_like(scale)
    xy_only[ix] = xy_only[iy] = 1e-3

    floating = scale.copy()
    for k in ("m_ks", "g_ks", "m_rho", "g_rho", "m_a1", "g_a1"):
        floating[I.theta_index(model, k)] = 2e-3

    def run(max_slots, budget, sc=scale, streamed=False, burst=False, prec="fp64", cap=500):
        with M.Server(model, mc_host, None if streamed else shape, precision=prec,
                      max_slots=max_slots, hbm_budget=budget) as srv:
            tickets = []
            t_start = time.perf_counter()
            for i in range(nf):
                dly = t_start + arrivals[i] - time.perf_counter()
                if dly > 0 and not burst:
                    time.sleep(dly)
                tickets.append(srv.submit(toys[i][0], toys[i][1], theta, sc, max_evals=cap,
                                          edm_tol=1e-4))
            res = [srv.wait(tk, release=True) for tk in tickets]
            st = srv.stats()
        out = _latency_stats(res)
        if not streamed:
            # the Gram-mode evaluation reads the fits' bases and decay times
            # only: 16 values (B_k of the eight chains) + the time per event
            rec_bytes = 16 * (8 if prec == "fp64" else 4) + 8
            out["hbm_frac"] = out["events_per_s"] * rec_bytes / (HBM_PEAK_GBS * 1e9)
        out.update(max_slots=max_slots, hbm_budget_mb=budget / 2 ** 20, precision=prec,
                   eval_cap=cap, free_parameters=int((sc > 0).sum()), floating_shapes=streamed,
                   arrivals="all at once" if burst else "Poisson 200/s",
                   hbm_peak_mb=st["hbm_peak"] / 2 ** 20, active_peak=st["active_peak"])
        log(f"[bench] serving slots={max_slots} budget={budget / 2**20:.0f} MB "
            f"free={int((sc > 0).sum())}{' streamed MC' if streamed else ''}"
            f"{' burst' if burst else ''}: "
            f"p50 {out['p50_ms']:.1f} ms, p99 {out['p99_ms']:.1f} ms, {out['fits_per_s']:.1f} fits/s, "
            f"{out['events_per_s']:.3g} events/s, {out['evals_mean']:.0f} evaluations per fit, "
            f"{out['converged']} converged, {out['max_evals']} capped, queue p50 "
            f"{out['queue_p50_ms']:.1f} ms, peak {out['active_peak']} fits / {out['hbm_peak_mb']:.0f} MB")
        return out

    return {"fits": nf, "arrival_rate_per_s": 200.0, "events_mean": float(sizes.mean()),
            "events_median": float(np.median(sizes)), "n_mc": int(mc_host.shape[0]),
            "precision": "fp64", "free_parameters": int((scale > 0).sum()),
            "toy_generation_s": t_gen,
            "batched": run(64, 8 << 30), "budget_256MB": run(64, 256 << 20),
            "one_at_a_time": run(1, 8 << 30),
            "burst_batched": run(64, 8 << 30, burst=True),
            "burst_budget_256MB": run(64, 256 << 20, burst=True),
            "burst_one_at_a_time": run(1, 8 << 30, burst=True),
            "fp32amp_batched": run(64, 8 << 30, prec="fp32amp", cap=1000),
            # the paper's own toy study: amplitude model fixed, x and y float
            "xy_only_batched": run(64, 8 << 30, xy_only, prec="fp32amp"),
            "xy_only_one_at_a_time": run(1, 8 << 30, xy_only, prec="fp32amp"),
            # masses and widths floating: the shared MC streamed once per tick
            "floating_shapes_batched": run(64, 8 << 30, floating, True, prec="fp32amp"),
            "floating_shapes_one_at_a_time": run(1, 8 << 30, floating, True, prec="fp32amp")}


def streamed_ticks(M, model, theta, ctx_gen, env, mc_host, ks, precisions, single_us):
    """Fits with the masses and widths floating (34 free parameters) on the
    streamed server, which evaluates all active fits' MC sums in one walk over
    the shared 4M-event MC sample per tick: with K slots, 3K fits of 50,000
    events each, 150 evaluations each (no early stop), so K fits are active
    in almost every tick. Time per tick and per fit evaluation (first
    admission to last result), against one single-context NLL+gradient
    evaluation of the same sizes (the headline step)."""
    samples = []
    for k in range(8):
        p4, t, _, _ = ctx_gen.generate(M.MXA_DATA, 50_000, seed=2_000_000 + k, envelope=env)
        samples.append((p4.cpu().numpy().reshape(-1, 16), t.cpu().numpy()))
    sc = np.zeros(I.n_theta(model))
    nc = len(model["comp_a"]) + len(model["comp_ab"])
    sc[:2 * nc] = 0.05
    j = len(model["comp_a"]) + model["comp_ab"].index(5)
    sc[2 * j:2 * j + 2] = 0.0
    sc[I.theta_index(model, "x")] = sc[I.theta_index(model, "y")] = 1e-3
    for k in ("m_ks", "g_ks", "m_rho", "g_rho", "m_a1", "g_a1"):
        sc[I.theta_index(model, k)] = 2e-3
    out = {"n_data": 50_000, "n_mc": int(mc_host.shape[0]), "free_parameters": int((sc > 0).sum()),
           "evaluations_per_fit": 150, "points": []}
    for prec in precisions:
        for K in ks:
            with M.Server(model, mc_host, None, precision=prec, max_slots=K) as srv:
                srv.wait(srv.submit(*samples[0], theta, sc, max_evals=5))  # graph capture
                s0 = srv.stats()
                tks = [srv.submit(*samples[i % 8], theta, sc, max_evals=150, gtol=1e-12)
                       for i in range(3 * K)]
                res = [srv.wait(tk) for tk in tks]
                s1 = srv.stats()
            span = (max(r["t_done_ns"] for r in res) - min(r["t_start_ns"] for r in res)) * 1e-9
            ev, ticks = s1["evals"] - s0["evals"], s1["ticks"] - s0["ticks"]
            rec = {"precision": prec, "slots": K, "fits": len(res), "evaluations": ev, "ticks": ticks,
                   "us_per_tick": span / ticks * 1e6, "us_per_fit_evaluation": span / ev * 1e6,
                   "single_context_us": single_us[prec],
                   "speedup_vs_single_context": single_us[prec] / (span / ev * 1e6)}
            out["points"].append(rec)
            log(f"[bench] streamed server {prec} K={K}: {rec['us_per_tick']:.1f} us/tick, "
                f"{rec['us_per_fit_evaluation']:.1f} us per fit evaluation "
                f"({rec['speedup_vs_single_context']:.2f}x one evaluation alone)")
    return out


def fit_time(M, model, theta, ctx_gen, mc_dev, sync, reps=3):
    """The paper's fit-time benchmark (Sec. 5, Table 3): one fit to 100,000
    pseudo-events with 0.75M, 1.5M, 3M and 6M normalisation points, the
    amplitude model fixed and x, y floating, started at x = y = 0, stopped
    at an estimated distance to the minimum below 1e-4 and followed by the
    error (Hessian) evaluations. Wall time of mxa_fit with the samples
    resident in HBM (the per-event cache built at load, not timed), median of
    `reps` fits: MC streamed at every evaluation (direct, FP32 amplitudes and
    FP64), and the normalisation through the MC Gram matrix (its build at the
    first evaluation included)."""
    ix, iy = I.theta_index(model, "x"), I.theta_index(model, "y")
    d4, dt, _ = ctx_gen.draw_data(theta, 100_000, seed=777)
    start = theta.copy()
    start[ix] = start[iy] = 0.0
    sc = np.zeros(I.n_theta(model))
    sc[ix] = sc[iy] = 1e-3
    out = {"n_data": 100_000, "free": ["x", "y"], "start": "x = y = 0", "stop": "edm < 1e-4",
           "errors": True, "points": {}}
    with M.Context(model, device=0) as c:
        c.load_events_device(M.MXA_DATA, d4, dt)
        for n_mc in (750_000, 1_500_000, 3_000_000, 6_000_000):
            rec = {}
            for name, prec, mode in (("direct_fp32amp", "fp32amp", M.MXA_MC_DIRECT),
                                     ("direct_fp64", "fp64", M.MXA_MC_DIRECT),
                                     ("gram_fp64", "fp64", M.MXA_MC_GRAM)):
                c.set_mc_mode(mode)
                times, res = [], None
                for _ in range(reps):
                    c.load_events_device(M.MXA_MC, mc_dev[:n_mc])  # invalidates the Gram matrix
                    sync()
                    t0 = time.perf_counter()
                    res = c.fit(start, sc, precision=prec, max_evals=100, gtol=1e-12, edm_tol=1e-4,
                                errors=True)
                    times.append(time.perf_counter() - t0)
                rec[name] = {"seconds": float(np.median(times)), "evaluations": res["n_evals"],
                             "status": res["status"], "x": res["theta"][ix], "y": res["theta"][iy],
                             "err_x": res["err"][ix], "err_y": res["err"][iy]}
            out["points"][str(n_mc)] = rec
            log(f"[bench] fit, 100k events, {n_mc} points: "
                + ", ".join(f"{k} {v['seconds'] * 1e3:.1f} ms ({v['evaluations']} evals)"
                            for k, v in rec.items()))
    return out


def coefficient_scales(model, with_shapes=False):
    """Step scales of the fits with every coefficient free except Abar_f's a1
    S-wave one (fixed: the NLL does not change under a common complex scale
    of all coefficients), x, y free; masses and widths too if asked."""
    sc = np.zeros(I.n_theta(model))
    nc = len(model["comp_a"]) + len(model["comp_ab"])
    sc[:2 * nc] = 0.05
    j = len(model["comp_a"]) + model["comp_ab"].index(5)
    sc[2 * j:2 * j + 2] = 0.0
    sc[I.theta_index(model, "x")] = sc[I.theta_index(model, "y")] = 1e-3
    if with_shapes:
        for k in ("m_ks", "g_ks", "m_rho", "g_rho", "m_a1", "g_a1"):
            sc[I.theta_index(model, k)] = 2e-3
    return sc


def full_fit(M, model, theta, ctx, sync):
    """The full plain fit (50,000 data / 4M MC, 28 free parameters: every
    coefficient but one, x and y) from the generating point to convergence
    (estimated distance to the minimum below 1e-4, at most 300 gradient
    evaluations): with the adjoint gradient (FP32 amplitudes and FP64, MC
    streamed) and with numerical gradients, central differences of FP64 NLL
    values (Sec. 5: the paper's fits are numerically differentiated), in
    Gram mode all 57 points of a gradient in one many-set call and in direct
    mode one MC pass per point. Wall time of mxa_fit, gradient evaluations
    and NLL points."""
    sc = coefficient_scales(model)
    out = {"n_data": ctx.sample_size(M.MXA_DATA), "n_mc": ctx.sample_size(M.MXA_MC),
           "free_parameters": int((sc > 0).sum()), "runs": {}}
    for name, prec, mode, central in (("adjoint_fp32amp", "fp32amp", M.MXA_MC_DIRECT, False),
                                      ("adjoint_fp64", "fp64", M.MXA_MC_DIRECT, False),
                                      ("central_fp64_gram", "fp64", M.MXA_MC_GRAM, True),
                                      ("central_fp64_direct", "fp64", M.MXA_MC_DIRECT, True)):
        ctx.set_mc_mode(mode)
        sync()
        t0 = time.perf_counter()
        r = ctx.fit(theta, sc, precision=prec, max_evals=300, gtol=1e-12, edm_tol=1e-4,
                    central=central)
        dt = time.perf_counter() - t0
        out["runs"][name] = {"seconds": dt, "status": r["status"], "evaluations": r["n_evals"],
                             "nll_points": r["n_points"], "nll": r["nll"],
                             "x": r["theta"][I.theta_index(model, "x")],
                             "y": r["theta"][I.theta_index(model, "y")]}
        log(f"[bench] full fit {name}: {dt * 1e3:.1f} ms, {r['n_evals']} evaluations, "
            f"{r['n_points']} NLL points, {r['status']}, NLL {r['nll']:.4f}")
    ctx.set_mc_mode(M.MXA_MC_DIRECT)
    ctx.set_params(theta)
    return out


def differentiation_form(M, model, theta, mc_dev, sync, reps=20):
    """Time per minimiser step at 1,000,000 data / 4,000,000 MC events with 36
    parameters: one adjoint NLL+gradient evaluation (FP32 amplitudes, FP64)
    against a gradient by central differences of FP64 NLL values, 73 points
    (one evaluation each), and against the Gram-mode form where the 61 points
    of the coefficients and x, y share one many-set call and the 12 points
    of the masses and widths take an evaluation each."""
    W = I.WORKLOADS["gradient"]
    out = {"n_data": W.n_data, "n_mc": W.n_mc, "parameters": I.n_theta(model)}
    with M.Context(model, device=0) as c:
        d4, dt, _ = c.draw_data(theta, W.n_data, W.seed_data)
        c.load_events_device(M.MXA_DATA, d4, dt)
        c.load_events_device(M.MXA_MC, mc_dev)
        del d4, dt
        c.set_params(theta)
        nt = I.n_theta(model)
        h = 1e-4 * np.maximum(coefficient_scales(model, True), 1e-3)
        pts = np.tile(theta, (2 * nt + 1, 1))
        for j in range(nt):
            pts[1 + 2 * j, j] += h[j]
            pts[2 + 2 * j, j] -= h[j]
        nstd = 2 * (len(model["comp_a"]) + len(model["comp_ab"])) + 2

        def central_direct():
            for q in pts:
                c.set_params(q)
                c.nll("fp64")

        def central_gram():
            c.set_mc_mode(M.MXA_MC_GRAM)
            c.nll_multi(pts[:2 * nstd + 1], "fp64")
            c.set_mc_mode(M.MXA_MC_DIRECT)
            for q in pts[2 * nstd + 1:]:
                c.set_params(q)
                c.nll("fp64")

        forms = (("adjoint_fp32amp", lambda: c.nll_grad("fp32amp")),
                 ("adjoint_fp64", lambda: c.nll_grad("fp64")),
                 ("central_fp64_73_points", central_direct),
                 ("central_fp64_gram_61_sets_plus_12_points", central_gram))
        for name, f in forms:
            c.set_params(theta)
            for _ in range(3):
                f()
            sync()
            t0 = time.perf_counter()
            for _ in range(reps):
                c.set_params(theta)
                f()
            sync()
            out[name + "_ms"] = (time.perf_counter() - t0) / reps * 1e3
        out["adjoint_speedup_vs_central_fp64"] = (out["central_fp64_73_points_ms"]
                                                 / out["adjoint_fp64_ms"])
        log("[bench] differentiation form: " + ", ".join(
            f"{k} {v:.4g}" for k, v in out.items() if k.endswith("_ms")))
    return out


def precision_form(M, model, theta, sync, with_oracle):
    """The precision form, 10,000,000 data / 50,000,000 MC events: the NLL+
    gradient step time in both precisions, and x, y fitted (model fixed, MC
    streamed, estimated distance below 1e-4) with FP32 amplitudes and in
    FP64, their difference in units of the FP64 fit's errors, and the
    oracle's NLL at the FP64-fitted point against the library's."""
    W = I.WORKLOADS["precision"]
    ix, iy = I.theta_index(model, "x"), I.theta_index(model, "y")
    sc = np.zeros(I.n_theta(model))
    sc[ix] = sc[iy] = 1e-3
    out = {"n_data": W.n_data, "n_mc": W.n_mc}
    with M.Context(model, device=0) as c:
        mc, _, _, _ = c.generate(M.MXA_MC, W.n_mc, W.seed_mc)
        c.load_events_device(M.MXA_MC, mc)
        d4, dt, _ = c.draw_data(theta, W.n_data, W.seed_data)
        c.load_events_device(M.MXA_DATA, d4, dt)
        c.set_params(theta)
        for prec in ("fp32amp", "fp64"):
            for _ in range(3):
                c.nll_grad(prec)
            sync()
            t0 = time.perf_counter()
            for _ in range(10):
                c.nll_grad(prec)
            out[f"{prec}_grad_ms"] = (time.perf_counter() - t0) / 10 * 1e3
            out[f"{prec}_events_per_s"] = (W.n_data + W.n_mc) / (out[f"{prec}_grad_ms"] * 1e-3)
        fits = {}
        for prec in ("fp32amp", "fp64"):
            r = c.fit(theta, sc, precision=prec, max_evals=100, gtol=1e-12, edm_tol=1e-4,
                      errors=True)
            fits[prec] = r
        a, b = fits["fp32amp"], fits["fp64"]
        out["fit"] = {p: {"x": r["theta"][ix], "y": r["theta"][iy], "err_x": r["err"][ix],
                          "err_y": r["err"][iy], "nll": r["nll"], "evaluations": r["n_evals"],
                          "status": r["status"]} for p, r in fits.items()}
        out["dx_over_sigma"] = abs(a["theta"][ix] - b["theta"][ix]) / b["err"][ix]
        out["dy_over_sigma"] = abs(a["theta"][iy] - b["theta"][iy]) / b["err"][iy]
        log(f"[bench] precision form: FP32-amp {out['fp32amp_grad_ms']:.2f} ms, FP64 "
            f"{out['fp64_grad_ms']:.2f} ms per NLL+grad; fitted x, y differ by "
            f"{out['dx_over_sigma']:.2e} / {out['dy_over_sigma']:.2e} sigma")
        if with_oracle:
            import oracle
            th64 = b["theta"]
            c.set_params(th64)
            v64 = c.nll("fp64")
            pd, td, pm = d4.cpu().numpy(), dt.cpu().numpy(), mc.cpu().numpy()
            del d4, dt, mc
            t0 = time.perf_counter()
            ref, _, _, S = oracle.nll(model, th64, pd, td, pm, diag=True)
            out["oracle_at_fp64_fit"] = {"oracle_nll": ref, "gpu_fp64_nll": v64,
                                         "nll_rel": abs(v64 - ref) / abs(ref),
                                         "nll_over_S": abs(v64 - ref) / S,
                                         "oracle_seconds": time.perf_counter() - t0}
            log(f"[bench] precision form: oracle NLL at the FP64-fitted point {ref:.10g}, GPU "
                f"{v64:.10g}, relative {abs(v64 - ref) / abs(ref):.2e}")
    return out


def sensitivity(M, model, theta, mc_host, ctx_gen, toys_per_size):
    """The paper's sensitivity study (Sec. 4, Table 1) through the fit server:
    toys of 20,000, 50,000 and 70,000 pseudo-events generated by the library
    at x = 0.49%, y = 0.61% (amplitude model fixed), each fitted in x and y
    (FP64, shared 4M-event MC through its Gram matrix) with errors from the
    Hessian. Per size: the spread of the fitted x, y over the toys (the
    statistical sensitivity), the mean fitted error, the pulls
    (fitted - true) / error, and sigma * sqrt(N)."""
    ix, iy = I.theta_index(model, "x"), I.theta_index(model, "y")
    sc = np.zeros(I.n_theta(model))
    sc[ix] = sc[iy] = 1e-3
    shape = [model[k] for k in ("m_ks", "g_ks", "m_rho", "g_rho", "m_a1", "g_a1")]
    _, _, st0 = ctx_gen.draw_data(theta, 1000, seed=600)
    env = st0["envelope"]
    ctx_gen.set_params(theta)
    t0 = time.perf_counter()
    out = {"toys_per_size": toys_per_size, "precision": "fp64", "n_mc": int(mc_host.shape[0]),
           "x_true": theta[ix], "y_true": theta[iy], "sizes": {}}
    with M.Server(model, mc_host, shape, precision="fp64", max_slots=64) as srv:
        for n in (20_000, 50_000, 70_000):
            tickets = []
            for k in range(toys_per_size):
                p4, t, _, st = ctx_gen.generate(M.MXA_DATA, n, seed=1_000_000 + 1000 * (n // 1000) + k,
                                                envelope=env)
                if st["n_exceed"]:
                    raise RuntimeError("toy envelope exceeded")
                # the toy stays on the device: submitted in place
                tickets.append(srv.submit(p4, t, theta, sc, max_evals=100, gtol=1e-6, errors=True))
            res = [srv.wait(tk, release=True) for tk in tickets]
            ok = [r for r in res if r["status"] == "converged" and r["errors_ok"]]
            rec = {"fits": len(res), "converged_with_errors": len(ok)}
            for name, j in (("x", ix), ("y", iy)):
                v = np.array([r["theta"][j] for r in ok])
                e = np.array([r["err"][j] for r in ok])
                pull = (v - theta[j]) / e
                m = len(v)
                rec[name] = {"sigma_pct": 100 * float(v.std(ddof=1)),
                             "sigma_pct_stat_err": 100 * float(v.std(ddof=1)) / math.sqrt(2 * (m - 1)),
                             "mean_error_pct": 100 * float(e.mean()),
                             "bias_pct": 100 * float(v.mean() - theta[j]),
                             "pull_mean": float(pull.mean()),
                             "pull_mean_err": float(pull.std(ddof=1) / math.sqrt(m)),
                             "pull_width": float(pull.std(ddof=1)),
                             "pull_width_err": float(pull.std(ddof=1) / math.sqrt(2 * (m - 1))),
                             "sigma_sqrt_n": float(v.std(ddof=1)) * math.sqrt(n)}
            out["sizes"][str(n)] = rec
            log(f"[bench] sensitivity {n}: sigma(x) {rec['x']['sigma_pct']:.4f}%, "
                f"sigma(y) {rec['y']['sigma_pct']:.4f}%, pulls x {rec['x']['pull_mean']:+.2f} / "
                f"{rec['x']['pull_width']:.2f}, y {rec['y']['pull_mean']:+.2f} / {rec['y']['pull_width']:.2f}")
    out["seconds"] = time.perf_counter() - t0
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=1000,
                    help="untimed steps of every form before any is timed")
    ap.add_argument("--workload", default="full", choices=["full", "gradient", "small"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="least CPU time the oracle baseline accumulates")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the toy-fit serving measurement")
    ap.add_argument("--fits", type=int, default=512, help="toy fits in the serving measurement")
    ap.add_argument("--no-fits", action="store_true",
                    help="skip the full-fit, differentiation-form, fit-time and sensitivity "
                         "measurements")
    ap.add_argument("--no-precision-form", action="store_true",
                    help="skip the 10M / 50M precision form")
    ap.add_argument("--toys", type=int, default=100,
                    help="toys per sample size in the sensitivity measurement")
    ap.add_argument("--streamed-ks", default="1,4,16",
                    help="slot counts of the streamed-server measurement ('' skips it)")
    ap.add_argument("--streamed-precisions", default="fp32amp,fp64")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; run with --gpus 1"}))
        sys.exit(2)

    import torch
    from paper_1702_06735_amd import mixamp as M
    M.load_library()

    W = I.WORKLOADS[args.workload]
    model = W.model
    theta = I.make_theta(model, I.draw_coefficients(model, W.seed_coeff))
    ctx = M.Context(model, device=0)
    # inputs from the library's generator (GENBOD + accept-reject by Eq. (1)),
    # left on the device
    sync = torch.cuda.synchronize
    ctx.generate(M.MXA_MC, 1000, 1)          # first call allocates the scratch
    sync()
    t0 = time.perf_counter()
    mc, _, _, mc_st = ctx.generate(M.MXA_MC, W.n_mc, W.seed_mc)
    sync()
    t_mc = time.perf_counter() - t0
    d4, dt, d_st = ctx.draw_data(theta, W.n_data, W.seed_data)
    env = d_st["envelope"]
    # pseudo-experiments of the sizes of the paper's generation benchmark
    # (Sec. 5, Table 2), envelope known
    table2 = {}
    for n in (20_000, 50_000, 70_000):
        sync()
        t0 = time.perf_counter()
        _, _, _, st = ctx.generate(M.MXA_DATA, n, W.seed_data + n, envelope=env)
        sync()
        table2[str(n)] = {"seconds": time.perf_counter() - t0, "candidates": st["n_candidates"]}
    log(f"[bench] generated {W.n_mc} MC events in {t_mc * 1e3:.1f} ms; pseudo-data "
        + ", ".join(f"{k}: {v['seconds'] * 1e3:.1f} ms" for k, v in table2.items()))
    generation = {"mc_events_per_s": W.n_mc / t_mc,
                  "mc_candidates_per_s": mc_st["n_candidates"] / t_mc,
                  "data_acceptance": W.n_data / d_st["n_candidates"],
                  "pseudo_data_seconds": table2}

    ctx.load_events_device(M.MXA_MC, mc)
    ctx.load_events_device(M.MXA_DATA, d4, dt)
    ctx.set_params(theta)
    n_ev = W.n_data + W.n_mc

    forms = (("fp32amp_grad", lambda: ctx.nll_grad("fp32amp")),
             ("fp64_grad", lambda: ctx.nll_grad("fp64")),
             ("fp32amp_nll", lambda: ctx.nll("fp32amp")),
             ("fp64_nll", lambda: ctx.nll("fp64")))
    # every form warms up before any is timed: the first seconds of sustained
    # load on a fresh device show one-off stalls of tens of milliseconds
    for _, f in forms:
        for _ in range(args.warmup):
            f()
    sync()
    results = {}
    for name, f in forms:
        st = timed_steps(ctx, f, args.steps, sync)
        results[name] = st
        log(f"[bench] {name}: {st.mean_s * 1e6:.1f} us/step (median {st.median_s * 1e6:.1f}, "
            f"p99 {st.p99_s * 1e6:.1f}), kernel {st.kernel_ms * 1e3:.1f} us, "
            f"{n_ev / st.mean_s:.3e} events/s")

    # dense forms on the matrix cores: the MC Gram matrix (fixed lineshapes)
    # and many parameter sets at once (a 61-point stencil around theta, one
    # data pass for all sets, the normalisation from the Gram matrix)
    dense = {}
    for prec in ("fp64", "fp32amp"):
        for _ in range(3):
            ctx.gram(prec)
        sync()
        t0 = time.perf_counter()
        for _ in range(20):
            ctx.gram(prec)
        sync()
        dense[f"gram_{prec}_ms"] = (time.perf_counter() - t0) / 20 * 1e3
    rng = np.random.default_rng(61)
    sets = np.tile(theta, (61, 1))
    nc2 = 2 * (len(model["comp_a"]) + len(model["comp_ab"]))
    sets[:, :nc2 + 2] += 1e-3 * rng.standard_normal((61, nc2 + 2))
    for prec in ("fp64", "fp32amp"):
        for _ in range(20):
            ctx.nll_multi(sets, prec)
        sync()
        t0 = time.perf_counter()
        for _ in range(100):
            ctx.nll_multi(sets, prec)
        sync()
        dt_m = (time.perf_counter() - t0) / 100
        dense[f"multi61_{prec}_us"] = dt_m * 1e6
        dense[f"multi61_{prec}_event_sets_per_s"] = W.n_data * 61 / dt_m
    log("[bench] dense forms: " + ", ".join(f"{k} {v:.4g}" for k, v in dense.items()))

    # the model with a background component (fraction 0.1 of the same data):
    # MC pass, its reduction, then the data pass with Nhat known
    mb = I.with_background(model)
    with M.Context(mb, device=0) as cb:
        cb.load_events_device(M.MXA_MC, mc)
        cb.load_events_device(M.MXA_DATA, d4, dt)
        cb.set_params(np.concatenate([theta, [0.1]]))
        bforms = (("fp32amp_grad", lambda: cb.nll_grad("fp32amp")),
                  ("fp64_grad", lambda: cb.nll_grad("fp64")))
        background = {}
        for name, f in bforms:
            for _ in range(min(args.warmup, 200)):
                f()
            st = timed_steps(cb, f, min(args.steps, 200), sync)
            background[name] = {"events_per_s": n_ev / st.mean_s, "us_per_step": st.mean_s * 1e6,
                                "us_per_step_median": st.median_s * 1e6,
                                "mc_kernel_us": st.kernel_ms * 1e3}
            log(f"[bench] background {name}: {st.mean_s * 1e6:.1f} us/step, "
                f"MC kernel {st.kernel_ms * 1e3:.1f} us")

    # the model with CP violation in mixing: the same data split into D0 and
    # D0bar tags (the second half handed over as D0bar records), q/p =
    # 1.05 exp(0.1 i): two flavours, each one evaluation of the model
    # without CP violation
    mcp = I.with_cp_violation(model)
    half = W.n_data // 2
    with M.Context(mcp, device=0) as cc:
        cc.load_events_device(M.MXA_MC, mc)
        cc.load_events_device(M.MXA_DATA, d4[:half], dt[:half])
        bar = d4[half:].clone()
        bar[..., 1:] = -bar[..., 1:]
        cc.load_events_device(M.MXA_DATA_BAR, bar, dt[half:].contiguous())
        cc.set_params(np.concatenate([theta, [1.05, 0.1]]))
        for name, f in (("fp32amp_grad", lambda: cc.nll_grad("fp32amp")),
                        ("fp64_grad", lambda: cc.nll_grad("fp64"))):
            for _ in range(min(args.warmup, 200)):
                f()
            st = timed_steps(cc, f, min(args.steps, 200), sync)
            background["cpv_" + name] = {"events_per_s": n_ev / st.mean_s,
                                         "us_per_step": st.mean_s * 1e6,
                                         "us_per_step_median": st.median_s * 1e6,
                                         "mc_kernel_us": st.kernel_ms * 1e3}
            log(f"[bench] CP violation {name}: {st.mean_s * 1e6:.1f} us/step")

    # mxa_nll_multi leaves the context at its first set: back to theta, the
    # point the oracle evaluates
    ctx.set_params(theta)
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

    head = results["fp32amp_grad"]
    # the dominant kernel is the launch of both adjoint passes; its algorithmic
    # bytes are the 21-value records of every event (FP32: 84 B per MC event,
    # 88 B per data event)
    alg = algorithmic_bytes(W.n_data, W.n_mc, 4)
    alg64 = algorithmic_bytes(W.n_data, W.n_mc, 8)
    achieved = alg / (head.kernel_ms * 1e-3) / 1e9
    traffic = read_traffic()
    k64 = results["fp64_grad"]
    out = {
        "metric": METRIC,
        "value": n_ev / head.mean_s,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head.mean_s * 1e3,
        "ms_per_step_median": head.median_s * 1e3,
        "ms_per_step_p99": head.p99_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 amplitudes + f64 mixing/logs/sums",
        "data": "synthetic (the library's seeded GENBOD generator; pseudo-data by accept-reject from the model)",
        "config": {"workload": f"{W.name}: fourteen-chain model, NLL+gradient (36 parameters), "
                               f"{W.n_data} data + {W.n_mc} MC events",
                   "n_data": W.n_data, "n_mc": W.n_mc, "precision": "fp32amp"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "algorithmic_bytes": alg,
                     "traffic_over_algorithmic": traffic / alg if traffic else None,
                     "kernel": HEADLINE_KERNEL,
                     "kernel_us_median": head.kernel_ms * 1e3,
                     "frac_step": alg / head.median_s / 1e9 / HBM_PEAK_GBS,
                     "fp64": {"algorithmic_bytes": alg64, "kernel_us_median": k64.kernel_ms * 1e3,
                              "frac": alg64 / (k64.kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              "frac_step": alg64 / k64.median_s / 1e9 / HBM_PEAK_GBS},
                     "valu": read_utilisation(HEADLINE_KERNEL)},
        "kernel_us": head.kernel_ms * 1e3,
        "forms": {k: st.summary(n_ev) for k, st in results.items()},
        "error": err,
        "extension_forms": background,
        "dense_forms": dense,
    }
    out["generation"] = generation
    mc_host = mc.cpu().numpy().reshape(-1, 16)
    if args.streamed_ks:
        try:
            out["streamed_server"] = streamed_ticks(
                M, model, theta, ctx, env, mc_host, [int(v) for v in args.streamed_ks.split(",")],
                args.streamed_precisions.split(","),
                {"fp32amp": results["fp32amp_grad"].mean_s * 1e6, "fp64": results["fp64_grad"].mean_s * 1e6})
            ctx.set_params(theta)
        except Exception as e:  # reported, not fatal to the headline
            out["streamed_server"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_fits:
        try:
            out["full_fit"] = full_fit(M, model, theta, ctx, sync)
            out["differentiation_form"] = differentiation_form(M, model, theta, mc, sync)
            mc6, _, _, _ = ctx.generate(M.MXA_MC, 6_000_000, W.seed_mc + 1)
            out["fit_time"] = fit_time(M, model, theta, ctx, mc6, sync)
            del mc6
            out["sensitivity"] = sensitivity(M, model, theta, mc_host, ctx, args.toys)
        except Exception as e:  # reported, not fatal to the headline
            out["fits_error"] = f"{type(e).__name__}: {e}"
    if not args.no_precision_form:
        try:
            out["precision_form"] = precision_form(M, model, theta, sync,
                                                   with_oracle=not args.no_cpu_baseline)
        except Exception as e:  # reported, not fatal to the headline
            out["precision_form"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_serving:
        try:
            out["serving"] = serving(M, model, theta, mc_host, args)
        except Exception as e:  # reported, not fatal to the headline
            out["serving"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_cpu_baseline:
        log("[bench] oracle baseline on the host")
        out["cpu_baseline"], ref = cpu_baseline(model, theta, d4.cpu().numpy(), dt.cpu().numpy(),
                                                mc_host, args.cpu_seconds)
        out["error_vs_oracle"] = errors_vs_oracle(ref, {"fp32amp": (v32, g32), "fp64": (v64, g64)})
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
