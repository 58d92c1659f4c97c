"""Throughput of the batched Galactic-binary likelihood on one MI355X.

One step = one pass of the hot path over the ragged batch: the Metropolis-Hastings stage of
every window in one call (logL of every proposal, one persistent launch per (N, C, precision)
bucket, then the chain of every window in one launch) and the gradient of every candidate (one
persistent launch per (N, C) group).  Inputs are synthetic and resident
in HBM before the timed region.  Prints ONE JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--windows 256] [--cands 10000]
"""

from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GB logL evals/s + grad evals/s (ragged, mixed prec) vs plain FP64 on same GPU"
PEAK_VALU_TFLOPS = 78.6     # MI355X vector FMA rate (FP64, and FP32 without packed math)
PEAK_HBM_GBS = 8000.0
COPY_N = 1 << 28            # copy calibration: 256 M doubles = 2 GiB read + 2 GiB written per launch
N_SIMD = 256 * 4            # MI355X: 256 compute units of 4 SIMDs
SQ_COUNTERS = ("SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY",
               "SQ_ACTIVE_INST_ANY", "SQ_ACTIVE_INST_VALU", "SQ_INSTS_VALU")
# a second pass (eight SQ counters per rocprofv3 --pmc run): LDS instructions and their stalls
LDS_COUNTERS = ("SQ_WAVES", "SQ_INSTS_LDS", "SQ_ACTIVE_INST_LDS", "SQ_LDS_IDX_ACTIVE", "SQ_LDS_BANK_CONFLICT",
                "SQ_LDS_ADDR_CONFLICT", "SQ_LDS_UNALIGNED_STALL", "SQ_WAIT_INST_LDS")


# ------------------------------------------------------------------------------------------
# algorithmic work per evaluation: floating-point operations of the executed code path per
# sample, counted from the gfx950 assembly of the kernels (one FMA = 2 flops), with the sin/cos
# evaluations counted separately, not as flops; the DFT at the usual 5 N log2 N per channel
def flops_per_eval(N: int, C: int, overlap: int, grad: bool) -> float:
    per_sample = 324.0 + (10.0 if C == 3 else 0.0)          # slow series (response, TDI, channels)
    fft = C * 5.0 * N * math.log2(N)                          # one radix-2-equivalent DFT per channel
    red = 20.0 * C * overlap                                  # residual and four FP64 accumulations
    f = per_sample * N + fft + red
    if grad:
        f += fft + 825.0 * N + 6.0 * C * overlap              # inverse DFT, per-sample adjoint, cotangent
    return f


def sincos_per_eval(N: int, grad: bool) -> float:
    # carrier, D and two spacecraft phases per sample; the adjoint recomputes the same four
    return (4.0 + (4.0 if grad else 0.0)) * N


def bytes_per_eval(C: int, overlap: int, grad: bool) -> float:
    """Algorithmic HBM bytes per evaluation: theta in, logL (+ gradient) out; the window data
    and weights (24 B per bin and channel) are shared by all candidates of a window and
    counted once per window separately."""
    return 64.0 + 8.0 + (64.0 if grad else 16.0)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--windows", type=int, default=256)
    ap.add_argument("--cands", type=int, default=10000)
    ap.add_argument("--temperature", type=float, default=1.0)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--rho-mixed", type=float, default=8.0)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-posterior", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the throughput of C1, C2, C4 and C5")
    ap.add_argument("--posterior-sources", type=int, default=3)
    ap.add_argument("--no-pipeline", action="store_true")
    ap.add_argument("--pipeline-segments", type=int, nargs=2, default=(2000, 3000), metavar=("FIRST", "END"),
                    help="the contiguous block of the 4000 full-band segments that the pipeline leg analyses")
    ap.add_argument("--pipeline-full", action="store_true", help="the pipeline leg over all 4000 segments")
    ap.add_argument("--pipeline-only", action="store_true", help="run the pipeline leg alone and print its JSON")
    ap.add_argument("--pipeline-catalogue", metavar="NPZ",
                    help="also write the pipeline's catalogue (recovered parameters, their segment, delta, "
                         "matched injection; the injected set with optimal SNRs; posterior samples' mean and "
                         "standard deviation) to this .npz file")
    ap.add_argument("--traffic", nargs=4, metavar=("K_FETCH_DIR", "K_WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="print the profiles/hbm_traffic.txt line from rocprofv3 --pmc outputs and exit")
    ap.add_argument("--tune-cache", metavar="JSON",
                    help="reuse (or store) the synthetic autotune report in this cache file, keyed by library "
                         "build, device and context (api.autotune_cached)")
    ap.add_argument("--tune-from", metavar="BENCH_JSON",
                    help="use the launch shapes that an earlier bench run chose (its output line)")
    ap.add_argument("--trace-summary", nargs=2, metavar=("BENCH_JSON", "TRACE_DIR"),
                    help="print the timed-region kernel summary of a rocprofv3 --kernel-trace and exit")
    ap.add_argument("--counter-summary", nargs=2, metavar=("BENCH_JSON", "PMC_DIR"),
                    help="print per-kernel issue statistics of the timed region from a rocprofv3 --pmc run of "
                         "the SQ counters " + " ".join(SQ_COUNTERS) + " (or LDS statistics from a run of " +
                         " ".join(LDS_COUNTERS) + ") and exit")
    return ap.parse_args()


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.traffic:
        print(traffic_summary(*args.traffic))
        return
    if args.trace_summary:
        print(trace_summary(*args.trace_summary))
        return
    if args.counter_summary:
        print(counter_summary(*args.counter_summary))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE={world}); "
              f"the library does not shard the likelihood path across GPUs.",
              flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2307_03763_amd import api
    from paper_2307_03763_amd import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)
    if args.pipeline_only:
        print(json.dumps({"pipeline": pipeline_leg(None if args.pipeline_full else tuple(args.pipeline_segments),
                                                   log, catalogue=args.pipeline_catalogue)}), flush=True)
        return

    # ---------------------------------------------------------------- workload (resident in HBM)
    T = I.T1
    ctx = api.context_for(T)
    t0 = time.time()
    wl = I.workload_c3(api.template_fn(ctx, api.GB_FP64), n_win=args.windows, n_cand=args.cands)
    log(f"workload built in {time.time() - t0:.1f}s: {wl.n_win} windows, {len(wl.theta)} candidates")
    d = torch.as_tensor(wl.data, device="cuda")
    w = torch.as_tensor(wl.weights, device="cuda")
    th = torch.as_tensor(wl.theta, device="cuda")
    rng = np.random.default_rng(I.SEED_BASE + 30)
    log_g = torch.as_tensor(rng.normal(0.0, 0.1, len(wl.theta)), device="cuda")
    u = torch.as_tensor(rng.random(len(wl.theta)), device="cuda")
    table = wl.window_table()
    rows = len(wl.theta)

    # ---------------------------------------------------------------- autotune launch shapes
    t0 = time.time()
    if args.tune_from:
        # the launch shapes of an earlier run (its output line), so that a profiling run of this
        # command launches exactly the kernels that run timed
        tune = "\n".join(_last_json(args.tune_from)["autotune"])
        log(f"launch shapes of {args.tune_from}: {api.apply_tuning(ctx.handle, tune)} set")
    else:
        # every family on synthetic candidates, then the families of this workload on its own
        # windows, data and candidates (the choice that its plans use)
        if args.tune_cache:
            generic, hit = api.autotune_cached(ctx, args.tune_cache, 3)
            log(f"synthetic autotune {'from' if hit else 'stored in'} {args.tune_cache}")
        else:
            generic = api.gb_autotune(ctx.handle, 3)
        tune = api.merge_tuning(generic, api.gb_autotune_windows(ctx.handle, table, d, w, th, 3))
    log(f"autotune {time.time() - t0:.1f}s:\n{tune}")

    # ---------------------------------------------------------------- precision policy
    # SNR of the loudest injection of every window (FP64 components on the GPU); windows at or
    # below RHO_MIXED run in mixed precision, louder ones in FP64 (Sec. III G sampling needs
    # logL differences to 1e-5; the mixed error grows like 6e-7 rho)
    rho_w = window_snr(api, ctx, wl, d, w)
    prec_w = np.where(rho_w <= args.rho_mixed, api.GB_MIXED, api.GB_FP64)
    log(f"precision policy: rho <= {args.rho_mixed}: {int((prec_w == api.GB_MIXED).sum())} of {wl.n_win} windows mixed")

    stream = torch.cuda.current_stream()
    logL = torch.empty(rows, dtype=torch.float64, device="cuda")
    chain = torch.empty(rows, dtype=torch.int32, device="cuda")
    grad = torch.empty((rows, 8), dtype=torch.float64, device="cuda")
    glog = torch.empty(rows, dtype=torch.float64, device="cuda")
    E = lambda: torch.cuda.Event(enable_timing=True)

    def make_groups(prec_of_window, grad_prec_of_window):
        """The plans of one step and the per-group likelihood plans.

        step: the MH stage of every window as one plan with per-window precision (one
        persistent likelihood launch per (N, C, precision) bucket, then one chain launch over
        all windows), followed by one gradient plan per (N, C, precision) group (one persistent
        launch each, so that each is timed on its own). mh_groups: one plan per (N, C,
        precision) group of the MH windows, used only to time each likelihood launch alone."""
        tab = np.concatenate([table, np.asarray(prec_of_window, dtype=np.int64)[:, None]], axis=1)
        p_all = api.Plan(ctx, tab, api.GB_PER_WINDOW)
        p_all.prepare(d, w)
        step = [(("mh", 0, 0, -1), list(range(wl.n_win)), p_all,
                 torch.empty(wl.n_win, dtype=torch.int64, device="cuda"))]
        mh_groups = []
        groups = {}
        for i, win in enumerate(wl.windows):
            groups.setdefault(("mh", win.N, win.C, int(prec_of_window[i])), []).append(i)
            groups.setdefault(("gr", win.N, win.C, int(grad_prec_of_window[i])), []).append(i)
        for key in sorted(groups, key=lambda k: (k[0], -k[1], -k[2], k[3])):
            idx = groups[key]
            p = api.Plan(ctx, table[idx], key[3])
            p.prepare(d, w)
            entry = (key, idx, p, None)
            (step if key[0] == "gr" else mh_groups).append(entry)
        return step, mh_groups

    def run_steps(groups, steps, warmup, region=None):
        def one(ev):
            for j, (key, idx, p, nacc) in enumerate(groups):
                if ev is not None:
                    ev[j][0].record(stream)
                if key[0] == "mh":
                    api.gb_mh_step(p.handle, d, w, th, log_g, u, args.temperature, logL, chain, nacc, stream)
                else:
                    api.gb_loglik_grad(p.handle, d, w, th, glog, grad, stream)
                if ev is not None:
                    ev[j][1].record(stream)
        for _ in range(warmup):
            one(None)
        torch.cuda.synchronize()
        evs = [[[E(), E()] for _ in groups] for _ in range(steps)]
        start, end = E(), E()
        if region is not None:
            region.resume()
        start.record(stream)
        for s_ in range(steps):
            one(evs[s_])
        end.record(stream)
        torch.cuda.synchronize()
        ms = start.elapsed_time(end) / steps
        per = np.array([[evs[s_][j][0].elapsed_time(evs[s_][j][1]) for j in range(len(groups))] for s_ in range(steps)])
        assert bool(torch.isfinite(logL).all()) and bool(torch.isfinite(grad).all()), "non-finite outputs"
        return ms, per.mean(axis=0)

    def summary(groups, ms, per):
        ms_mh = float(sum(t for (k, *_), t in zip(groups, per) if k[0] == "mh"))
        ms_gr = float(sum(t for (k, *_), t in zip(groups, per) if k[0] == "gr"))
        return {"ms_per_step": round(ms, 4), "value": round(2 * rows / (ms * 1e-3), 1),
                "logl_evals_per_s": round(rows / (ms_mh * 1e-3), 1),
                "grad_evals_per_s": round(rows / (ms_gr * 1e-3), 1)}

    # adaptive ragged (the headline); gradients run in mixed precision (the FP64 gradient is
    # switched off in this version of the library)
    grad_prec = np.full(wl.n_win, api.GB_MIXED)
    step_ad, mh_ad = make_groups(prec_w, grad_prec)
    region = TimedRegion()
    ms_ad, per_ad = run_steps(step_ad, args.steps, args.warmup, region)
    # the likelihood kernel alone for every MH group (the MH stage is those kernels plus the
    # chain kernel): the same launches through gb_loglik, still inside the profiled region
    kern = [(key, idx, float(t)) for (key, idx, _, _), t in zip(step_ad, per_ad) if key[0] == "gr"]
    for key, idx, p, _ in mh_ad:
        ev = [[E(), E()] for _ in range(args.steps)]
        for s_ in range(args.steps):
            ev[s_][0].record(stream)
            api.gb_loglik(p.handle, d, w, th, logL, None, stream)
            ev[s_][1].record(stream)
        torch.cuda.synchronize()
        kern.append((key, idx, float(np.mean([a.elapsed_time(b) for a, b in ev]))))
    region.pause()
    adaptive = summary(step_ad, ms_ad, per_ad)
    log(f"adaptive ragged: {ms_ad:.2f} ms/step {adaptive}")

    # mixed precision everywhere
    allmix = np.full(wl.n_win, api.GB_MIXED)
    step_mx, _ = make_groups(allmix, allmix)
    ms_mx, per_mx = run_steps(step_mx, args.steps, args.warmup)
    mixed = summary(step_mx, ms_mx, per_mx)
    log(f"mixed ragged: {ms_mx:.2f} ms/step {mixed}")
    logl_mixed = logL.cpu().numpy().copy()

    def time_calls(fn, reps):
        """Mean time of one call of fn (a sequence of launches on `stream`), HIP events."""
        fn()
        torch.cuda.synchronize()
        ev = [[E(), E()] for _ in range(reps)]
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return float(np.mean([a.elapsed_time(b) for a, b in ev]))

    # logL kernels alone (no chain) of the adaptive step: its MH plan (every window, one
    # persistent launch per (N, C, precision) bucket) through gb_loglik, the batching of the FP64
    # ragged figure below
    p_mh = step_ad[0][2]
    ms_ad_logl = time_calls(lambda: api.gb_loglik(p_mh.handle, d, w, th, logL, None, stream), args.steps)
    adaptive["logl_only_evals_per_s"] = round(rows / (ms_ad_logl * 1e-3), 1)

    # FP64 ragged: the headline's plan structure (one MH call over all windows: one persistent
    # logL launch per (N, C) bucket, one chain launch) with every window in FP64, so that mixed
    # against FP64 compares precision at equal batching
    fp64r = None
    if not args.no_fp64:
        tab64 = np.concatenate([table, np.full((wl.n_win, 1), api.GB_FP64, dtype=np.int64)], axis=1)
        p64 = api.Plan(ctx, tab64, api.GB_PER_WINDOW)
        p64.prepare(d, w)
        nacc64 = torch.empty(wl.n_win, dtype=torch.int64, device="cuda")
        ms_64 = time_calls(lambda: api.gb_mh_step(p64.handle, d, w, th, log_g, u, args.temperature, logL, chain,
                                                  nacc64, stream), args.steps)
        ms_64l = time_calls(lambda: api.gb_loglik(p64.handle, d, w, th, logL, None, stream), args.steps)
        fp64r = {"logl_evals_per_s": round(rows / (ms_64 * 1e-3), 1), "ms_mh_stage": round(ms_64, 3),
                 "logl_only_evals_per_s": round(rows / (ms_64l * 1e-3), 1), "ms_logl_only": round(ms_64l, 3),
                 "grad_evals_per_s": None,
                 "note": "MH stage of all windows in one call, every window FP64 (the headline's batching); "
                         "logl_only: the same likelihood launches without the chain; the FP64 gradient is "
                         "switched off in this version, so the FP64 comparison is one of likelihoods"}
        log(f"FP64 ragged: MH stage {ms_64:.2f} ms, logL only {ms_64l:.2f} ms")
        p64.close()

    # dominant kernel of the headline step (largest k_batch time per step)
    key, idx, dur_ms = max(kern, key=lambda e: e[2])
    kind, kN, kC, kP = key
    n_dom = int(sum(wl.n_cand[i] for i in idx))
    is_grad = kind == "gr"
    fl = sum(int(wl.n_cand[i]) * flops_per_eval(kN, kC, min(wl.windows[i].W, kN), is_grad) for i in idx)
    achieved_tf = fl / (dur_ms * 1e-3) / 1e12
    kname = tuned_kernel_name(tune, kP, is_grad, kN, kC)
    roofline = {"bound": "alu", "achieved": round(achieved_tf, 3), "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved_tf / PEAK_VALU_TFLOPS, 4), "traffic": committed_traffic(kname, n_dom),
                "kernel": kname,
                "launch_ms": round(dur_ms, 4), "evals_per_launch": n_dom,
                "timing": "HIP events on the launch stream, mean over the timed launches",
                "launches_in_region": args.steps * (2 if kind == "mh" else 1),
                "flops_per_eval": round(fl / n_dom, 1),
                "hbm_gbs": round((n_dom * bytes_per_eval(kC, kN, is_grad) +
                                  sum(24.0 * kC * wl.windows[i].W for i in idx)) / (dur_ms * 1e-3) / 1e9, 3),
                "sincos_per_s": round(n_dom * sincos_per_eval(kN, is_grad) / (dur_ms * 1e-3), 1)}

    # ---------------------------------------------------------------- plain FP64: one launch per window
    fp64 = None
    if not args.no_fp64:
        win_plans = []
        for i in range(wl.n_win):
            p = api.Plan(ctx, table[i:i + 1], api.GB_FP64)
            p.prepare(d, w)
            win_plans.append(p)
        nacc1 = torch.empty(1, dtype=torch.int64, device="cuda")

        def plain(ev):
            ev[0].record(stream)
            for p in win_plans:
                api.gb_mh_step(p.handle, d, w, th, log_g, u, args.temperature, logL, chain, nacc1, stream)
            ev[1].record(stream)

        plain([E(), E()])
        torch.cuda.synchronize()
        ev = [E(), E()]
        plain(ev)
        torch.cuda.synchronize()
        f_l = ev[0].elapsed_time(ev[1])

        def plain_logl():
            for p in win_plans:
                api.gb_loglik(p.handle, d, w, th, logL, None, stream)
        f_ll = time_calls(plain_logl, 2)
        fp64 = {"logl_evals_per_s": round(rows / (f_l * 1e-3), 1), "ms_mh_stage": round(f_l, 3),
                "logl_only_evals_per_s": round(rows / (f_ll * 1e-3), 1), "ms_logl_only": round(f_ll, 3),
                "grad_evals_per_s": None,
                "note": "MH stage (logL of every proposal + its chain) in FP64, one likelihood launch and one "
                        "chain launch per window; logl_only: the per-window likelihood launches alone; the "
                        "FP64 gradient is switched off in this version, so the comparison is one of likelihoods"}
        log(f"plain FP64 per window: logL {fp64['logl_evals_per_s']:.3e}/s, logL only {f_ll:.2f} ms")
        for p in win_plans:
            p.close()

    cfgs = None
    if not args.no_configs:
        cfgs = configs_leg(log)

    post = None
    if not args.no_posterior:
        post = posterior_leg(args.posterior_sources, log)

    pipe = None
    if not args.no_pipeline:
        pipe = pipeline_leg(None if args.pipeline_full else tuple(args.pipeline_segments), log,
                            catalogue=args.pipeline_catalogue)

    # gradient accuracy scale of every row: the mixed gradient's error against the gradient's own
    # noise scale sqrt(F_ii) grows like sqrt(<d|d> + <h|h>) (the FP32 template error times the
    # residual norm); rows with sqrt(<d|d> + <h|h>) <= GRAD_NORM_LIMIT stay within 1e-5 sqrt(F_ii)
    pmx = api.Plan(ctx, table, api.GB_MIXED)
    pmx.prepare(d, w)
    _, comps_mx = pmx.loglik(th, comps=True)
    dd_w = torch.as_tensor([float(np.sum(wl.window_data(i)[1] * np.abs(wl.window_data(i)[0]) ** 2))
                            for i in range(wl.n_win)], device="cuda")
    win_of_row = torch.as_tensor(np.repeat(np.arange(wl.n_win), wl.n_cand), device="cuda")
    norm_row = torch.sqrt(dd_w[win_of_row] + comps_mx[:, 1])
    n_within = int((norm_row <= GRAD_NORM_LIMIT).sum())
    pmx.close()
    grad_acc = {"bar": "|g_gpu - g_oracle|_i <= 1e-5 sqrt(F_ii), F the Fisher matrix at the candidate",
                "rows_with_norm_within_limit": n_within, "rows": rows,
                "norm_limit": f"sqrt(<d|d> + <h|h>) <= {GRAD_NORM_LIMIT:g}",
                "model": "error ~ (2e-7 .. 1.1e-6) sqrt(<d|d> + <h|h>) sqrt(F_ii), largest in the amplitude "
                         "and inclination components (FP32 template error times the residual norm)",
                "grad_evals_per_s_within_bar": round(n_within / (float(sum(t for (k, *_), t in zip(step_ad, per_ad)
                                                                           if k[0] == "gr")) * 1e-3), 1)}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(wl, args.cpu_seconds, logl_mixed, rho_w, log, grad, grad_acc)

    value = adaptive["value"]
    out = {
        "metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": adaptive["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "windows": wl.n_win, "candidates": rows, "T_s": T,
                   "precision": f"adaptive: mixed (FP64 phase and accumulation, FP32 response and DFT) for "
                                f"windows with injected SNR <= {args.rho_mixed}, FP64 otherwise",
                   "mixed_windows": int((prec_w == api.GB_MIXED).sum()),
                   "step": "MH stage of all windows in one call (one persistent logL launch per (N, C, "
                           "precision) bucket, then one chain launch over all windows), then the "
                           "gradients, one persistent launch per (N, C) group"},
        "logl_evals_per_s": adaptive["logl_evals_per_s"],
        "grad_evals_per_s": adaptive["grad_evals_per_s"],
        "logl_only_evals_per_s": adaptive["logl_only_evals_per_s"],
        "grad_accuracy": grad_acc,
        "mixed_everywhere": mixed,
        "fp64_ragged": fp64r,
        "fp64_plain": fp64,
        "speedup_vs_fp64": (round(adaptive["logl_evals_per_s"] / fp64["logl_evals_per_s"], 3) if fp64 else None),
        "speedup_basis": "logL evals/s of the MH stage, adaptive ragged vs plain FP64 per window: precision "
                         "and batching together; 'speedups' separates them",
        "speedups": speedups(adaptive, mixed, fp64r, fp64),
        "roofline": roofline,
        "configs": cfgs,
        "posterior": post,
        "pipeline": pipe,
        "timed_region_ns": region.t,
        "cpu_baseline": cpu,
        "autotune": tune.strip().split("\n"),
        "library": library_hash(),
        "kernel_src": kernel_source_hash(),
        "context": "paper: 1.8 s per posterior of 6 x 10,000 likelihoods on a Quadro RTX 4000 Mobile "
                   "(about 3.3e4 logL/s including chain and KDE); different hardware and work",
    }
    print(json.dumps(out), flush=True)


GRAD_NORM_LIMIT = 25.0      # sqrt(<d|d> + <h|h>) below which mixed gradients meet 1e-5 sqrt(F_ii)


def speedups(adaptive, mixed, fp64r, fp64p):
    """Likelihood-rate ratios, each named by the effect it measures."""
    if not fp64r or not fp64p:
        return None
    r = lambda a, b: round(a / b, 3)
    return {
        "precision_at_equal_batching (MH stage, adaptive ragged / FP64 ragged)":
            r(adaptive["logl_evals_per_s"], fp64r["logl_evals_per_s"]),
        "precision_at_equal_batching (MH stage, all-mixed ragged / FP64 ragged)":
            r(mixed["logl_evals_per_s"], fp64r["logl_evals_per_s"]),
        "precision_at_equal_batching (logL kernels only, adaptive ragged / FP64 ragged)":
            r(adaptive["logl_only_evals_per_s"], fp64r["logl_only_evals_per_s"]),
        "batching_at_equal_precision (MH stage, FP64 ragged / FP64 per window)":
            r(fp64r["logl_evals_per_s"], fp64p["logl_evals_per_s"]),
        "batching_at_equal_precision (logL kernels only, FP64 ragged / FP64 per window)":
            r(fp64r["logl_only_evals_per_s"], fp64p["logl_only_evals_per_s"]),
        "both (MH stage, adaptive ragged / FP64 per window)":
            r(adaptive["logl_evals_per_s"], fp64p["logl_evals_per_s"]),
    }


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


class TimedRegion:
    """Host clock readings (CLOCK_MONOTONIC and CLOCK_BOOTTIME, ns) around the timed launches,
    taken after a device synchronisation on both sides, so that the launches of a rocprofv3
    trace of the same command that fall inside the window are exactly the timed ones."""

    def __init__(self):
        self.t = {}

    @staticmethod
    def _now():
        return {"monotonic": time.clock_gettime_ns(time.CLOCK_MONOTONIC),
                "boottime": time.clock_gettime_ns(time.CLOCK_BOOTTIME)}

    def resume(self):
        import torch
        torch.cuda.synchronize()
        self.t0 = self._now()

    def pause(self):
        import torch
        torch.cuda.synchronize()
        t1 = self._now()
        self.t = {k: [self.t0[k], t1[k]] for k in t1}


def tuned_kernel_name(tune: str, prec: int, grad: bool, N: int, C: int) -> str:
    """The k_batch instantiation the autotuner chose for (precision, mode, N, C), as
    'k_batch<R,N,LPC,C,WPB,MODE,OCC>' (the template arguments of the kernel symbol)."""
    head = ("fp64 " if prec == 0 else "mixed") + " " + ("grad  " if grad else "loglik") + f" N={N} C={C}:"
    for line in tune.splitlines():
        if line.startswith(head) and "kernel=" in line:
            return line.split("kernel=", 1)[1].strip()
    return f"k_batch<{'double' if prec == 0 else 'float'},{N},?,{C},?,{2 if grad else 1},?>"


def _kernel_key(name: str) -> str:
    """'void gbx::k_batch<double, 512, 128, 3, 4, 1, 1>(gbx::BatchArgs)' -> 'k_batch<double,512,128,3,4,1,1>'."""
    n = name.replace(" ", "")
    if n.startswith("void"):
        n = n[4:]
    n = n.split("(", 1)[0]
    return n[5:] if n.startswith("gbx::") else n


def _dispatches(run_dir: str, counter: str = None) -> list:
    """Kernel dispatches of a rocprofv3 output directory as (kernel key, start ns, end ns, value):
    from the SQLite database (rocprofv3's default output) or from its CSV files; value is the
    counter's value for a --pmc run (counter given), else None."""
    import csv
    import glob
    import sqlite3
    out = []
    dbs = glob.glob(os.path.join(run_dir, "**", "*.db"), recursive=True)
    if dbs:
        for fn in dbs:
            con = sqlite3.connect(fn)
            if counter is None:
                q = "select name, start, end, NULL from kernels"
            else:
                q = f"select name, start, end, counter_value from pmc_events where counter_name = '{counter}'"
            out += [(_kernel_key(n), int(t0), int(t1), v) for n, t0, t1, v in con.execute(q)]
            con.close()
        return out
    pat = "*kernel_trace.csv" if counter is None else "*counter_collection.csv"
    for fn in glob.glob(os.path.join(run_dir, "**", pat), recursive=True):
        with open(fn) as f:
            for row in csv.DictReader(f):
                if counter is not None and row.get("Counter_Name") != counter:
                    continue
                out.append((_kernel_key(row["Kernel_Name"]), int(row.get("Start_Timestamp", 0) or 0),
                            int(row.get("End_Timestamp", 0) or 0),
                            float(row["Counter_Value"]) if counter is not None else None))
    if not out:
        raise FileNotFoundError(f"no rocprofv3 output under {run_dir}")
    return out


def _in_region(disp: list, bench: dict) -> list:
    """The dispatches inside the bench's timed region, on the host clock under which the dominant
    kernel shows exactly the expected number of launches."""
    kern = bench["roofline"]["kernel"]
    want = bench["roofline"]["launches_in_region"]
    for clock, (t0, t1) in bench["timed_region_ns"].items():
        sel = [d for d in disp if d[1] >= t0 and d[2] <= t1]
        if sum(1 for d in sel if d[0] == kern) == want:
            return sel
    raise ValueError(f"no clock puts {want} launches of {kern} inside the timed region")


def _last_json(path: str) -> dict:
    import json as _json
    return _json.loads(open(path).read().strip().splitlines()[-1])


def trace_summary(bench_json: str, trace_dir: str) -> str:
    """Per-kernel durations of the launches inside the bench's timed region, from a rocprofv3
    --kernel-trace of the same command, beside the bench's own event timing of its dominant
    kernel."""
    b = _last_json(bench_json)
    sel = _in_region(_dispatches(trace_dir), b)
    per = {}
    for k, t0, t1, _ in sel:
        per.setdefault(k, []).append((t1 - t0) * 1e-6)
    span = (max(d[2] for d in sel) - min(d[1] for d in sel)) * 1e-6
    kern = b["roofline"]["kernel"]
    lines = [f"timed region: {len(sel)} dispatches over {span:.3f} ms (first start to last end)",
             f"{'kernel':<44} {'calls':>6} {'avg ms':>9} {'total ms':>10} {'% busy':>7}"]
    busy = sum(sum(v) for v in per.values())
    for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"{k:<44} {len(v):>6} {sum(v) / len(v):>9.4f} {sum(v):>10.3f} {100 * sum(v) / busy:>6.1f}%")
    dom = per[kern]
    lines.append(f"dominant kernel {kern}: rocprofv3 average {sum(dom) / len(dom):.4f} ms over {len(dom)} "
                 f"launches; bench HIP-event average {b['roofline']['launch_ms']:.4f} ms")
    return "\n".join(lines)


def _counter_sums(bench_json: str, pmc_dir: str, counters) -> dict:
    """Per k_batch kernel: the counters summed over its dispatches inside the timed region (each
    counter's per-shader-engine values summed per dispatch), and the set of those dispatches."""
    b = _last_json(bench_json)
    per = {}
    for ctr in counters:
        tot = {}
        for k, t0, t1, v in _dispatches(pmc_dir, ctr):
            tot[(k, t0, t1)] = tot.get((k, t0, t1), 0.0) + v
        for k, t0, t1, v in _in_region([key + (v,) for key, v in tot.items()], b):
            if not k.startswith("k_batch"):
                continue
            d = per.setdefault(k, {"disp": set()})
            d["disp"].add((t0, t1))
            d[ctr] = d.get(ctr, 0.0) + v
    return per


def lds_summary(bench_json: str, pmc_dir: str) -> str:
    """Per-kernel LDS statistics from a rocprofv3 --pmc run of LDS_COUNTERS over the bench: LDS
    instructions per wave, and the shares of the cycles in which the LDS was busy with a
    wave's request (SQ_LDS_IDX_ACTIVE) that went to bank conflicts and to address conflicts."""
    per = _counter_sums(bench_json, pmc_dir, LDS_COUNTERS)
    lines = [f"{'kernel':<34} {'disp':>5} {'avg ms':>8} {'LDS inst/wave':>13} {'bank-conflict':>13} "
             f"{'addr-conflict':>13} {'unaligned':>9}",
             f"{'':<34} {'':>5} {'':>8} {'':>13} {'/ LDS active':>13} {'/ LDS active':>13} {'/ active':>9}"]
    for k, d in sorted(per.items(), key=lambda kv: -sum(t1 - t0 for t0, t1 in kv[1]["disp"])):
        n = len(d["disp"])
        ms = sum(t1 - t0 for t0, t1 in d["disp"]) * 1e-6 / n
        act = max(d["SQ_LDS_IDX_ACTIVE"], 1.0)
        lines.append(f"{k:<34} {n:>5} {ms:>8.3f} {d['SQ_INSTS_LDS'] / d['SQ_WAVES']:>13.1f} "
                     f"{d['SQ_LDS_BANK_CONFLICT'] / act:>13.4f} {d['SQ_LDS_ADDR_CONFLICT'] / act:>13.4f} "
                     f"{d['SQ_LDS_UNALIGNED_STALL'] / act:>9.4f}")
    return "\n".join(lines)


def counter_summary(bench_json: str, pmc_dir: str) -> str:
    """Per-kernel issue statistics from one rocprofv3 --pmc run of SQ_COUNTERS over the bench
    (its output line in bench_json), summed over the dispatches of each k_batch kernel inside
    the timed region.  Per wave: the share of its cycles spent issuing VALU
    instructions (SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES) and waiting (SQ_WAIT_ANY /
    SQ_WAVE_CYCLES).  The persistent kernels launch exactly the waves that stay resident, so
    waves per SIMD = waves per dispatch / N_SIMD, and that times the per-wave VALU share is the
    share of the SIMD's cycles with a VALU instruction in flight."""
    if not _dispatches(pmc_dir, "SQ_WAVE_CYCLES") and _dispatches(pmc_dir, "SQ_LDS_BANK_CONFLICT"):
        return lds_summary(bench_json, pmc_dir)
    per = _counter_sums(bench_json, pmc_dir, SQ_COUNTERS)
    lines = [f"{'kernel':<34} {'disp':>5} {'avg ms':>8} {'waves/SIMD':>10} {'VALU/wave':>9} {'wait/wave':>9} "
             f"{'SIMD VALU busy':>14} {'VALU cyc/inst':>13}"]
    for k, d in sorted(per.items(), key=lambda kv: -sum(t1 - t0 for t0, t1 in kv[1]["disp"])):
        n = len(d["disp"])
        ms = sum(t1 - t0 for t0, t1 in d["disp"]) * 1e-6 / n
        wc = d["SQ_WAVE_CYCLES"]
        wps = d["SQ_WAVES"] / n / N_SIMD
        valu = d["SQ_ACTIVE_INST_VALU"] / wc
        lines.append(f"{k:<34} {n:>5} {ms:>8.3f} {wps:>10.2f} {valu:>9.3f} {d['SQ_WAIT_ANY'] / wc:>9.3f} "
                     f"{valu * wps:>14.3f} {d['SQ_ACTIVE_INST_VALU'] / d['SQ_INSTS_VALU']:>13.3f}")
    return "\n".join(lines)


def traffic_summary(k_fetch: str, k_write: str, c_fetch: str, c_write: str) -> str:
    """One line for profiles/hbm_traffic.txt: HBM bytes per launch of the dominant kernel from
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch; two rocprofv3 --pmc runs of the bench, each
    directory DIR beside DIR.json, the bench's output line of that run), each scaled by what
    the same counter reads for the copy calibration of known size (its largest dispatch)."""
    vals, kern, b = {}, None, None
    for ctr, run in (("FETCH_SIZE", k_fetch), ("WRITE_SIZE", k_write)):
        b = _last_json(run.rstrip("/") + ".json")
        if kern is not None and b["roofline"]["kernel"] != kern:
            raise ValueError("the two counter runs chose different kernels")
        kern = b["roofline"]["kernel"]
        sel = [d for d in _in_region(_dispatches(run, ctr), b) if d[0] == kern]
        vals[ctr] = sum(d[3] for d in sel) / len(sel)
    copy_f = max(d[3] for d in _dispatches(c_fetch, "FETCH_SIZE"))
    copy_w = max(d[3] for d in _dispatches(c_write, "WRITE_SIZE"))
    s_f = 8 * COPY_N / (copy_f * 1024.0)
    s_w = 8 * COPY_N / (copy_w * 1024.0)
    by = vals["FETCH_SIZE"] * 1024.0 * s_f + vals["WRITE_SIZE"] * 1024.0 * s_w
    return (f"kernel_src={b.get('kernel_src', '?')} library={b['library']} kernel={kern} "
            f"evals={b['roofline']['evals_per_launch']} bytes={by:.0f} "
            f"fetch_kib={vals['FETCH_SIZE']:.1f} write_kib={vals['WRITE_SIZE']:.1f} "
            f"copy_scale_fetch={s_f:.4f} copy_scale_write={s_w:.4f}")


def library_hash() -> str:
    import hashlib
    from paper_2307_03763_amd import api
    return hashlib.sha256(open(api.LIB_PATH, "rb").read()).hexdigest()[:16]


KERNEL_SOURCES = ("gbx_device.h", "gbx_kernels.h", "gbx_variants.h", "k_f64_loglik.hip", "k_mixed_loglik.hip",
                  "k_mixed_grad.hip", "k_waveform.hip")


def kernel_source_hash() -> str:
    """sha256[:16] of the sources the k_batch kernels are compiled from and of the compile flags:
    a counter summary stays valid while these are unchanged."""
    import hashlib
    from paper_2307_03763_amd import build
    h = hashlib.sha256(" ".join(build.FLAGS[:-2]).encode())
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2307_03763_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def committed_traffic(kernel: str, evals: int):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/hbm_traffic.txt, lines 'kernel_src=<hash> kernel=<name> evals=<n> bytes=<B> ...'),
    scaled to `evals`; None when absent or taken from other kernel sources."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    h = kernel_source_hash()
    want = kernel.replace(" ", "")
    for line in open(path):
        if line.lstrip().startswith("#"):
            continue
        f = dict(x.split("=", 1) for x in line.split() if "=" in x)
        # only the same instantiation: the last template argument is the occupancy bound of
        # __launch_bounds__, which changes the register allocation and so the machine code
        if f.get("kernel_src") == h and f.get("kernel") == want:
            return round(float(f["bytes"]) * evals / float(f["evals"]), 1)
    return None


def copy_calibration():
    """A device copy of a known size, profiled with the same counters as the kernels
    (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE) to scale them to bytes."""
    import torch
    n = COPY_N
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 1.0, out=b)  # an elementwise copy kernel: reads n doubles, writes n doubles
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "launches": 3}), flush=True)


def window_snr(api, ctx, wl, d, w):
    """sqrt(<h|h>) of the loudest injection of every window (FP64 components on the GPU)."""
    import numpy as np
    import torch
    tab = wl.window_table().copy()
    srcs, off = [], 0
    for i, win in enumerate(wl.windows):
        tab[i, 6] = off
        tab[i, 7] = len(win.sources)
        srcs.append(win.sources)
        off += len(win.sources)
    p = api.Plan(ctx, tab, api.GB_FP64)
    p.prepare(d, w)
    _, comps = p.loglik(torch.as_tensor(np.concatenate(srcs), device="cuda"), comps=True)
    hh = comps[:, 1].cpu().numpy()
    out = np.array([np.sqrt(hh[tab[i, 6]:tab[i, 6] + tab[i, 7]].max()) for i in range(wl.n_win)])
    p.close()
    return out


def posterior_leg(n_sources, log):
    """Algorithm 4 end to end for the target source of the C2 window (three overlapping GBs,
    the other two subtracted): Fisher matrix, reduced box, six temperatures x 10,000 proposals
    with pairwise-KDE proposals after the first; wall-clock seconds per source (host work
    included), over `n_sources` repetitions with different random streams."""
    import numpy as np
    import torch

    from paper_2307_03763_amd import api
    from paper_2307_03763_amd import drivers as D
    from paper_2307_03763_amd import inputs as I
    ctx = api.context_for(I.T2)
    wl = I.workload_c2(api.template_fn(ctx, api.GB_FP64), n_cand=1)
    row = wl.window_table()[0]
    be = D.GpuPosteriorBackend(ctx, row, torch.as_tensor(wl.data, device="cuda"),
                               torch.as_tensor(wl.weights, device="cuda"))
    src = wl.windows[0].sources[0]
    box = wl.window_box(0)
    D.tune_on_windows(ctx, row[None, :], be.d, be.w, [box], per_window=10000)
    D.annealed_posterior(be, src, box, np.random.default_rng(0), n=10000)   # warm-up (plans, code)
    times, acc = [], []
    for k in range(n_sources):
        torch.cuda.synchronize()
        t0 = time.time()
        stages, _, _ = D.annealed_posterior(be, src, box, np.random.default_rng(100 + k), n=10000)
        torch.cuda.synchronize()
        times.append(time.time() - t0)
        acc.append([s["n_accept"] for s in stages])
    log(f"posterior: {np.median(times):.3f} s per source (6 x 10,000)")
    return {"seconds_per_source": round(float(np.median(times)), 4), "temperatures": [15, 10, 5, 3, 2, 1],
            "proposals_per_stage": 10000, "accepted_per_stage": acc[0],
            "workload": "C2 target source (8 mHz, N=256, T=2^22*15 s), injected parameters as the MLE",
            "context": "paper: 1.8 s per signal for the same six stages on a Quadro RTX 4000 Mobile"}


def configs_leg(log, reps: int = 5):
    """Throughput of the other workloads, each at its full size on the device (inputs resident,
    launch shapes tuned on the workload's own windows, HIP events around the call, mean of `reps` after one untimed call):
    C1 (1,000 candidates, one window), C2 (10,000 candidates in the reduced box of three
    overlapping GBs, then the 10,000-step chain: the MH stage), C4 (64 windows x 4,096 gradients)
    and C5 (4,000 full-band windows x 512 DE candidates, logL as the search scores them).  Per
    call: evaluations per second and the algorithmic FLOP rate of the flop model against the
    78.6 TFLOP/s vector peak (whole call, all its launches)."""
    import numpy as np
    import torch

    from paper_2307_03763_amd import api
    from paper_2307_03763_amd import inputs as I
    E = lambda: torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    ctxs = {}

    def ctx_for(T):
        if T not in ctxs:
            ctxs[T] = api.context_for(T)
            api.gb_autotune(ctxs[T].handle, 2)
        return ctxs[T]

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = E(), E()
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    def flops(wl, grad):
        return sum(float(wl.n_cand[i]) * flops_per_eval(w.N, w.C, min(w.W, w.N), grad) for i, w in enumerate(wl.windows))

    def entry(wl, ms, grad, extra=None):
        rows = int(sum(wl.n_cand))
        tf = flops(wl, grad) / (ms * 1e-3) / 1e12
        out = {"evals_per_s": round(rows / (ms * 1e-3), 1), "ms_per_call": round(ms, 4), "evals_per_call": rows,
               "tflops": round(tf, 3), "frac_of_78.6": round(tf / PEAK_VALU_TFLOPS, 4)}
        out.update(extra or {})
        return out

    res = {}
    for name in ("C1", "C2", "C4", "C5"):
        t0 = time.time()
        T = I.T2 if name in ("C2", "C5") else I.T1
        ctx = ctx_for(T)
        tf = api.template_fn(ctx, api.GB_FP64)
        wl = {"C1": lambda: I.workload_c1(tf, n_cand=1000), "C2": lambda: I.workload_c2(tf, n_cand=10000),
              "C4": lambda: I.workload_c4(tf, n_win=64, n_cand=4096), "C5": lambda: I.workload_c5(tf)}[name]()
        d = torch.as_tensor(wl.data, device="cuda")
        w = torch.as_tensor(wl.weights, device="cuda")
        th = torch.as_tensor(wl.theta, device="cuda")
        rows = len(wl.theta)
        logL = torch.empty(rows, dtype=torch.float64, device="cuda")
        api.gb_autotune_windows(ctx.handle, wl.window_table(), d, w, th, 2)
        r = {"workload": wl.name}
        for pname, prec in (("fp64", api.GB_FP64), ("mixed", api.GB_MIXED)):
            p = api.Plan(ctx, wl.window_table(), prec)
            p.prepare(d, w)
            if name == "C2":
                rng = np.random.default_rng(5)
                log_g = torch.zeros(rows, dtype=torch.float64, device="cuda")
                u = torch.as_tensor(rng.random(rows), device="cuda")
                chain = torch.empty(rows, dtype=torch.int32, device="cuda")
                nacc = torch.empty(wl.n_win, dtype=torch.int64, device="cuda")
                ms = timed(lambda: api.gb_mh_step(p.handle, d, w, th, log_g, u, 1.0, logL, chain, nacc, stream))
                r[f"{pname}_mh_stage"] = entry(wl, ms, False, {"note": "logL of every proposal, then the chain"})
            ms = timed(lambda: api.gb_loglik(p.handle, d, w, th, logL, None, stream))
            r[f"{pname}_logl"] = entry(wl, ms, False)
            if name == "C4" and prec == api.GB_MIXED:
                grad = torch.empty((rows, 8), dtype=torch.float64, device="cuda")
                ms = timed(lambda: api.gb_loglik_grad(p.handle, d, w, th, logL, grad, stream))
                r["mixed_grad"] = entry(wl, ms, True)
            p.close()
        res[name] = r
        log(f"configs: {name} in {time.time() - t0:.1f} s: " +
            ", ".join(f"{k} {v['evals_per_s']:.3e}/s" for k, v in r.items() if isinstance(v, dict)))
    for c in ctxs.values():
        c.close()
    # C3 on numerical orbits: the exact Keplerian orbits (arms breathing by +-0.24%) given as
    # positions on a grid, one light time per arm in the templates, likelihoods and gradients
    # (gb_set_orbit); injections computed on the same orbits.  Rates only: the flop model is the
    # equal-arm one.
    t0 = time.time()
    ctx = api.context_for(I.T1)
    pos, g0, gdt = I.orbit_grid(lambda t: I.keplerian_orbits(t), I.T1, 4097)
    ctx.set_orbit(pos, g0, gdt)
    wl = I.workload_c3(api.template_fn(ctx, api.GB_FP64), n_win=256, n_cand=10000)
    d = torch.as_tensor(wl.data, device="cuda")
    w = torch.as_tensor(wl.weights, device="cuda")
    th = torch.as_tensor(wl.theta, device="cuda")
    rows = len(wl.theta)
    logL = torch.empty(rows, dtype=torch.float64, device="cuda")
    r = {"workload": wl.name + ", on exact Keplerian orbits (one light time per arm)"}
    for pname, prec in (("fp64", api.GB_FP64), ("mixed", api.GB_MIXED)):
        p = api.Plan(ctx, wl.window_table(), prec)
        p.prepare(d, w)
        ms = timed(lambda: api.gb_loglik(p.handle, d, w, th, logL, None, stream))
        r[f"{pname}_logl"] = {"evals_per_s": round(rows / (ms * 1e-3), 1), "ms_per_call": round(ms, 4),
                              "evals_per_call": rows}
        if prec == api.GB_MIXED:
            grad = torch.empty((rows, 8), dtype=torch.float64, device="cuda")
            ms = timed(lambda: api.gb_loglik_grad(p.handle, d, w, th, logL, grad, stream))
            r["mixed_grad"] = {"evals_per_s": round(rows / (ms * 1e-3), 1), "ms_per_call": round(ms, 4),
                               "evals_per_call": rows}
        p.close()
    ctx.close()
    res["C3_numerical_orbits"] = r
    log(f"configs: C3 on numerical orbits in {time.time() - t0:.1f} s: " +
        ", ".join(f"{k} {v['evals_per_s']:.3e}/s" for k, v in r.items() if isinstance(v, dict)))
    return res


S_PARTIAL = 0.7   # share of the recovered signals subtracted for the posterior's noise (Sec. III G)


def pipeline_leg(segments, log, precision: str = "mixed", catalogue=None, noise: str = "median",
                 posterior_noise: str = "residual", **search_kw):
    """Algorithm 5 end to end over a contiguous block of the full-band workload (4000 segments
    over 0.3-30 mHz, 20,000 GBs, T = 2^22*15 s, PSD noise): the global search (Algorithm 3 with
    the three runs of Table II; per signal three searches of DE/best/1/bin with 512 members x up
    to 1000 generations on the device (SciPy's convergence stop) plus the gradient polish, four
    joint sweeps; the search's noise level the paper's dynamic per-segment median periodogram
    (``noise``="psd" uses the true PSD); mixed gradient, the
    likelihood in ``precision``), the residual, and the annealed posterior (6 x 10,000) of every
    recovered source, batched, its likelihood in ``precision`` too.  Wall-clock seconds per
    phase (host work included); recovered sources scored with the match metric of Sec. IV
    (delta < 0.3 against the nearest injected sources) and injected sources counted by their
    optimal SNR in their segment's window.  The posterior's noise (``posterior_noise``):
    "residual", the global estimate (Sec. III F) of the residual; "partial", that of the partial
    residual d - 0.7 sum s (Sec. III G, the paper's option for overlapping signals); "psd", the
    true PSD.  Both estimates are reported against the true PSD."""
    import numpy as np
    import torch

    from paper_2307_03763_amd import api
    from paper_2307_03763_amd import drivers as D
    from paper_2307_03763_amd import inputs as I
    ctx = api.context_for(I.T2)
    t_setup = time.time()
    wl = I.workload_c5(api.template_fn(ctx, api.GB_FP64), pop=1, segments=segments)
    T = wl.T
    table = wl.window_table()
    segs = wl.segments
    d = torch.as_tensor(wl.data, device="cuda")
    w = torch.as_tensor(wl.weights, device="cuda")
    boxes = [wl.window_box(i) for i in range(wl.n_win)]
    # injected sources whose frequency lies in the block's unpadded segments, with their optimal
    # SNR in the window of their segment
    pop = wl.population
    seg_of = np.searchsorted(segs[:, 0], pop[:, 0], side="right") - 1
    inside = (seg_of >= 0) & (seg_of < len(segs))
    inside[inside] &= pop[inside, 0] < segs[seg_of[inside], 1]
    inj, inj_seg = pop[inside], seg_of[inside]
    tab = table[inj_seg].copy()
    tab[:, 6] = np.arange(len(inj))
    tab[:, 7] = 1
    p = api.Plan(ctx, tab, api.GB_FP64)
    p.prepare(d, w)
    _, comps = p.loglik(torch.as_tensor(inj, device="cuda"), comps=True)
    rho_opt = np.sqrt(comps[:, 1].cpu().numpy())
    p.close()
    t_tune = time.time()
    D.tune_on_windows(ctx, table, d, w, boxes, per_window=512)
    log(f"pipeline: {wl.n_win} segments {segs[0, 0] * 1e3:.3f}-{segs[-1, 1] * 1e3:.3f} mHz, {len(inj)} injected "
        f"({int((rho_opt > 9).sum())} with optimal SNR > 9), setup {time.time() - t_setup:.1f} s "
        f"(launch shapes tuned on the segments in {time.time() - t_tune:.1f} s)")

    prec = {"mixed": api.GB_MIXED, "fp64": api.GB_FP64}[precision]

    def factory(rows, d_an):
        return D.GpuSearchBackend(ctx, table[rows], d_an, w, [boxes[r] for r in rows], prec, api.GB_MIXED,
                                  noise=noise)

    def subtract(dd, srcs, win):
        return api.gb_add_templates(ctx.handle, table, torch.as_tensor(srcs, device="cuda"), win, -1.0, dd)

    torch.cuda.synchronize()
    t0 = time.time()
    kw = dict(n_searches=3, pop=512, generations=1000, polish_iterations=20, joint_sweeps=4, strategy="best1",
              tol=0.01)
    kw.update(search_kw)
    found, found_seg = D.global_search(factory, table, T, segs, d, np.random.default_rng(2023), subtract,
                                       progress=lambda m: log(f"pipeline: {m}"), **kw)
    torch.cuda.synchronize()
    t1 = time.time()
    log(f"pipeline: global search {t1 - t0:.1f} s, {len(found)} recovered")
    si, wi = D.overlapping_windows(table, found, T)
    th_si = torch.as_tensor(found[si], device="cuda")
    d_res = api.gb_add_templates(ctx.handle, table, th_si, wi, -1.0, d) if len(si) else d
    # global noise estimates (Sec. III F) over the block's segments (each clipped to its window)
    seg_bins = np.stack([np.ceil(segs[:, 0] * T), np.ceil(segs[:, 1] * T)], axis=1).astype(np.int64)
    seg_bins[:, 0] = np.maximum(seg_bins[:, 0], table[:, 0])
    seg_bins[:, 1] = np.minimum(seg_bins[:, 1], table[:, 0] + table[:, 1])
    noise_fit = {}
    w_post = w
    t_noise = time.time()
    L_welch, M_ser = 16384, int(round(T / I.DT))
    j_lo = -((-int(seg_bins[:, 0].min()) * L_welch) // M_ser)           # ceil(lo L / M)
    j_hi = ((int(seg_bins[:, 1].max()) - 1) * L_welch) // M_ser
    n_welch = j_hi - j_lo + 1
    if n_welch < 70:
        noise_fit = {"skipped": f"the block's band holds {n_welch} Welch bins of {L_welch} samples, fewer than the "
                                f"70-bin Savitzky-Golay window: the posterior uses the PSD"}
        posterior_noise = "psd"
    for kind, dd in (() if n_welch < 70 else
                     (("residual", d_res),
                      ("partial", api.gb_add_templates(ctx.handle, table, th_si, wi, -S_PARTIAL, d) if len(si) else d))):
        w_k, S_k, _, _ = api.gb_noise_global(table, seg_bins, dd, T, I.DT)
        ratio = S_k.cpu().numpy() / wl.psd
        noise_fit[kind] = {"median_S_over_psd": round(float(np.median(ratio)), 4),
                           "p05_p95": [round(float(np.quantile(ratio, 0.05)), 4),
                                       round(float(np.quantile(ratio, 0.95)), 4)]}
        if kind == posterior_noise:
            w_post = w_k
    torch.cuda.synchronize()
    log(f"pipeline: global noise estimates {time.time() - t_noise:.2f} s: {noise_fit}")
    states, acc, _ = D.posterior_batch(ctx, table, T, d_res, w_post, found, found_seg, boxes, seed=7, n=10000,
                                       precision=prec)
    torch.cuda.synchronize()
    t2 = time.time()
    log(f"pipeline: posteriors {t2 - t1:.1f} s ({(t2 - t1) / max(1, len(found)):.4f} s per source)")
    delta, which, overlap = D.match_delta(ctx, table, T, w, found, found_seg, inj)
    matched = delta < 0.3
    inj_matched = np.unique(which[matched])
    if catalogue:
        np.savez(catalogue, recovered=found, recovered_segment=found_seg, delta=delta, matched_injection=which,
                 overlap=overlap, injected=inj, injected_segment=inj_seg, injected_rho=rho_opt, segments=segs,
                 posterior_mean=(states.mean(axis=1) if len(states) else np.zeros((0, 8))),
                 posterior_std=(states.std(axis=1) if len(states) else np.zeros((0, 8))))
    return {
        "workload": f"full band 0.3-30 mHz in 4000 segments, 20,000 GBs, T=2^22*15 s, PSD noise; segments "
                    f"{'all' if segments is None else f'{segments[0]}..{segments[1] - 1}'} "
                    f"({segs[0, 0] * 1e3:.3f}-{segs[-1, 1] * 1e3:.3f} mHz)",
        "segments": int(wl.n_win),
        "injected": int(len(inj)), "injected_snr_gt_9": int((rho_opt > 9).sum()),
        "injected_snr_gt_10": int((rho_opt > 10).sum()),
        "recovered": int(len(found)), "matched_delta_lt_0.3": int(matched.sum()),
        "match_rate_delta": round(float(matched.mean()), 4) if len(found) else None,
        "matched_overlap_gt_0.9": int((overlap > 0.9).sum()),
        "injected_matched": int(len(inj_matched)),
        "injected_snr_gt_9_matched": int((rho_opt[inj_matched] > 9).sum()),
        "delta_median": (round(float(np.median(delta)), 5) if len(delta) else None),
        "seconds_search": round(t1 - t0, 2), "seconds_posterior": round(t2 - t1, 2),
        "seconds_posterior_per_source": round((t2 - t1) / max(1, len(found)), 5),
        "posterior_accepted_median": (np.median(acc, axis=0).astype(int).tolist() if len(acc) else None),
        "search": f"Algorithm 3, runs (even, 3), (odd, 10), (even, 10); {kw['n_searches']} searches per signal, "
                  f"DE/{kw['strategy'][:-1]}/1/bin {kw['pop']} x up to {kw['generations']} "
                  f"(stop at spread {kw['tol']} of the mean), "
                  f"polish {kw['polish_iterations']} iterations, "
                  f"{kw['joint_sweeps']} joint sweeps, rho threshold 9",
        "precision": f"likelihood {precision} (search and posterior), gradient mixed, templates for "
                     f"subtraction and Fisher FP64",
        "noise": (("search: per-segment median periodogram of the residual, updated after every found "
                   "signal" if noise == "median" else "search: the PSD") +
                  {"partial": f"; posterior: global estimate (Welch, median clip, Savitzky-Golay, spline) of the "
                              f"partial residual d - {S_PARTIAL} sum s",
                   "residual": "; posterior: global estimate of the residual",
                   "psd": "; posterior: the PSD"}[posterior_noise] + "; match metric: the PSD"),
        "noise_estimate_vs_psd": noise_fit,
        "context": "paper: 6 h on a CPU cluster (3300 core hours) for the 2-yr LDC1-4 band search; 1.8 s per "
                   "posterior on a laptop GPU; different data and hardware",
    }


def cpu_baseline(wl, seconds, logL_gpu, rho_w, log, grad_gpu=None, grad_acc=None):
    """The oracle, unmodified, on a stratified sample of the same workload: a few candidates of
    windows spread over every (N, C) group; logL and gradient of each, on all host threads and
    on one.  Also reports the largest disagreement with the GPU values of the same candidates:
    mixed logL differences, and (into grad_acc) the mixed gradient's error against sqrt(F_ii)."""
    import numpy as np

    from oracle import oracle as O
    g = O.Geometry(wl.T)
    threads = O.max_threads()
    order = sorted(range(wl.n_win), key=lambda i: (wl.windows[i].N, wl.windows[i].C))
    sample = order[:: max(1, len(order) // 16)][:16]
    check = sample   # the accuracy checks below: the same 16 windows whatever the timing sample
    lg = np.asarray(logL_gpu)

    def run(n_cand, sample, nthreads=0):
        nonlocal_max = 0.0
        t = time.time()
        evals = 0
        for i in sample:
            win = wl.windows[i]
            dd, ww = wl.window_data(i)
            th = wl.window_theta(i)[:n_cand]
            a = int(wl.cand_off[i])
            l, _ = O.loglik(th, win.k0, win.W, win.N, win.C, dd, ww, g, nthreads)
            O.loglik_grad(th, win.k0, win.W, win.N, win.C, dd, ww, g, nthreads)
            evals += 2 * len(th)
            ref = lg[a:a + len(th)]
            dl = (ref - ref[0]) - (l - l[0])
            nonlocal_max = max(nonlocal_max, float(np.max(np.abs(dl) / np.maximum(1.0, np.abs(l - l[0])))))
        return evals, time.time() - t, nonlocal_max

    # pilot, then size the sample to `seconds`: more candidates per window up to all of a
    # window's, then more windows (at most 64), spread over the (N, C) groups
    ev1, dt1, _ = run(256, sample)
    per = max(dt1, 1e-3) / (256 * len(sample))
    n_cand = int(min(10000, max(256, seconds / (per * len(sample)))))
    if n_cand == 10000:
        n_w = int(min(64, len(order), max(16, seconds / (per * 10000))))
        sample = order[:: max(1, len(order) // n_w)][:n_w]
    evals, spent, max_dl = run(n_cand, sample)
    # one core: the same windows, candidates cut to about a tenth of the budget
    n1 = int(max(16, min(n_cand, 0.1 * seconds / (per * threads * len(sample)))))
    ev_1, spent_1, _ = run(n1, sample, 1)
    errs = {}
    for i in check:
        win = wl.windows[i]
        dd, ww = wl.window_data(i)
        th = wl.window_theta(i)[:64]
        a = int(wl.cand_off[i])
        l, _ = O.loglik(th, win.k0, win.W, win.N, win.C, dd, ww, g, 0)
        ref = lg[a:a + len(th)]
        e = float(np.max(np.abs((ref - ref[0]) - (l - l[0])) / np.maximum(1.0, np.abs(l - l[0]))))
        errs[f"window {i} (N={win.N}, C={win.C}, rho={rho_w[i]:.0f})"] = e
    if grad_gpu is not None and grad_acc is not None:
        # mixed gradients of 4 rows in each of 16 sampled windows against the oracle gradient, in
        # units of sqrt(F_ii) (the oracle's Fisher matrix at the row)
        e_f, norm = [], []
        for i in check:
            win = wl.windows[i]
            dd, ww = wl.window_data(i)
            a = int(wl.cand_off[i])
            th = wl.window_theta(i)[:4]
            gg = grad_gpu[a:a + len(th)].cpu().numpy()
            _, go = O.loglik_grad(th, win.k0, win.W, win.N, win.C, dd, ww, g, 0)
            _, co = O.loglik(th, win.k0, win.W, win.N, win.C, dd, ww, g, 0)
            ddv = float(np.sum(ww * np.abs(dd) ** 2))
            for b in range(len(th)):
                F = O.fisher(th[b], win.k0, win.W, win.N, win.C, ww, g)
                e_f.append(float(np.max(np.abs(gg[b] - go[b]) / np.sqrt(np.maximum(np.diag(F), 1e-300)))))
                norm.append(math.sqrt(ddv + co[b, 1]))
        e_f, norm = np.array(e_f), np.array(norm)
        quiet = norm <= GRAD_NORM_LIMIT
        grad_acc["sampled_rows"] = int(len(e_f))
        grad_acc["sampled_worst_err_over_sqrtF"] = float(e_f.max())
        grad_acc["sampled_median_err_over_sqrtF"] = float(np.median(e_f))
        grad_acc["sampled_frac_within_bar"] = float(np.mean(e_f <= 1e-5))
        grad_acc["sampled_worst_within_norm_limit"] = float(e_f[quiet].max()) if quiet.any() else None
        grad_acc["sampled_worst_err_over_sqrtF_norm"] = float(np.max(e_f / norm))
    log(f"cpu oracle: {evals} evals in {spent:.1f}s on {threads} threads; one core: {ev_1} in {spent_1:.1f}s")
    return {"value": round(evals / spent, 2), "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(sample)} windows spread over the (N, C) groups x {n_cand} candidates each, "
                      f"logL + gradient per candidate (FP64 C++ oracle, OpenMP over candidates)",
            "cpu": cpu_model(),
            "one_core": {"value": round(ev_1 / spent_1, 2), "unit": "evals/s", "cores": 1,
                         "sample": f"the same {len(sample)} windows x {n1} candidates"},
            "mixed_dlogl_err_vs_oracle": errs}


if __name__ == "__main__":
    main()
