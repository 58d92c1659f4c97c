"""Throughput of the batched Galactic-binary likelihood on one MI355X.

One step = one pass of the hot path over the ragged batch: for every (N, C) group of windows
(one persistent launch each) the Metropolis-Hastings stage (logL of every proposal, then the
chain of every window) and the gradient of every candidate.  Inputs are synthetic and resident
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


# ------------------------------------------------------------------------------------------
# algorithmic work per evaluation (counted from the model, one FMA = 2 flops;
# sin/cos counted separately, not as flops)
def flops_per_eval(N: int, C: int, overlap: int, grad: bool) -> float:
    per_sample = 333.0 + (12.0 if C == 3 else 0.0)          # slow series (response, TDI, channels)
    fft = C * 5.0 * N * math.log2(N)                          # one radix-2-equivalent DFT per channel
    red = 20.0 * C * overlap                                  # residual and four FP64 accumulations
    f = per_sample * N + fft + red
    if grad:
        f += fft + 1290.0 * N + 6.0 * C * overlap             # inverse DFT, per-sample adjoint, cotangent
    return f


def sincos_per_eval(N: int, grad: bool) -> float:
    return (5.0 + (5.0 if grad else 0.0)) * N


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
    return ap.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}, "
              f"WORLD_SIZE={world}); multi-GPU sharding is described in DESIGN.md, not run.",
              flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2307_03763_amd import api
    from paper_2307_03763_amd import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)

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

    # one plan per (N, C) group: each is one persistent launch over all of its windows
    groups = {}
    for i, win in enumerate(wl.windows):
        groups.setdefault((win.N, win.C), []).append(i)
    keys = sorted(groups, key=lambda k: (-k[0], -k[1]))

    def make_plans(prec):
        plans = []
        for k in keys:
            p = api.Plan(ctx, table[groups[k]], prec)
            p.rows = rows
            p.prepare(d, w)
            plans.append(p)
        return plans

    plans = make_plans(api.GB_MIXED)
    stream = torch.cuda.current_stream()
    logL = torch.empty(rows, dtype=torch.float64, device="cuda")
    chain = torch.empty(rows, dtype=torch.int32, device="cuda")
    grad = torch.empty((rows, 8), dtype=torch.float64, device="cuda")
    nacc = [torch.empty(len(groups[k]), dtype=torch.int64, device="cuda") for k in keys]
    glog = torch.empty(rows, dtype=torch.float64, device="cuda")

    def step(plans, ev=None):
        for j, p in enumerate(plans):
            if ev is not None:
                ev[j][0].record(stream)
            api.gb_mh_step(p.handle, d, w, th, log_g, u, args.temperature, logL, chain, nacc[j], stream)
            if ev is not None:
                ev[j][1].record(stream)
            api.gb_loglik_grad(p.handle, d, w, th, glog, grad, stream)
            if ev is not None:
                ev[j][2].record(stream)

    for _ in range(args.warmup):
        step(plans)
    torch.cuda.synchronize()

    E = lambda: torch.cuda.Event(enable_timing=True)
    evs = [[[E(), E(), E()] for _ in keys] for _ in range(args.steps)]
    start, end = E(), E()
    torch.cuda.synchronize()
    start.record(stream)
    for s in range(args.steps):
        step(plans, evs[s])
    end.record(stream)
    torch.cuda.synchronize()
    ms_step = start.elapsed_time(end) / args.steps
    t_mh = np.array([[evs[s][j][0].elapsed_time(evs[s][j][1]) for j in range(len(keys))] for s in range(args.steps)])
    t_gr = np.array([[evs[s][j][1].elapsed_time(evs[s][j][2]) for j in range(len(keys))] for s in range(args.steps)])
    ms_logl = float(t_mh.sum(axis=1).mean())
    ms_grad = float(t_gr.sum(axis=1).mean())
    assert bool(torch.isfinite(logL).all()) and bool(torch.isfinite(grad).all()), "non-finite outputs"
    log(f"mixed ragged: {ms_step:.2f} ms/step (MH stage {ms_logl:.2f} ms, gradients {ms_grad:.2f} ms)")

    # dominant kernel: the gradient launch of the group with the largest share of the step
    j_dom = int(np.argmax(t_gr.mean(axis=0)))
    kN, kC = keys[j_dom]
    idx = groups[keys[j_dom]]
    n_dom = int(sum(wl.n_cand[i] for i in idx))
    fl = sum(int(wl.n_cand[i]) * flops_per_eval(kN, kC, min(wl.windows[i].W, kN), True) for i in idx)
    dur_ms = float(t_gr[:, j_dom].mean())
    achieved_tf = fl / (dur_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved_tf, 3), "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved_tf / PEAK_VALU_TFLOPS, 4), "traffic": None,
                "kernel": f"k_batch<float, N={kN}, C={kC}, gradient>", "launch_ms": round(dur_ms, 4),
                "evals_per_launch": n_dom,
                "hbm_gbs": round((n_dom * bytes_per_eval(kC, kN, True) +
                                  sum(24.0 * kC * wl.windows[i].W for i in idx)) / (dur_ms * 1e-3) / 1e9, 3),
                "sincos_per_s": round(sum(int(wl.n_cand[i]) for i in idx) * sincos_per_eval(kN, True) / (dur_ms * 1e-3), 1)}

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
            for p in win_plans:
                api.gb_loglik_grad(p.handle, d, w, th, glog, grad, stream)
            ev[2].record(stream)

        plain([E(), E(), E()])
        torch.cuda.synchronize()
        ev = [E(), E(), E()]
        plain(ev)
        torch.cuda.synchronize()
        f_l, f_g = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
        fp64 = {"ms_per_step": round(f_l + f_g, 3), "logl_evals_per_s": round(rows / (f_l * 1e-3), 1),
                "grad_evals_per_s": round(rows / (f_g * 1e-3), 1),
                "value": round(2 * rows / ((f_l + f_g) * 1e-3), 1)}
        log(f"plain FP64 per window: {f_l + f_g:.2f} ms/pass (MH stage {f_l:.2f}, gradients {f_g:.2f})")
        for p in win_plans:
            p.close()

    # ---------------------------------------------------------------- CPU oracle on a bounded sample
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(wl, args.cpu_seconds, logL, grad, log)

    value = 2 * rows / (ms_step * 1e-3)
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "windows": wl.n_win, "candidates": rows,
                   "groups": [f"N={k[0]},C={k[1]}:{len(groups[k])}" for k in keys],
                   "T_s": T, "precision": "mixed (FP64 phase and accumulation, FP32 response and DFT)",
                   "step": "per (N, C) group: MH stage (logL of all proposals + chains), then all gradients"},
        "logl_evals_per_s": round(rows / (ms_logl * 1e-3), 1),
        "grad_evals_per_s": round(rows / (ms_grad * 1e-3), 1),
        "fp64_plain": fp64,
        "speedup_vs_fp64": round(value / fp64["value"], 3) if fp64 else None,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "context": "paper: 1.8 s per posterior of 6 x 10,000 likelihoods on a Quadro RTX 4000 Mobile "
                   "(about 3.3e4 logL/s including chain and KDE); different hardware and work",
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(wl, seconds, logL_gpu, grad_gpu, log):
    """The oracle, unmodified, on a stratified sample of the same workload: a few candidates of
    windows spread over every (N, C) group; logL and gradient of each.  Also reports the largest
    disagreement with the GPU values of the same candidates."""
    import numpy as np

    from oracle import oracle as O
    g = O.Geometry(wl.T)
    threads = O.max_threads()
    order = sorted(range(wl.n_win), key=lambda i: (wl.windows[i].N, wl.windows[i].C))
    sample = order[:: max(1, len(order) // 16)][:16]
    lg = logL_gpu.cpu().numpy()
    def run(n_cand):
        nonlocal_max = 0.0
        t = time.time()
        evals = 0
        for i in sample:
            win = wl.windows[i]
            dd, ww = wl.window_data(i)
            th = wl.window_theta(i)[:n_cand]
            a = int(wl.cand_off[i])
            l, _ = O.loglik(th, win.k0, win.W, win.N, win.C, dd, ww, g, 0)
            O.loglik_grad(th, win.k0, win.W, win.N, win.C, dd, ww, g, 0)
            evals += 2 * len(th)
            ref = lg[a:a + len(th)]
            dl = (ref - ref[0]) - (l - l[0])
            nonlocal_max = max(nonlocal_max, float(np.max(np.abs(dl) / np.maximum(1.0, np.abs(l - l[0])))))
        return evals, time.time() - t, nonlocal_max

    _, dt1, _ = run(2)
    n_cand = int(min(4096, max(2, 2 * seconds / max(dt1, 1e-3))))
    evals, spent, max_dl = run(n_cand)
    log(f"cpu oracle: {evals} evals in {spent:.1f}s on {threads} threads")
    return {"value": round(evals / spent, 2), "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(sample)} windows spread over the (N, C) groups x {n_cand} candidates each, "
                      f"logL + gradient per candidate (FP64 C++ oracle, OpenMP over candidates)",
            "cpu": platform.processor() or platform.machine(),
            "max_mixed_dlogl_err_vs_oracle": max_dl}


if __name__ == "__main__":
    main()
