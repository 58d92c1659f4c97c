"""Helpers shared by the GPU tests: build workloads with oracle injections, run both sides."""

import math

import numpy as np
import torch

from paper_2307_03763_amd import api
from paper_2307_03763_amd import inputs as I


def banner(msg: str):
    print(f"[gpu-test] {msg}", flush=True)


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def loglik_tolerance(dd, dh, hh, rel=1e-10):
    """|logL_gpu - logL_oracle| bound: rel * (<d|d> + 2|<d|h>| + <h|h>) (the terms cancel)."""
    return rel * (dd + 2 * np.abs(dh) + hh)


def window_dd(wl: I.Workload):
    out = []
    for i in range(wl.n_win):
        d, w = wl.window_data(i)
        out.append(float(np.sum(w * np.abs(d) ** 2)))
    return np.array(out)


def run_gpu_loglik(wl: I.Workload, precision: int, comps=True, table_prec=None):
    ctx = api.context_for(wl.T)
    table = wl.window_table()
    if table_prec is not None:
        table = np.concatenate([table, np.asarray(table_prec, dtype=np.int64)[:, None]], axis=1)
    plan = api.Plan(ctx, table, precision)
    d = dev(wl.data, torch.complex128)
    w = dev(wl.weights)
    plan.prepare(d, w)
    th = dev(wl.theta)
    out = plan.loglik(th, comps=comps)
    torch.cuda.synchronize()
    if comps:
        return out[0].cpu().numpy(), out[1].cpu().numpy(), (ctx, plan, d, w, th)
    return out.cpu().numpy(), None, (ctx, plan, d, w, th)


def delta_logl_error(l_gpu, l_or, ref_gpu, ref_or):
    """Error of logL differences against a reference point, relative to max(1, |difference|)."""
    dg = l_gpu - ref_gpu
    do = l_or - ref_or
    return np.abs(dg - do) / np.maximum(1.0, np.abs(do))


def check_logl_and_grad(O, ctx, wl: I.Workload, g):
    """FP64 logL within the FP64 bound, mixed logL differences within the mixed model (slope
    times the loudest injection's SNR), and the mixed gradient within the bar of the natural
    scale, all against the oracle with geometry g, on every window of wl under context ctx.
    Returns the gradient's worst error over the natural scale."""
    from tests.test_gpu_grad import MIXED_NAT, _scales
    from tests.test_gpu_parity import MIXED_SLOPE
    d, w, th = dev(wl.data, torch.complex128), dev(wl.weights), dev(wl.theta)
    dd = window_dd(wl)
    worst = 0.0
    for prec in (api.GB_FP64, api.GB_MIXED):
        plan = api.Plan(ctx, wl.window_table(), prec)
        plan.prepare(d, w)
        l = plan.loglik(th).cpu().numpy()
        for i in range(wl.n_win):
            win = wl.windows[i]
            a, n = int(wl.cand_off[i]), int(wl.n_cand[i])
            dw, ww = wl.window_data(i)
            lo, co = O.loglik(wl.theta[a:a + n], win.k0, win.W, win.N, win.C, dw, ww, g)
            if prec == api.GB_FP64:
                tol = loglik_tolerance(dd[i], co[:, 0], co[:, 1])
                assert np.all(np.abs(l[a:a + n] - lo) <= tol), i
            else:
                _, cs = O.loglik(win.sources, win.k0, win.W, win.N, win.C, dw, ww, g)
                rho = float(np.sqrt(cs[:, 1].max()))
                e = delta_logl_error(l[a:a + n], lo, l[a], lo[0]).max()
                assert e <= max(1e-5, MIXED_SLOPE * rho), (i, e, rho)
        if prec == api.GB_MIXED:
            _, gr = plan.loglik_grad(th)
            gr = gr.cpu().numpy()
            for i in range(wl.n_win):
                win = wl.windows[i]
                a, n = int(wl.cand_off[i]), int(wl.n_cand[i])
                dw, ww = wl.window_data(i)
                _, go = O.loglik_grad(wl.theta[a:a + n], win.k0, win.W, win.N, win.C, dw, ww, g)
                _, co = O.loglik(wl.theta[a:a + n], win.k0, win.W, win.N, win.C, dw, ww, g)
                err = np.abs(gr[a:a + n] - go) / _scales(O, wl, i, wl.theta[a:a + n], co[:, 1])
                worst = max(worst, float(err.max()))
                assert err.max() <= MIXED_NAT, (i, err.max(axis=0))
        plan.close()
    return worst
