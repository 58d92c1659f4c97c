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
