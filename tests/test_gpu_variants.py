"""Every compiled launch shape of the likelihood and gradient kernels against the oracle.

For each (precision, mode, N, C) the autotuner keeps whichever compiled shape is fastest on the
device at hand. A shape is a number of lanes per template (4 or 8 slow-series samples per lane),
a number of waves per workgroup (4, or 2 for templates of two waves) and a register budget.
Each shape is selected in turn and run on three ragged windows of that N and C, one narrower
than the template, with candidate counts that leave partial tiles.

* FP64 logL must meet the 1e-10 bar.
* Mixed logL must meet the mixed error model.
* The mixed gradient must meet the bar of its own parity test (MIXED_NAT); its logL must meet the
  mixed model too.
"""

import math

import numpy as np
import pytest

from paper_2307_03763_amd import api
from paper_2307_03763_amd import inputs as I
from tests.gpu_common import banner, delta_logl_error, dev, loglik_tolerance, window_dd
from tests.test_gpu_grad import MIXED_NAT, _scales
from tests.test_gpu_parity import MIXED_SLOPE

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MODE_LOGLIK, MODE_GRAD = 1, 2


def _group(O, N, C, seed):
    """Three windows of N samples and C channels: widths N/2 + 13, N + 7 and 2N bins; 9, 23 and
    5 candidates drawn around each window's injected source."""
    T = I.T1
    rng = np.random.default_rng(seed)
    wins, thetas = [], []
    for i, (W, n) in enumerate(((N // 2 + 13, 9), (N + 7, 23), (2 * N, 5))):
        fc = (2e-3 if C == 2 else 12e-3) + 1e-3 * i + rng.uniform(0, 5e-4)
        q = int(fc * T)
        k0 = q - W // 2
        src = I.make_theta([(q + 0.3) / T], I.fdot_gr(fc, 0.5), 3e-22, I.random_angles(rng, 1))
        wins.append(I.WindowSpec(k0, W, N, C, k0 / T, (k0 + W) / T, src))
        box = I.table1_box((k0 + W / 6) / T, (k0 + 5 * W / 6) / T, T)
        thetas.append(I.draw_gaussian_around(rng, src[0], box, 1e-3, n))
    wl = I._concat(wins, thetas, f"launch shapes N={N} C={C}", T)
    I.finalize_data(wl, O.template_fn(), np.random.default_rng(seed + 1))
    return wl


def _shapes(N):
    out = [(N // 4, 4), (N // 8, 4)]
    if N in (512, 1024):
        out.append((128, 2))
    return out


def _reference(O, wl, grad):
    g = O.Geometry(wl.T)
    ref = []
    for i in range(wl.n_win):
        w = wl.windows[i]
        d, ww = wl.window_data(i)
        th = wl.window_theta(i)
        lo, co = O.loglik(th, w.k0, w.W, w.N, w.C, d, ww, g)
        _, cs = O.loglik(w.sources, w.k0, w.W, w.N, w.C, d, ww, g)
        r = dict(lo=lo, co=co, rho=math.sqrt(cs[:, 1].max()))
        if grad:
            _, go = O.loglik_grad(th, w.k0, w.W, w.N, w.C, d, ww, g)
            r["go"] = go
            r["sc"] = _scales(O, wl, i, th, co[:, 1])
        ref.append(r)
    return ref


@pytest.mark.parametrize("N", [64, 128, 256, 512, 1024])
@pytest.mark.parametrize("C", [2, 3])
def test_every_launch_shape(oracle_lib, N, C):
    banner(f"every compiled launch shape, N={N} C={C}")
    O = oracle_lib
    wl = _group(O, N, C, seed=900 + 10 * N + C)
    ref = _reference(O, wl, grad=True)
    dd = window_dd(wl)
    ctx = api.context_for(wl.T)
    d, w, th = dev(wl.data, torch.complex128), dev(wl.weights), dev(wl.theta)
    ran = {}
    for prec, mode in ((api.GB_FP64, MODE_LOGLIK), (api.GB_MIXED, MODE_LOGLIK), (api.GB_MIXED, MODE_GRAD)):
        for lpc, wpb in _shapes(N):
            for occ in (1, 2, 3, 4):
                try:
                    api.gb_select_variant(ctx.handle, prec, mode, N, C, lpc, wpb, occ)
                except api.GbxError:
                    continue                         # not compiled
                shape = f"prec={prec} mode={mode} lanes={lpc} waves={wpb} occ={occ}"
                ran[(prec, mode)] = ran.get((prec, mode), 0) + 1
                plan = api.Plan(ctx, wl.window_table(), prec)
                plan.prepare(d, w)
                if mode == MODE_GRAD:
                    l, g = plan.loglik_grad(th)
                    g = g.cpu().numpy()
                else:
                    l = plan.loglik(th)
                torch.cuda.synchronize()
                l = l.cpu().numpy()
                for i in range(wl.n_win):
                    a, n = int(wl.cand_off[i]), int(wl.n_cand[i])
                    r = ref[i]
                    if prec == api.GB_FP64:
                        tol = loglik_tolerance(dd[i], r["co"][:, 0], r["co"][:, 1])
                        assert np.all(np.abs(l[a:a + n] - r["lo"]) <= tol), (shape, i)
                    else:
                        e = delta_logl_error(l[a:a + n], r["lo"], l[a], r["lo"][0]).max()
                        assert e <= max(1e-5, MIXED_SLOPE * r["rho"]), (shape, i, e, r["rho"])
                    if mode == MODE_GRAD:
                        err = np.abs(g[a:a + n] - r["go"]) / r["sc"]
                        assert err.max() <= MIXED_NAT, (shape, i, err.max(axis=0))
                plan.close()
    banner("  shapes run: " + ", ".join(f"prec={p} mode={m}: {k}" for (p, m), k in sorted(ran.items())))
    # every family has at least the two lane counts at one register budget
    assert all(ran.get(k, 0) >= 2 for k in ((api.GB_FP64, MODE_LOGLIK), (api.GB_MIXED, MODE_LOGLIK),
                                             (api.GB_MIXED, MODE_GRAD))), ran
    ctx.close()


def test_autotune_on_windows(oracle_lib):
    """gb_autotune_windows tunes exactly the families its windows hold (logL in both precisions,
    the gradient in mixed), on all of their candidates (37 here), names compiled kernels of those
    families, and plans created afterwards meet the oracle bars.  Arrays too small for the
    windows, and null arrays, are refused on the host."""
    banner("autotune on windows, N=256 C=3")
    O = oracle_lib
    wl = _group(O, 256, 3, seed=4242)
    ref = _reference(O, wl, grad=True)
    dd = window_dd(wl)
    ctx = api.context_for(wl.T)
    d, w, th = dev(wl.data, torch.complex128), dev(wl.weights), dev(wl.theta)
    table = wl.window_table()
    rep = api.gb_autotune_windows(ctx.handle, table, d, w, th, 2)
    banner("  " + rep.replace("\n", "\n[gpu-test]   "))
    lines = [l for l in rep.splitlines() if l.strip()]
    heads = sorted(l.split(":", 1)[0] for l in lines)
    assert heads == ["fp64  loglik N=256 C=3", "mixed grad   N=256 C=3", "mixed loglik N=256 C=3"], heads
    for l in lines:
        assert f"/ {int(wl.n_cand.sum())} (" in l, l
        kern = l.split("kernel=", 1)[1]
        r, N, lpc, C, wpb, mode, occ = kern[len("k_batch<"):-1].split(",")
        assert (N, C) == ("256", "3")
        assert r == ("double" if l.startswith("fp64") else "float")
        assert mode == ("2" if "grad" in l else "1")
        api.gb_select_variant(ctx.handle, api.GB_FP64 if r == "double" else api.GB_MIXED, int(mode), 256, 3,
                              int(lpc), int(wpb), int(occ))      # a compiled variant
    # re-apply the report (gb_select_variant above leaves the same choice) and check the plans
    assert api.apply_tuning(ctx.handle, rep) == 3
    for prec in (api.GB_FP64, api.GB_MIXED):
        plan = api.Plan(ctx, table, prec)
        plan.prepare(d, w)
        l = plan.loglik(th)
        if prec == api.GB_MIXED:
            l2, g = plan.loglik_grad(th)
            g = g.cpu().numpy()
        torch.cuda.synchronize()
        l = l.cpu().numpy()
        for i in range(wl.n_win):
            a, n = int(wl.cand_off[i]), int(wl.n_cand[i])
            r = ref[i]
            if prec == api.GB_FP64:
                tol = loglik_tolerance(dd[i], r["co"][:, 0], r["co"][:, 1])
                assert np.all(np.abs(l[a:a + n] - r["lo"]) <= tol), i
            else:
                e = delta_logl_error(l[a:a + n], r["lo"], l[a], r["lo"][0]).max()
                assert e <= max(1e-5, MIXED_SLOPE * r["rho"]), (i, e)
                err = np.abs(g[a:a + n] - r["go"]) / r["sc"]
                assert err.max() <= MIXED_NAT, (i, err.max(axis=0))
        plan.close()
    with pytest.raises(ValueError):
        api.gb_autotune_windows(ctx.handle, table, d, w, th[:-1], 1)
    with pytest.raises(ValueError):
        api.gb_autotune_windows(ctx.handle, table, d[:-1], w, th, 1)
    arr = api.windows_array(table)
    assert api.lib().gb_autotune_windows(ctx.handle, arr, len(arr), None, None, None, 1, None, 0) == api.GB_EINVAL
    ctx.close()
