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
