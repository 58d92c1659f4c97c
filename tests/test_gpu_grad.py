"""GPU gradient parity: the hand-written adjoint against the oracle's dual-number gradient and
against central differences of the GPU logL.

Scale of a gradient component: |dlogL/dtheta_i| <= ||d - h|| ||d_i h|| <= sqrt(F_ii (<d|d> + <h|h>))
up to a factor of order one, so errors are measured against s_i = sqrt(F_ii (<d|d> + <h|h>)).
Bars: FP64 1e-9 s_i; mixed precision MIXED_NAT s_i.  The mixed error is the FP32 template's
relative error (about 5e-7) times the residual norm, so measured against the gradient's own
noise scale sqrt(F_ii) it grows like sqrt(<d|d> + <h|h>): the full-size tests state it there.

The torch.autograd wrapper (api.loglik) returns the library's gradient through the chain rule.

The FP64 gradient is switched off in the library (its kernels faulted on the GPU while a CPU
emulation of the same source is clean; cause not yet known), so its cases are skipped and a test
checks that the call is refused with GB_EUNSUPPORTED before any kernel runs.
"""

import math

import numpy as np
import pytest
import torch

from paper_2307_03763_amd import api
from paper_2307_03763_amd import inputs as I
from tests.gpu_common import banner, dev, window_dd

pytestmark = pytest.mark.gpu


def _workload(oracle_lib, C, f_lo=12e-3, f_span=4e-3):
    """Gradient workload shaped like the paper's windows, small enough for the oracle.  C = 3
    moves every window to a frequency in [f_lo, f_lo + f_span] above f*/2, so the T channel is
    used."""
    wl = I.workload_c4(oracle_lib.template_fn(), n_win=6, n_cand=9)
    if C == 3:
        T = wl.T
        wins, thetas = [], []
        rng = np.random.default_rng(31)
        for w in wl.windows:
            fc = f_lo + rng.uniform(0, f_span)
            q = int(fc * T)
            k0 = q - w.W // 2
            src = I.make_theta([(q + 0.3) / T], I.fdot_gr(fc, 0.5), 2e-22, I.random_angles(rng, 1))
            wins.append(I.WindowSpec(k0, w.W, w.N, 3, k0 / T, (k0 + w.W) / T, src))
            box = I.table1_box((k0 + w.W / 6) / T, (k0 + 5 * w.W / 6) / T, T)
            thetas.append(I.draw_gaussian_around(rng, src[0], box, 1e-3, 9))
        wl = I._concat(wins, thetas, "grad C=3", T)
        I.finalize_data(wl, oracle_lib.template_fn(), np.random.default_rng(32))
    return wl


def _scales(O, wl, i, th, comps_hh):
    w = wl.windows[i]
    _, ww = wl.window_data(i)
    g = O.Geometry(wl.T, tdi=wl.tdi)
    dd = float(np.sum(ww * np.abs(wl.window_data(i)[0]) ** 2))
    out = []
    for b in range(len(th)):
        F = O.fisher(th[b], w.k0, w.W, w.N, w.C, ww, g)
        out.append(np.sqrt(np.maximum(np.diag(F), 0) * (dd + comps_hh[b])))
    return np.array(out)


def _run(wl, prec):
    ctx = api.context_for(wl.T)
    plan = api.Plan(ctx, wl.window_table(), prec)
    d, w = dev(wl.data, torch.complex128), dev(wl.weights)
    plan.prepare(d, w)
    th = dev(wl.theta)
    l, g = plan.loglik_grad(th)
    l2 = plan.loglik(th)
    torch.cuda.synchronize()
    return l.cpu().numpy(), g.cpu().numpy(), l2.cpu().numpy(), (ctx, plan, d, w, th)


MIXED_NAT = 2e-6   # measured worst 1.1e-6 on the full-size workloads (C4), 9e-7 here

FP64_GRAD_OFF = "FP64 gradient switched off: its kernels faulted on the GPU; cause not yet known"


@pytest.mark.parametrize("C", [2, 3])
@pytest.mark.parametrize("prec,bar", [pytest.param(api.GB_FP64, 1e-9, marks=pytest.mark.skip(reason=FP64_GRAD_OFF)),
                                      (api.GB_MIXED, MIXED_NAT)])
def test_gradient_matches_oracle(oracle_lib, C, prec, bar):
    banner(f"gradient vs oracle C={C} prec={prec}")
    _check_against_oracle(oracle_lib, _workload(oracle_lib, C), prec, bar)


def test_gradient_high_frequency(oracle_lib):
    """Windows at 30-60 mHz: above about c / (pi L) = 38 mHz a link's transfer argument
    pi f L (1 +- k.n) / c can pass 2, and on those links the forward sinc and the adjoint's
    sinc derivative switch from their series to their quotient forms; the windows below keep
    the series everywhere."""
    banner("gradient vs oracle, 30-60 mHz, C=3, mixed")
    wl = _workload(oracle_lib, 3, f_lo=30e-3, f_span=30e-3)
    f = np.array([w.sources[0, 0] for w in wl.windows])
    f_series = 0.999 / (np.pi * I.ARM_L / I.C_LIGHT)      # below it every link argument is below 2
    assert np.any(f < f_series) and np.any(f > 40e-3), f
    _check_against_oracle(oracle_lib, wl, api.GB_MIXED, MIXED_NAT)


def _check_against_oracle(oracle_lib, wl, prec, bar):
    O = oracle_lib
    l, g, l2, _ = _run(wl, prec)
    worst = np.zeros(8)
    for i in range(wl.n_win):
        w = wl.windows[i]
        d, ww = wl.window_data(i)
        a, n = int(wl.cand_off[i]), int(wl.n_cand[i])
        th = wl.window_theta(i)
        lo, go = O.loglik_grad(th, w.k0, w.W, w.N, w.C, d, ww, O.Geometry(wl.T))
        _, co = O.loglik(th, w.k0, w.W, w.N, w.C, d, ww, O.Geometry(wl.T))
        sc = _scales(O, wl, i, th, co[:, 1])
        err = np.abs(g[a:a + n] - go) / sc
        worst = np.maximum(worst, err.max(axis=0))
        if prec == api.GB_FP64:
            assert np.array_equal(l[a:a + n], l2[a:a + n]) or np.allclose(l[a:a + n], l2[a:a + n], rtol=1e-13)
    banner("  worst scaled error per parameter: " + " ".join(f"{x:.1e}" for x in worst))
    assert worst.max() <= bar, worst


def test_gradient_central_differences(oracle_lib):
    """Mixed-precision GPU gradient against central differences of the FP64 GPU logL (steps 1e-6
    of the Table I widths; candidates kept away from a carrier-bin change)."""
    banner("gradient vs central differences")
    O = oracle_lib
    wl = _workload(O, 2)
    T = wl.T
    base = wl.theta.copy()
    # keep f0 T at least 0.2 from an integer so +-step never changes the carrier bin
    frac = base[:, 0] * T - np.floor(base[:, 0] * T)
    base[:, 0] += (np.clip(frac, 0.2, 0.8) - frac) / T
    wlb = I.Workload(wl.name, T, wl.windows, base, wl.n_cand, wl.cand_off, wl.data, wl.weights, wl.data_off)
    _, g0, _, _ = _run(wlb, api.GB_MIXED)
    ctx = api.context_for(T)
    plan = api.Plan(ctx, wl.window_table(), api.GB_FP64)
    d, w = dev(wl.data, torch.complex128), dev(wl.weights)
    plan.prepare(d, w)
    # Table I widths at 5 mHz: f over a 256-bin window, fdot over its bounds, angles over their ranges
    f5 = 5e-3
    widths = np.array([256.0 / T, 1.02e-6 * f5 ** (11 / 3) + 5e-6 * f5 ** (13 / 3), 1.0, 2 * math.pi, 0.0,
                       math.pi, math.pi, 2 * math.pi])
    rel_errs = []
    for i in range(8):
        hv = np.full(len(base), 1e-6 * widths[i]) if i != 4 else 1e-6 * base[:, 4]
        tp, tm = base.copy(), base.copy()
        tp[:, i] += hv
        tm[:, i] -= hv
        lp = plan.loglik(dev(tp)).cpu().numpy()
        lm = plan.loglik(dev(tm)).cpu().numpy()
        fd = (lp - lm) / (2 * hv)
        err = np.abs(fd - g0[:, i]) / np.maximum(np.abs(g0[:, i]), 1e-2 / hv)
        rel_errs.append(np.median(err))
        assert np.median(err) < 1e-4, (i, np.median(err))
    banner("  median relative FD error per parameter: " + " ".join(f"{x:.1e}" for x in rel_errs))


@pytest.fixture(scope="module")
def c3_grad(oracle_lib):
    return I.workload_c3(oracle_lib.template_fn(), n_win=16, n_cand=6)


def test_gradient_ragged_mixed(oracle_lib, c3_grad):
    """Mixed-precision gradients on ragged windows (N 64-512, C 2-3) against the oracle."""
    banner("gradient ragged mixed")
    O = oracle_lib
    wl = c3_grad
    l, g, _, _ = _run(wl, api.GB_MIXED)
    worst = np.zeros(8)
    for i in range(wl.n_win):
        w = wl.windows[i]
        d, ww = wl.window_data(i)
        a, n = int(wl.cand_off[i]), int(wl.n_cand[i])
        th = wl.window_theta(i)
        _, go = O.loglik_grad(th, w.k0, w.W, w.N, w.C, d, ww, O.Geometry(wl.T))
        _, co = O.loglik(th, w.k0, w.W, w.N, w.C, d, ww, O.Geometry(wl.T))
        sc = _scales(O, wl, i, th, co[:, 1])
        worst = np.maximum(worst, (np.abs(g[a:a + n] - go) / sc).max(axis=0))
    banner("  worst scaled error per parameter: " + " ".join(f"{x:.1e}" for x in worst))
    assert worst.max() <= MIXED_NAT


def test_gradient_edge_cases(oracle_lib):
    """Mixed gradients on the edge windows of the likelihood tests: N = 1024 with C = 3 and
    W = 4096, an empty window, a window of one bin and one of N = 64.  A template entirely outside
    its window has logL = -<d|d>/2 and a gradient of exactly zero; a zero amplitude leaves only
    dlogL/dA = <d|h_u> (the other components exactly zero); NaN parameters and a negative
    amplitude give NaN rows; every other row matches the oracle at the mixed bar."""
    banner("gradient edge cases (mixed)")
    O = oracle_lib
    T = I.T1
    rng = np.random.default_rng(17)
    specs = [(int(12e-3 * T) - 2048, 4096, 1024, 3), (int(2e-3 * T), 100, 128, 2),
             (int(5e-3 * T), 1, 256, 2), (int(1e-3 * T) - 32, 64, 64, 2)]
    ncand = [6, 0, 5, 7]
    wins, thetas = [], []
    for (k0, W, N, C), n in zip(specs, ncand):
        f = (k0 + W / 2) / T
        th = I.make_theta(np.full(n, f) + rng.uniform(-20, 20, n) / T, 1e-17, 1e-22, I.random_angles(rng, n))
        wins.append(I.WindowSpec(k0, W, N, C, k0 / T, (k0 + W) / T, th[:1] if n else np.zeros((0, 8))))
        thetas.append(th)
    thetas[2][1, 0] = (specs[2][0] + 5000) / T   # far outside its window
    thetas[2][2, 4] = 0.0                          # zero amplitude
    thetas[3][2, 2] = np.nan
    thetas[3][4, 4] = -1e-22
    wl = I._concat(wins, thetas, "grad edge", T)
    I.finalize_data(wl, O.template_fn(), np.random.default_rng(18))
    l, g, _, _ = _run(wl, api.GB_MIXED)
    g_or = O.Geometry(T)
    worst = 0.0
    for i in range(wl.n_win):
        w = wl.windows[i]
        d, ww = wl.window_data(i)
        a, n = int(wl.cand_off[i]), int(wl.n_cand[i])
        if n == 0:
            continue
        th = wl.window_theta(i)
        ok = np.isfinite(th).all(axis=1) & (th[:, 4] >= 0)
        assert np.all(np.isnan(l[a:a + n][~ok])) and np.all(np.isnan(g[a:a + n][~ok]))
        _, go = O.loglik_grad(th[ok], w.k0, w.W, w.N, w.C, d, ww, g_or)
        _, co = O.loglik(th[ok], w.k0, w.W, w.N, w.C, d, ww, g_or)
        sc = _scales(O, wl, i, th[ok], co[:, 1])
        err = np.abs(g[a:a + n][ok] - go) / np.where(sc > 0, sc, 1.0)
        worst = max(worst, float(err.max()))
        assert err.max() <= MIXED_NAT, (i, err.max(axis=0))
    dd = float(np.sum(wl.window_data(2)[1] * np.abs(wl.window_data(2)[0]) ** 2))
    a = int(wl.cand_off[2])
    assert abs(l[a + 1] + 0.5 * dd) <= 1e-12 * dd and np.all(g[a + 1] == 0.0)
    assert np.all(g[a + 2][[0, 1, 2, 3, 5, 6, 7]] == 0.0) and g[a + 2][4] != 0.0
    banner(f"  worst scaled error {worst:.1e}")


def test_fp64_gradient_is_refused(c3_grad):
    """The FP64 gradient is switched off: the call returns GB_EUNSUPPORTED and launches nothing."""
    banner("fp64 gradient refused")
    wl = c3_grad
    ctx = api.context_for(wl.T)
    plan = api.Plan(ctx, wl.window_table(), api.GB_FP64)
    d, w = dev(wl.data, torch.complex128), dev(wl.weights)
    plan.prepare(d, w)
    with pytest.raises(api.GbxError) as e:
        plan.loglik_grad(dev(wl.theta))
    assert e.value.status == api.GB_EUNSUPPORTED
    assert "FP64 gradient" in str(e.value)


def test_autograd_function(oracle_lib):
    banner("torch.autograd wrapper of the adjoint gradient (mixed plan)")
    wl = _workload(oracle_lib, 2)
    l, g, _, (ctx, plan, d, w, th) = _run(wl, api.GB_MIXED)
    x = th.clone().requires_grad_(True)
    out = api.loglik(plan, x)
    assert out.requires_grad and torch.equal(out.detach().cpu(), torch.as_tensor(l))
    weights = torch.linspace(0.5, 2.0, len(out), dtype=torch.float64, device=out.device)
    (weights * out).sum().backward()
    # the chain rule with the library's gradient, bit for bit (the kernels are deterministic)
    assert torch.equal(x.grad.cpu(), (weights[:, None] * torch.as_tensor(g, device=out.device)).cpu())
    # composes with other torch operations: d/dtheta of sum(exp(logL - max)) = softmax-weighted gradient
    x.grad = None
    y = api.loglik(plan, x)
    z = torch.exp(y - y.max().detach()).sum()
    z.backward()
    ref = torch.exp(torch.as_tensor(l) - torch.as_tensor(l).max())[:, None] * torch.as_tensor(g)
    np.testing.assert_allclose(x.grad.cpu().numpy(), ref.numpy(), rtol=1e-12, atol=0)
    plan.close()
    ctx.close()
