"""Second-generation TDI (a context created with tdi_generation = 2) against the oracle for the
same generation, which is itself pinned to the sixteen-link time-domain combination
(tests/test_oracle_pins.py): FP64 templates at every N and C, FP64 and mixed log-likelihoods on
a ragged batch whose data hold second-generation injections and noise, and mixed gradients
against the oracle's dual-number gradient."""

import numpy as np
import pytest
import torch

from paper_2307_03763_amd import api
from paper_2307_03763_amd import inputs as I
from tests.gpu_common import banner, check_logl_and_grad, delta_logl_error, dev, loglik_tolerance, rel_l2, window_dd
from tests.test_gpu_grad import MIXED_NAT, _scales, _workload
from tests.test_gpu_parity import MIXED_SLOPE

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N", [64, 128, 256, 512, 1024])
@pytest.mark.parametrize("C", [2, 3])
def test_tdi2_waveform_fp64(oracle_lib, N, C):
    banner(f"second-generation templates, FP64, N={N} C={C}")
    O = oracle_lib
    rng = np.random.default_rng(700 + N + C)
    T = I.T1
    f = np.exp(rng.uniform(np.log(0.5e-3), np.log(25e-3), 12))
    th = I.make_theta(f, I.fdot_gr(f, 0.6), 10 ** rng.uniform(-23, -21, 12), I.random_angles(rng, 12))
    ctx = api.context_for(T, tdi=2)
    h, fb = ctx.waveform(dev(th), N, C, api.GB_FP64)
    h, fb = h.cpu().numpy(), fb.cpu().numpy()
    ho, fbo = O.waveform(th, N, C, O.Geometry(T, tdi=2))
    h1, _ = O.waveform(th, N, C, O.Geometry(T, tdi=1))
    assert np.array_equal(fb, fbo)
    for b in range(len(th)):
        assert rel_l2(h[b], ho[b]) <= 1e-10, (b, rel_l2(h[b], ho[b]))
        assert rel_l2(h1[b], ho[b]) > 1e-3          # the generations differ
    ctx.close()


@pytest.fixture(scope="module")
def tdi2_batch(oracle_lib):
    O = oracle_lib
    wl = I.workload_c3(O.template_fn(), n_win=16, n_cand=8)
    wl.tdi = 2
    return I.finalize_data(wl, O.template_fn(tdi=2), np.random.default_rng(77))


def test_tdi2_loglik_fp64_and_mixed(oracle_lib, tdi2_batch):
    banner("second-generation logL: 16 ragged windows (N 64-512, C 2-3), FP64 and mixed")
    O = oracle_lib
    wl = tdi2_batch
    g = O.Geometry(wl.T, tdi=2)
    dd = window_dd(wl)
    ctx = api.context_for(wl.T, tdi=2)
    d, w, th = dev(wl.data, torch.complex128), dev(wl.weights), dev(wl.theta)
    out = {}
    for prec in (api.GB_FP64, api.GB_MIXED):
        plan = api.Plan(ctx, wl.window_table(), prec)
        plan.prepare(d, w)
        out[prec] = plan.loglik(th, comps=True)[0].cpu().numpy()
        plan.close()
    for i, win in enumerate(wl.windows):
        a, n = int(wl.cand_off[i]), int(wl.n_cand[i])
        dw, ww = wl.window_data(i)
        lo, co = O.loglik(wl.window_theta(i), win.k0, win.W, win.N, win.C, dw, ww, g)
        _, cs = O.loglik(win.sources, win.k0, win.W, win.N, win.C, dw, ww, g)
        rho = float(np.sqrt(cs[:, 1].max()))
        tol = loglik_tolerance(dd[i], co[:, 0], co[:, 1])
        assert np.all(np.abs(out[api.GB_FP64][a:a + n] - lo) <= tol), i
        lm = out[api.GB_MIXED][a:a + n]
        e = delta_logl_error(lm, lo, lm[0], lo[0]).max()
        assert e <= max(1e-5, MIXED_SLOPE * rho), (i, e, rho)
    ctx.close()


def test_tdi2_gradient_mixed(oracle_lib, tdi2_batch):
    banner("second-generation mixed gradient against the oracle's dual-number gradient")
    O = oracle_lib
    wl = tdi2_batch
    g = O.Geometry(wl.T, tdi=2)
    ctx = api.context_for(wl.T, tdi=2)
    plan = api.Plan(ctx, wl.window_table(), api.GB_MIXED)
    d, w = dev(wl.data, torch.complex128), dev(wl.weights)
    plan.prepare(d, w)
    _, gr = plan.loglik_grad(dev(wl.theta))
    gr = gr.cpu().numpy()
    worst = np.zeros(8)
    for i, win in enumerate(wl.windows):
        a, n = int(wl.cand_off[i]), int(wl.n_cand[i])
        dw, ww = wl.window_data(i)
        th = wl.window_theta(i)
        _, go = O.loglik_grad(th, win.k0, win.W, win.N, win.C, dw, ww, g)
        _, co = O.loglik(th, win.k0, win.W, win.N, win.C, dw, ww, g)
        sc = _scales(O, wl, i, th, co[:, 1])
        worst = np.maximum(worst, (np.abs(gr[a:a + n] - go) / sc).max(axis=0))
    banner("  worst scaled error per parameter: " + " ".join(f"{x:.1e}" for x in worst))
    assert worst.max() <= MIXED_NAT
    plan.close()
    ctx.close()


def test_tdi2_high_frequency(oracle_lib):
    """Second generation on windows at 30-60 mHz, where the link arguments reach the quotient
    form of the sinc above about 38 mHz: FP64 and mixed logL and the mixed gradient against the
    oracle."""
    O = oracle_lib
    banner("second generation at 30-60 mHz: FP64 and mixed logL, mixed gradient")
    wl = _workload(O, 3, f_lo=30e-3, f_span=30e-3)
    wl.tdi = 2
    wl = I.finalize_data(wl, O.template_fn(tdi=2), np.random.default_rng(78))
    f = np.array([w.sources[0, 0] for w in wl.windows])
    assert np.any(f > 40e-3), f
    ctx = api.context_for(wl.T, tdi=2)
    worst = check_logl_and_grad(O, ctx, wl, O.Geometry(wl.T, tdi=2))
    banner(f"  mixed gradient: worst error / natural scale {worst:.2e}")
    ctx.close()
