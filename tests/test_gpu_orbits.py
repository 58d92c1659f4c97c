"""Numerical orbits (gb_set_orbit) on the GPU against the oracle given the same positions.

The exact Keplerian orbits (arms breathing by +-0.24%, centroid off the ecliptic) are sampled
on a grid; the library and the oracle each interpolate them with their own code.  Templates
and likelihoods take one light time per arm.

* FP64 templates within 1e-10 (relative L2) of the oracle's, both TDI generations, every N.
* FP64 logL within the FP64 bound, mixed logL differences within the mixed model, on windows
  of both channel counts.
* Mixed gradients within the bar of the equal-arm gradient (MIXED_NAT of the natural scale)
  against the oracle's dual-number gradient; the FP64 gradient is refused as on analytic orbits.
* The general link sinc up to its quotient form above about 38 mHz (templates at 35 mHz,
  likelihoods and gradients at 25-55 mHz).
* Returning to the analytic orbits restores the equal-arm templates.
"""

import numpy as np
import pytest

from paper_2307_03763_amd import api
from paper_2307_03763_amd import inputs as I
from tests.gpu_common import banner, check_logl_and_grad, delta_logl_error, dev, loglik_tolerance, window_dd
from tests.test_gpu_grad import MIXED_NAT, _scales, _workload
from tests.test_gpu_parity import MIXED_SLOPE

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture
def kepler(oracle_lib):
    """Keplerian positions on a grid over T1, set on the oracle; cleared afterwards."""
    T = I.T1
    pos, t0, dt = I.orbit_grid(lambda t: I.keplerian_orbits(t), T, 2049)
    oracle_lib.set_orbit(pos, t0, dt)
    yield pos, t0, dt
    oracle_lib.clear_orbit()


@pytest.mark.parametrize("tdi", [1, 2])
def test_templates_on_numerical_orbits(oracle_lib, kepler, tdi):
    O = oracle_lib
    pos, t0, dt = kepler
    banner(f"numerical orbits: FP64 templates, TDI {tdi}")
    ctx = api.context_for(I.T1, tdi=tdi)
    ctx.set_orbit(pos, t0, dt)
    rng = np.random.default_rng(70 + tdi)
    g = O.Geometry(I.T1, tdi=tdi)
    worst = 0.0
    for N, C, f0 in ((64, 2, 0.8e-3), (128, 2, 3e-3), (256, 3, 11e-3), (512, 3, 18e-3), (1024, 3, 27e-3),
                     (1024, 3, 35e-3)):
        th = I.make_theta([f0 * (1 + 0.01 * k) for k in range(3)], I.fdot_gr(f0, 0.6), 1e-22,
                          I.random_angles(rng, 3))
        h, fb = ctx.waveform(dev(th), N, C, api.GB_FP64)
        ho, fbo = O.waveform(th, N, C, g)
        assert np.array_equal(fb.cpu().numpy(), fbo)
        h = h.cpu().numpy()
        for b in range(3):
            e = _rel(h[b], ho[b])
            worst = max(worst, e)
            assert e < 1e-10, (N, C, b, e)
    banner(f"  worst relative L2 {worst:.2e}")
    # back to the analytic orbits: the equal-arm templates again
    ctx.set_orbit()
    O.clear_orbit()
    th = I.make_theta([3e-3], 0.0, 1e-22, I.random_angles(rng, 1))
    h, _ = ctx.waveform(dev(th), 128, 2, api.GB_FP64)
    ho, _ = O.waveform(th, 128, 2, g)
    assert _rel(h.cpu().numpy()[0], ho[0]) < 1e-10
    ctx.close()


@pytest.mark.parametrize("tdi", [1, 2])
def test_likelihoods_on_numerical_orbits(oracle_lib, kepler, tdi):
    O = oracle_lib
    pos, t0, dt = kepler
    banner(f"numerical orbits: FP64 and mixed logL, mixed gradient, TDI {tdi}")
    ctx = api.context_for(I.T1, tdi=tdi)
    ctx.set_orbit(pos, t0, dt)
    # injections from the oracle on these orbits, noise of the generation's PSD
    wl = I.workload_c3(None, n_win=12, n_cand=40, noise=False)
    wl.tdi = tdi
    wl = I.finalize_data(wl, O.template_fn(tdi=tdi), np.random.default_rng(80 + tdi))
    g = O.Geometry(wl.T, tdi=tdi)
    d, w, th = dev(wl.data, torch.complex128), dev(wl.weights), dev(wl.theta)
    dd = window_dd(wl)
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
            # the mixed gradient against the oracle's dual-number gradient on the same orbits,
            # at the bar of the equal-arm gradient (MIXED_NAT of the natural scale)
            l2, gr = plan.loglik_grad(th)
            gr = gr.cpu().numpy()
            worst = 0.0
            for i in range(0, wl.n_win, 2):
                win = wl.windows[i]
                a, n = int(wl.cand_off[i]), min(int(wl.n_cand[i]), 6)
                dw, ww = wl.window_data(i)
                _, go = O.loglik_grad(wl.theta[a:a + n], win.k0, win.W, win.N, win.C, dw, ww, g)
                _, co = O.loglik(wl.theta[a:a + n], win.k0, win.W, win.N, win.C, dw, ww, g)
                err = np.abs(gr[a:a + n] - go) / _scales(O, wl, i, wl.theta[a:a + n], co[:, 1])
                worst = max(worst, float(err.max()))
                assert err.max() <= MIXED_NAT, (i, err.max(axis=0))
            banner(f"  mixed gradient: worst error / natural scale {worst:.2e}")
        plan.close()
    # the FP64 gradient stays switched off on these orbits as on the analytic ones
    plan = api.Plan(ctx, wl.window_table(), api.GB_FP64)
    plan.prepare(d, w)
    with pytest.raises(api.GbxError) as err:
        plan.loglik_grad(th)
    assert err.value.status == api.GB_EUNSUPPORTED
    plan.close()
    ctx.close()


@pytest.mark.parametrize("tdi", [1, 2])
def test_high_frequency_on_numerical_orbits(oracle_lib, kepler, tdi):
    """Windows at 25-55 mHz on the same orbits, where the link arguments reach the quotient form
    of the sinc above about 38 mHz: FP64 and mixed logL and the mixed gradient against the
    oracle, both TDI generations."""
    O = oracle_lib
    pos, t0, dt = kepler
    banner(f"numerical orbits: 25-55 mHz, FP64 and mixed logL, mixed gradient, TDI {tdi}")
    wl = _workload(O, 3, f_lo=25e-3, f_span=30e-3)   # injections from the oracle on these orbits
    if tdi == 2:
        wl.tdi = 2
        wl = I.finalize_data(wl, O.template_fn(tdi=2), np.random.default_rng(90))
    f = np.array([w.sources[0, 0] for w in wl.windows])
    assert np.all(f > 20e-3) and np.any(f > 40e-3), f
    ctx = api.context_for(wl.T, tdi=tdi)
    ctx.set_orbit(pos, t0, dt)
    worst = check_logl_and_grad(O, ctx, wl, O.Geometry(wl.T, tdi=tdi))
    banner(f"  mixed gradient: worst error / natural scale {worst:.2e}")
    ctx.close()


def test_set_orbit_refuses_bad_grids():
    banner("numerical orbits: bad grids refused on the host")
    ctx = api.context_for(I.T1)
    pos, t0, dt = I.orbit_grid(lambda t: I.keplerian_orbits(t), I.T1, 65)
    for bad in ((pos[:3], t0, dt), (pos, t0, -dt), (pos, dt, dt), (pos[:40], t0, dt)):
        with pytest.raises(api.GbxError) as err:
            ctx.set_orbit(*bad)
        assert err.value.status == api.GB_EINVAL
    p2 = pos.copy()
    p2[5, 1] = p2[5, 0]
    with pytest.raises(api.GbxError):
        ctx.set_orbit(p2, t0, dt)
    p2 = pos.copy()
    p2[7, 2, 1] = np.nan
    with pytest.raises(api.GbxError):
        ctx.set_orbit(p2, t0, dt)
    ctx.close()
