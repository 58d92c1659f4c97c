"""Search / polish drivers on the CPU, scored by the oracle (the drivers only take decisions;
the likelihood comes from whatever backend they are given).

Pins:
* the injected source of the plain 3 mHz window (C1) is found by the DE search from a random
  population over the Table I box (Algorithm 2 / Sec. III D);
* the amplitude DE returns is the analytic maximiser A_max (Sec. III amplitude equation:
  d logL / dA = 0 there);
* the quasi-Newton polish ends at a stationary point of logL (gradient ~ 0 in Fisher units) at
  least as good as the injection, from the injection and from a 3-sigma perturbed start;
* batching bookkeeping: several windows searched together (DE, then polish) each end near
  their own loudest source, and polishing starts jointly gives exactly what polishing each
  alone gives."""

import numpy as np
import pytest

from paper_2307_03763_amd import drivers as D
from paper_2307_03763_amd import inputs as I


class OracleBackend:
    """Window-major batched evaluation with the oracle (rows i*n .. i*n+n-1 -> window i)."""

    def __init__(self, O, wl, windows):
        self.O, self.wl, self.windows = O, wl, list(windows)
        self.g = O.Geometry(wl.T)

    def _each(self, fn, theta):
        n = len(theta) // len(self.windows)
        outs = []
        for j, i in enumerate(self.windows):
            w = self.wl.windows[i]
            d, ww = self.wl.window_data(i)
            outs.append(fn(theta[j * n:(j + 1) * n], w.k0, w.W, w.N, w.C, d, ww, self.g))
        return np.concatenate([o[0] for o in outs]), np.concatenate([o[1] for o in outs])

    def loglik(self, theta):
        return self._each(self.O.loglik, theta)

    def loglik_grad(self, theta):
        return self._each(self.O.loglik_grad, theta)


def fisher_sigma_u(O, wl, i, theta):
    w = wl.windows[i]
    _, ww = wl.window_data(i)
    F = O.fisher(theta, w.k0, w.W, w.N, w.C, ww, O.Geometry(wl.T))
    J = D._table1_jacobian(theta)
    return np.sqrt(np.diag(np.linalg.inv(F * np.outer(J, J))))


@pytest.fixture(scope="module")
def c1(oracle_lib):
    O = oracle_lib
    wl = I.workload_c1(O.template_fn(), n_cand=4)
    src = wl.windows[0].sources[0]
    return O, wl, OracleBackend(O, wl, [0]), wl.window_box(0), src, fisher_sigma_u(O, wl, 0, src)


def _rho(be, th):
    _, c = be.loglik(np.atleast_2d(th))
    return c[:, 0] / np.sqrt(c[:, 1])


def test_de_search_finds_injection(c1):
    O, wl, be, box, src, _ = c1
    rho_inj = _rho(be, src)[0]
    th, rho, hist = D.de_search(be, box, np.random.default_rng(5), pop=512, generations=200, keep=4)
    assert th.shape == (1, 4, 8) and rho.shape == (1, 4) and hist.shape == (201, 1)
    assert np.all(np.diff(hist[:, 0]) >= 0.0), "elitist selection: the best SNR never decreases"
    assert np.all(np.diff(rho[0]) <= 0.0), "kept members come best first"
    assert rho[0, 0] > 0.9 * rho_inj, (rho, rho_inj)
    u = I.to_table1(th[0, 0])
    dims = list(D.SEARCH_DIMS)
    assert np.all(u[dims] >= box.lo[dims] - 1e-12) and np.all(u[dims] <= box.hi[dims] + 1e-12)
    assert abs(th[0, 0, 0] - src[0]) * wl.T < 1.0          # frequency within a bin
    # A = A_max: d logL / dA = <d|h_1> - A <h_1|h_1> vanishes, and rho is what the components give
    _, gr = be.loglik_grad(th[0])
    _, c = be.loglik(th[0])
    assert np.all(np.abs(gr[:, 4] * th[0, :, 4]) < 1e-9 * c[:, 1])
    np.testing.assert_allclose(rho[0], c[:, 0] / np.sqrt(c[:, 1]), rtol=1e-12)


def test_de_seeded_with_truth_keeps_it(c1):
    _, _, be, box, src, _ = c1
    _, rho, _ = D.de_search(be, box, np.random.default_rng(1), pop=64, generations=5, init=src)
    assert rho[0, 0] >= _rho(be, src)[0] * (1 - 1e-12)


@pytest.mark.parametrize("start", ["injection", "perturbed"])
def test_polish_reaches_stationary_point(c1, start):
    _, _, be, _, src, sig = c1
    th0 = src if start == "injection" else I.from_table1(
        I.to_table1(src) + 3 * sig * np.random.default_rng(1).standard_normal(8))
    th, hist = D.polish(be, th0, sig, iterations=60)
    assert th.shape == (8,) and hist.shape == (61,)
    assert np.all(np.diff(hist) >= 0.0)
    l_inj, _ = be.loglik(src[None, :])
    assert hist[-1] >= l_inj[0]
    _, g = be.loglik_grad(th[None, :])
    gu = g[0] * D._table1_jacobian(th) * sig       # gradient in Fisher-sigma units
    assert np.max(np.abs(gu)) < 1e-2, gu
    _, h_ref = D.polish(be, src, sig, iterations=60)
    assert hist[-1] == pytest.approx(h_ref[-1], abs=1e-6)


@pytest.fixture(scope="module")
def c4_two(oracle_lib):
    O = oracle_lib
    wl = I.workload_c4(O.template_fn(), n_win=2, n_cand=4)
    return O, wl


def test_search_batched_windows_find_their_sources(c4_two):
    """DE + polish of its 8 best members on two windows at once (W = 1024 and 512 bins, the
    full Table I box each): each window ends near its loudest source."""
    O, wl = c4_two
    be = OracleBackend(O, wl, [0, 1])
    boxes = [wl.window_box(0), wl.window_box(1)]
    th, l = D.search(be, boxes, np.random.default_rng(7), pop=256, generations=120, keep=8,
                     polish_iterations=40)
    assert th.shape == (2, 8) and l.shape == (2,)
    for i in range(2):
        one = OracleBackend(O, wl, [i])
        r_src = _rho(one, wl.windows[i].sources)
        assert r_src.max() > 10                      # loud enough to be found
        l_one, _ = one.loglik(th[i][None, :])
        assert l[i] == pytest.approx(l_one[0], rel=1e-12)
        assert _rho(one, th[i])[0] > 0.8 * r_src.max(), (i, _rho(one, th[i]), r_src)
        f_bins = np.abs(th[i, 0] - wl.windows[i].sources[:, 0]) * wl.T
        assert f_bins.min() < 5.0


def test_polish_batched_equals_separate(c4_two):
    O, wl = c4_two
    be2 = OracleBackend(O, wl, [0, 1])
    starts, sig = [], []
    rng = np.random.default_rng(3)
    for i in range(2):
        s = wl.windows[i].sources[0]
        su = fisher_sigma_u(O, wl, i, s)
        sig.append(su)
        starts.append(I.from_table1(I.to_table1(s) + 2 * su * rng.standard_normal((3, 8))))
    starts = np.stack(starts)                        # [2 windows, 3 starts, 8]
    sig = np.stack(sig)[:, None, :]
    th_b, h_b = D.polish(be2, starts, sig, iterations=15)
    assert th_b.shape == (2, 3, 8) and h_b.shape == (16, 2, 3)
    for i in range(2):
        th_s, h_s = D.polish(OracleBackend(O, wl, [i]), starts[i], sig[i], iterations=15)
        np.testing.assert_array_equal(th_b[i], th_s)
        np.testing.assert_array_equal(h_b[:, i], h_s)


def test_de_convergence_stop(c1):
    """SciPy's stopping rule (std(rho) <= tol |mean(rho)|): the window stops early, keeps its
    best member (the injection, within a bin) and its history stays flat afterwards."""
    O, wl, be, box, src, _ = c1
    th, rho, hist = D.de_search(be, box, np.random.default_rng(2), pop=64, generations=400, tol=0.01,
                                check_every=10)
    assert hist.shape == (401, 1) and np.all(np.diff(hist[:, 0]) >= 0)
    assert hist[-1, 0] == hist[-150, 0]            # stopped well before the last generation
    assert abs(th[0, 0, 0] - src[0]) * wl.T < 1.0


def test_destruction_inside_a_capture_is_deferred(monkeypatch):
    """Plans and contexts destroyed while a graph capture is open (as the cyclic collector may do
    at any allocation inside the captured body) queue their device frees until the outermost
    capture closes; outside a capture they free at once.  Checked with a stand-in library that
    records the calls."""
    import ctypes
    import gc

    from paper_2307_03763_amd import api

    calls = []

    class Stub:
        def gb_create(self, cfg, out):
            out._obj.value = 0x1000
            return 0

        def gb_plan_create(self, ctx, wins, n, prec, out):
            out._obj.value = 0x2000 + len(calls)
            return 0

        def gb_plan_destroy(self, h):
            calls.append(("plan", h))

        def gb_destroy(self, h):
            calls.append(("ctx", h))

    monkeypatch.setattr(api, "lib", lambda: Stub())
    table = [[1000, 64, 64, 2, 0, 0, 0, 4]]
    ctx = api.Context(1.0, 1.0, 1.0, 1.0)
    p0 = api.Plan(ctx, table, api.GB_MIXED)
    del p0
    gc.collect()
    assert calls == [("plan", 0x2000)]                 # no capture: freed at once
    p1 = api.Plan(ctx, table, api.GB_MIXED)
    with api.capturing():
        with api.capturing():                          # nested captures
            p2 = api.Plan(ctx, table, api.GB_MIXED)
            del p1, p2
            gc.collect()
            ctx.close()
        assert calls == [("plan", 0x2000)]             # still inside the outer capture
    assert sorted(c[0] for c in calls[1:]) == ["ctx", "plan", "plan"]
    assert api._deferred == [] and api._capture_depth == 0
    from paper_2307_03763_amd import drivers as D
    assert D.CAPTURE_MODE == "global"
