"""The posterior stage's helpers on the GPU against the oracle references, and the whole annealed
posterior (Algorithm 4) driven by the library.

* gb_fisher: 24 sources of a ragged batch (several (N, C) groups in one call), second-order
  forward differences; against the oracle's finite differences with the same steps and against
  the exact (dual-number) Fisher matrix, at the paper's step (1e-9 of the Table I widths,
  rounding-limited on both sides) and at 1e-7; and the sigmas that size the reduced box.
* gb_kde_logpdf: three pairs, ragged tile sizes, zero weights, single kernel point; several
  independent sets in one launch; against the definition.
* annealed_posterior with the GPU backend on a loud 8 mHz source: the final chain against the
  Fisher Gaussian (conditional on psi, phi0), as the CPU test does with the oracle backend; every
  stage's chain bit-exact against the oracle's chain on the GPU's own logL and log g.
* annealed_posterior_batch (two sources in two windows, one launch per stage): the same checks
  for each source.
"""

import numpy as np
import pytest
import torch

from paper_2307_03763_amd import api
from paper_2307_03763_amd import drivers as D
from paper_2307_03763_amd import inputs as I
from tests.gpu_common import banner, dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def post(oracle_lib):
    from oracle import posterior
    return posterior


def test_fisher_matches_oracle(oracle_lib, post):
    banner("gb_fisher: 24 sources, ragged (N, C)")
    O = oracle_lib
    wl = I.workload_c3(O.template_fn(), n_win=24, n_cand=2)
    ctx = api.context_for(wl.T)
    g = O.Geometry(wl.T)
    th = np.stack([w.sources[0] for w in wl.windows])
    widths = np.stack([wl.window_box(i).width for i in range(wl.n_win)])
    w_t = dev(wl.weights)
    # The paper's step (1e-9 of the widths) is dominated by template rounding on both sides
    # (the oracle's own differences reach 7e-4 of sqrt(F_ii F_jj) and 4e-3 in sigma on these
    # sources).  That rounding term scales as 1 / step, so at 1e-7 each side carries ~7e-6 and
    # two independent roundings differ by up to ~2e-5 on the worst of 24 sources (bar 3e-5),
    # while both sit near the exact matrix.
    for fac, bar_fd, bar_exact, bar_sigma in ((1e-9, 1e-2, 1e-2, 2e-2), (1e-7, 3e-5, 1e-4, 1e-4)):
        steps = fac * widths
        F = api.gb_fisher(ctx.handle, dev(th), dev(steps), wl.window_table(), w_t).cpu().numpy()
        worst_fd = worst_ex = worst_s = 0.0
        for i, w in enumerate(wl.windows):
            _, ww = wl.window_data(i)
            Ffd = post.fisher_fd(th[i], w.k0, w.W, w.N, w.C, ww, g, steps[i])
            Fex = post.fisher_u(th[i], w.k0, w.W, w.N, w.C, ww, g)
            sc = np.sqrt(np.outer(np.diag(Fex), np.diag(Fex)))
            worst_fd = max(worst_fd, float(np.max(np.abs(F[i] - Ffd) / sc)))
            worst_ex = max(worst_ex, float(np.max(np.abs(F[i] - Fex) / sc)))
            s_g = np.sqrt(np.diag(np.linalg.inv(F[i])))
            s_x = np.sqrt(np.diag(np.linalg.inv(Fex)))
            worst_s = max(worst_s, float(np.max(np.abs(s_g / s_x - 1))))
        banner(f"  steps {fac:g} x widths: vs oracle FD {worst_fd:.1e}, vs exact {worst_ex:.1e}, sigma {worst_s:.1e}")
        assert worst_fd <= bar_fd and worst_ex <= bar_exact and worst_s <= bar_sigma


@pytest.mark.parametrize("m,q", [(1, 7), (255, 300), (3001, 5000)])
def test_kde_logpdf_matches_oracle(post, m, q):
    banner(f"gb_kde_logpdf: 3 pairs, m={m}, q={q}")
    rng = np.random.default_rng(m + q)
    pts = rng.normal(size=(3, m, 2)) * [[1.0, 0.3]]
    wts = rng.random((3, m))
    if m > 10:
        wts[:, ::7] = 0.0
    wts /= wts.sum(axis=1, keepdims=True)
    chol = np.array([[0.2, 0.05, 0.1], [0.5, -0.2, 0.3], [0.05, 0.01, 0.02]])
    x = rng.normal(size=(q, 3, 2)) * 1.5
    got = api.gb_kde_logpdf(dev(pts), dev(wts), dev(chol), dev(x)).cpu().numpy()
    ref = post.kde_logpdf(pts, wts, chol, x)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-9)


def test_annealed_posterior_gpu(oracle_lib, post):
    banner("annealed posterior (6 temperatures x 10,000) on the GPU, loud 8 mHz source")
    from tests.test_posterior_cpu import OracleBackend, _loud_window
    O = oracle_lib
    wl = _loud_window(O)
    ctx = api.context_for(wl.T)
    row = wl.window_table()[0]
    be = D.GpuPosteriorBackend(ctx, row, dev(wl.data, torch.complex128), dev(wl.weights))
    ob = OracleBackend(O, post, wl, 0)
    box = wl.window_box(0)
    src = wl.windows[0].sources[0]
    F0 = post.fisher_u(src, ob.w.k0, ob.w.W, ob.w.N, ob.w.C, ob.ww, ob.g)
    mle, _ = D.polish(ob, src, np.sqrt(np.diag(np.linalg.inv(F0))), iterations=60)

    # every stage's chain against the oracle's chain on the GPU's own values
    class Checked:
        def fisher(self, t, s):
            return be.fisher(t, s)

        def kde_logpdf(self, p, w, c, x):
            return be.kde_logpdf(p, w, c, x)

        def mh(self, theta, log_g, u, T):
            l, ch, na = be.mh(theta, log_g, u, T)
            ref, acc = O.mh_chain(l, log_g, u, T)
            assert np.array_equal(ch, ref) and na == acc
            return l, ch, na

    stages, (lo, hi), sigma = D.annealed_posterior(Checked(), mle, box, np.random.default_rng(5), n=10000)
    Fm = post.fisher_u(mle, ob.w.k0, ob.w.W, ob.w.N, ob.w.C, ob.ww, ob.g)
    s_cond = np.sqrt(np.diag(np.linalg.inv(Fm[:6, :6])))
    u_mle = I.to_table1(mle)
    final = I.to_table1(stages[-1]["states"])
    banner(f"  accepted per stage {[s['n_accept'] for s in stages]}; std / sigma "
           f"{np.round(final[:, :6].std(axis=0) / s_cond, 2)}")
    for k in range(6):
        assert abs(final[:, k].mean() - u_mle[k]) < 0.6 * s_cond[k]
        assert 0.7 < final[:, k].std() / s_cond[k] < 1.4


def test_kde_logpdf_sets_match_oracle(post):
    banner("gb_kde_logpdf: 5 independent sets in one launch, zero-weight padding")
    rng = np.random.default_rng(17)
    S, P, m, q = 5, 3, 300, 700
    pts = rng.normal(size=(S, P, m, 2))
    wts = rng.random((S, P, m))
    for s in range(S):
        wts[s, :, m - 37 * s:] = 0.0        # set s holds m - 37 s points
    wts /= wts.sum(axis=2, keepdims=True)
    chol = np.abs(rng.normal(size=(S, P, 3))) * 0.3 + 0.05
    chol[:, :, 1] -= 0.1
    x = rng.normal(size=(S, q, P, 2))
    got = api.gb_kde_logpdf(dev(pts), dev(wts), dev(chol), dev(x)).cpu().numpy()
    assert got.shape == (S, q)
    for s in range(S):
        np.testing.assert_allclose(got[s], post.kde_logpdf(pts[s], wts[s], chol[s], x[s]), rtol=1e-12, atol=1e-9)


def test_annealed_posterior_batch_gpu(oracle_lib, post):
    banner("batched annealed posterior: two sources, six temperatures x 10,000, one launch per stage")
    from tests.test_posterior_cpu import _loud_pair, check_against_fisher, pair_mles
    O = oracle_lib
    wl = _loud_pair(O)
    mles = pair_mles(O, post, wl)
    ctx = api.context_for(wl.T)
    table = wl.window_table()
    d = dev(wl.data, torch.complex128)
    d_res = api.gb_add_templates(ctx.handle, table, dev(mles), np.arange(2, dtype=np.int32), -1.0, d)
    be = D.GpuPosteriorBatchBackend(ctx, table, d_res, dev(wl.weights), mles, [0, 1])
    # d_residual + own template gives back each window's data
    assert torch.max(torch.abs(be.d - d)).item() <= 1e-12 * torch.max(torch.abs(d)).item()

    class Checked:
        device = be.device

        def fisher(self, t, s):
            return be.fisher(t, s)

        def kde_logpdf(self, p, w, c, x):
            return be.kde_logpdf(p, w, c, x)

        def mh(self, theta, log_g, u, T):
            l, ch, na = be.mh(theta, log_g, u, T)
            n = len(theta) // 2
            lh, gh, uh, chh = l.cpu().numpy(), log_g.cpu().numpy(), u.cpu().numpy(), ch.cpu().numpy()
            for k in range(2):
                sl = slice(k * n, (k + 1) * n)
                ref, acc = O.mh_chain(lh[sl], gh[sl], uh[sl], T)
                assert np.array_equal(chh[sl], ref) and int(na[k]) == acc
            return l, ch, na

    stages, _, _ = D.annealed_posterior_batch(Checked(), mles, [wl.window_box(i) for i in range(2)], seed=5, n=10000)
    banner(f"  accepted per stage {[s['n_accept'].tolist() for s in stages]}")
    check_against_fisher(O, post, wl, mles, [{"states": s["states"].cpu().numpy()} for s in stages])
    be.close()
