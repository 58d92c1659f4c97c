"""Pins of the posterior-stage references in oracle/posterior.py (CPU).

* The finite-difference Fisher matrix (second-order forward differences, Sec. III G) agrees with
  the exact one from the oracle's dual-number derivatives: to 1e-6 of sqrt(F_ii F_jj) with steps
  of 1e-7 of the Table I widths, and to 1e-3 with the paper's 1e-9 (rounding of the templates
  amplified by the small step).
* The KDE log density: one kernel point is the bivariate normal log density (SciPy's); splitting
  a point's weight over copies of it changes nothing; the density integrates to one; pairs add.
"""

import math

import numpy as np
import pytest
from scipy import stats

from paper_2307_03763_amd import inputs as I


@pytest.fixture(scope="module")
def post(oracle_lib):
    from oracle import posterior
    return posterior


@pytest.mark.parametrize("case", ["c1", "c3_high"])
def test_fisher_fd_matches_exact(oracle_lib, post, case):
    O = oracle_lib
    if case == "c1":
        wl = I.workload_c1(O.template_fn(), n_cand=2)
        i = 0
    else:
        wl = I.workload_c3(O.template_fn(), n_win=256, n_cand=2)
        i = int(np.argmax([w.f_lo for w in wl.windows]))
    w = wl.windows[i]
    d, ww = wl.window_data(i)
    g = O.Geometry(wl.T)
    src = w.sources[0]
    Fx = post.fisher_u(src, w.k0, w.W, w.N, w.C, ww, g)
    sc = np.sqrt(np.outer(np.diag(Fx), np.diag(Fx)))
    width = wl.window_box(i).width
    F7 = post.fisher_fd(src, w.k0, w.W, w.N, w.C, ww, g, 1e-7 * width)
    F9 = post.fisher_fd(src, w.k0, w.W, w.N, w.C, ww, g, 1e-9 * width)
    assert np.max(np.abs(F7 - Fx) / sc) < 1e-6
    assert np.max(np.abs(F9 - Fx) / sc) < 1e-3
    # and the uncertainties that size the reduced box
    s7 = np.sqrt(np.diag(np.linalg.inv(F7)))
    sx = np.sqrt(np.diag(np.linalg.inv(Fx)))
    assert np.max(np.abs(s7 / sx - 1)) < 1e-5


def _chol(H):
    L = np.linalg.cholesky(H)
    return np.array([L[0, 0], L[1, 0], L[1, 1]])


def test_kde_single_point_is_gaussian(post):
    rng = np.random.default_rng(1)
    H = np.array([[2.0, 0.7], [0.7, 0.5]])
    y = np.array([0.3, -1.2])
    x = rng.normal(size=(50, 1, 2)) * 3
    got = post.kde_logpdf(y[None, None, :], np.ones((1, 1)), _chol(H)[None, :], x)
    ref = stats.multivariate_normal(mean=y, cov=H).logpdf(x[:, 0, :])
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_kde_weight_split_and_pairs(post):
    rng = np.random.default_rng(2)
    pts = rng.normal(size=(2, 40, 2))
    wts = rng.random((2, 40))
    wts /= wts.sum(axis=1, keepdims=True)
    ch = np.array([_chol(np.array([[0.3, 0.1], [0.1, 0.2]])), _chol(np.array([[1.0, -0.4], [-0.4, 0.8]]))])
    x = rng.normal(size=(30, 2, 2))
    base = post.kde_logpdf(pts, wts, ch, x)
    # split the weight of point 0 of each pair over three copies
    pts2 = np.concatenate([pts, pts[:, :1], pts[:, :1]], axis=1)
    wts2 = np.concatenate([wts, wts[:, :1] / 3, wts[:, :1] / 3], axis=1)
    wts2[:, 0] /= 3
    np.testing.assert_allclose(post.kde_logpdf(pts2, wts2, ch, x), base, rtol=1e-12, atol=1e-12)
    # pairs add
    one = post.kde_logpdf(pts[:1], wts[:1], ch[:1], x[:, :1]) + post.kde_logpdf(pts[1:], wts[1:], ch[1:], x[:, 1:])
    np.testing.assert_allclose(base, one, rtol=1e-12, atol=1e-12)


def test_kde_integrates_to_one(post):
    rng = np.random.default_rng(3)
    pts = rng.normal(size=(1, 25, 2)) * [1.0, 0.5]
    wts = rng.random((1, 25))
    wts /= wts.sum()
    ch = _chol(np.array([[0.09, 0.02], [0.02, 0.04]]))[None, :]
    gx = np.linspace(-6, 6, 401)
    gy = np.linspace(-4, 4, 321)
    X, Y = np.meshgrid(gx, gy, indexing="ij")
    q = np.stack([X.ravel(), Y.ravel()], axis=1)[:, None, :]
    dens = np.exp(post.kde_logpdf(pts, wts, ch, q)).reshape(X.shape)
    integral = np.trapezoid(np.trapezoid(dens, gy, axis=1), gx)
    assert abs(integral - 1.0) < 1e-6
