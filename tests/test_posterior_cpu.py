"""The annealed posterior driver (Algorithm 4, Sec. III G) on the CPU with the oracle as the
backend: six temperatures, the Fisher-reduced box, pairwise KDE proposals.  For the loud plain
window of a GB at 8 mHz (SNR ~ 60, fdot well inside its prior) the final (T = 1) chain must
look like the Gaussian the Fisher matrix predicts.  The paper keeps psi and phi0 in narrow boxes around the maximum-likelihood values
(their distributions are neglected), so the chain is conditional on them: the reference is the
inverse of the Fisher block of the other six parameters: means within 0.6 sigma of the
maximum-likelihood point, standard deviations within [0.7, 1.4] sigma, with the paper's 10,000
proposals per temperature.  (The first stage, uniform over a box whose fdot range is the whole
prior, accepts only tens of proposals; the KDE stages recover from that.)"""

import numpy as np
import pytest

from paper_2307_03763_amd import drivers as D
from paper_2307_03763_amd import inputs as I


class OracleBackend:
    def __init__(self, O, post, wl, i):
        self.O, self.post, self.wl, self.i = O, post, wl, i
        self.w = wl.windows[i]
        self.d, self.ww = wl.window_data(i)
        self.g = O.Geometry(wl.T)

    def fisher(self, theta, steps):
        w = self.w
        return np.stack([self.post.fisher_fd(t, w.k0, w.W, w.N, w.C, self.ww, self.g, s) for t, s in zip(theta, steps)])

    def mh(self, theta, log_g, u, T):
        w = self.w
        l, _ = self.O.loglik(theta, w.k0, w.W, w.N, w.C, self.d, self.ww, self.g)
        ch, acc = self.O.mh_chain(l, log_g, u, T)
        return l, ch, acc

    def kde_logpdf(self, pts, wts, chol, x):
        return self.post.kde_logpdf(pts, wts, chol, x)

    # for the polish
    def loglik(self, theta):
        w = self.w
        return self.O.loglik(theta, w.k0, w.W, w.N, w.C, self.d, self.ww, self.g)

    def loglik_grad(self, theta):
        w = self.w
        return self.O.loglik_grad(theta, w.k0, w.W, w.N, w.C, self.d, self.ww, self.g)


def _loud_window(O, f0=8e-3, rho=60.0, seed=3):
    """One T1 window at f0 with one GB (GR chirp of 0.8 Msun, well inside the fdot prior) of
    SNR ~ rho, plus PSD noise."""
    rng = np.random.default_rng(seed)
    T = I.T1
    q = int(np.floor(f0 * T))
    src = I.make_theta([f0 + 0.37 / T], float(I.fdot_gr(f0, 0.8)), 1e-22, I.random_angles(rng, 1))
    w = I.WindowSpec(k0=q - 128, W=256, N=256, C=I.channels_for(f0), f_lo=(q - 128) / T, f_hi=(q + 128) / T,
                     sources=src)
    wl = I._concat([w], [src], "loud test window", T)
    wl = I.finalize_data(wl, O.template_fn(), np.random.default_rng(seed + 1), noise=False)
    d, ww = wl.window_data(0)
    _, c = O.loglik(src, w.k0, w.W, w.N, w.C, d, ww, O.Geometry(T))
    src[0, 4] *= rho / np.sqrt(c[0, 1])
    w.sources = src
    wl = I._concat([w], [src], "loud test window", T)
    return I.finalize_data(wl, O.template_fn(), np.random.default_rng(seed + 1), noise=True)


def test_annealed_posterior_matches_fisher(oracle_lib):
    from oracle import posterior as post
    O = oracle_lib
    wl = _loud_window(O)
    be = OracleBackend(O, post, wl, 0)
    box = wl.window_box(0)
    src = wl.windows[0].sources[0]
    F0 = post.fisher_u(src, be.w.k0, be.w.W, be.w.N, be.w.C, be.ww, be.g)
    mle, _ = D.polish(be, src, np.sqrt(np.diag(np.linalg.inv(F0))), iterations=60)
    stages, (lo, hi), sigma = D.annealed_posterior(be, mle, box, np.random.default_rng(5), n=10000)
    assert [s["T"] for s in stages] == [15.0, 10.0, 5.0, 3.0, 2.0, 1.0]
    assert all(0 < s["n_accept"] < 10000 for s in stages)
    u_mle = I.to_table1(mle)
    assert np.all(u_mle >= lo) and np.all(u_mle <= hi)
    Fm = post.fisher_u(mle, be.w.k0, be.w.W, be.w.N, be.w.C, be.ww, be.g)
    s_cond = np.sqrt(np.diag(np.linalg.inv(Fm[:6, :6])))
    final = I.to_table1(stages[-1]["states"])
    for k in range(6):
        m, sd = final[:, k].mean(), final[:, k].std()
        assert abs(m - u_mle[k]) < 0.6 * s_cond[k], (k, m, u_mle[k], s_cond[k])
        assert 0.7 < sd / s_cond[k] < 1.4, (k, sd, s_cond[k])


def _loud_pair(O):
    """Two loud plain windows (8 mHz and 5 mHz, SNR ~ 60 each) in one workload."""
    a = _loud_window(O, 8e-3, 60.0, 3)
    b = _loud_window(O, 5e-3, 60.0, 8)
    wins = [a.windows[0], b.windows[0]]
    wl = I._concat(wins, [w.sources for w in wins], "two loud test windows", I.T1)
    return I.finalize_data(wl, O.template_fn(), np.random.default_rng(11), noise=True)


class OracleBatchBackend:
    """annealed_posterior_batch's calls with the oracle, one window per source (CPU tensors)."""

    def __init__(self, O, post, wl, rows):
        import torch
        self.torch = torch
        self.device = torch.device("cpu")
        self.one = [OracleBackend(O, post, wl, int(i)) for i in rows]
        self.O = O

    def fisher(self, theta, steps):
        return np.concatenate([b.fisher(t[None], s[None]) for b, t, s in zip(self.one, theta, steps)])

    def mh(self, theta, log_g, u, T):
        S = len(self.one)
        n = len(theta) // S
        th, lg, uu = theta.numpy(), log_g.numpy(), u.numpy()
        ls, cs, acc = [], [], []
        for k, b in enumerate(self.one):
            sl = slice(k * n, (k + 1) * n)
            l, ch, na = b.mh(th[sl], lg[sl], uu[sl], T)
            ls.append(l)
            cs.append(ch)
            acc.append(na)
        t = self.torch
        return t.as_tensor(np.concatenate(ls)), t.as_tensor(np.concatenate(cs).astype(np.int32)), t.as_tensor(acc)

    def kde_logpdf(self, pts, wts, chol, x):
        return self.torch.as_tensor(np.stack([self.one[0].kde_logpdf(p.numpy(), w.numpy(), c.numpy(), xx.numpy())
                                              for p, w, c, xx in zip(pts, wts, chol, x)]))


def pair_mles(O, post, wl):
    mles = []
    for i in range(wl.n_win):
        be = OracleBackend(O, post, wl, i)
        src = wl.windows[i].sources[0]
        F0 = post.fisher_u(src, be.w.k0, be.w.W, be.w.N, be.w.C, be.ww, be.g)
        mle, _ = D.polish(be, src, np.sqrt(np.diag(np.linalg.inv(F0))), iterations=60)
        mles.append(mle)
    return np.array(mles)


def check_against_fisher(O, post, wl, mles, stages):
    for i in range(wl.n_win):
        be = OracleBackend(O, post, wl, i)
        Fm = post.fisher_u(mles[i], be.w.k0, be.w.W, be.w.N, be.w.C, be.ww, be.g)
        s_cond = np.sqrt(np.diag(np.linalg.inv(Fm[:6, :6])))
        u_mle = I.to_table1(mles[i])
        final = I.to_table1(np.asarray(stages[-1]["states"][i]))
        for k in range(6):
            m, sd = final[:, k].mean(), final[:, k].std()
            assert abs(m - u_mle[k]) < 0.6 * s_cond[k], (i, k, m, u_mle[k], s_cond[k])
            assert 0.7 < sd / s_cond[k] < 1.4, (i, k, sd, s_cond[k])


def test_annealed_posterior_batch_matches_fisher(oracle_lib):
    """Algorithm 5's batched form: two sources in two windows through one call of the batched
    annealing (draws on torch tensors, one chain per source); each final chain against its own
    Fisher Gaussian as above (a mix-up between the sources would put a chain far off)."""
    from oracle import posterior as post
    O = oracle_lib
    wl = _loud_pair(O)
    mles = pair_mles(O, post, wl)
    be = OracleBatchBackend(O, post, wl, [0, 1])
    boxes = [wl.window_box(i) for i in range(2)]
    stages, (lo, hi), sigma = D.annealed_posterior_batch(be, mles, boxes, seed=5, n=10000)
    assert [s["T"] for s in stages] == [15.0, 10.0, 5.0, 3.0, 2.0, 1.0]
    assert all(np.all((np.asarray(s["n_accept"]) > 0) & (np.asarray(s["n_accept"]) < 10000)) for s in stages)
    u = I.to_table1(mles)
    assert np.all(u >= lo) and np.all(u <= hi)
    check_against_fisher(O, post, wl, mles, stages)
