"""Search / polish / posterior drivers on the GPU, checked against the oracle.

The DE search and the polish take decisions from GPU likelihoods; with FP64 scoring the DE run
takes the same decisions as the same run scored by the oracle (the values agree to ~1e-13, far
below any gap between competing members), so the two end at the same members.  Every value the
drivers report is recomputed by the oracle.  The posterior stage (Algorithm 4, one temperature)
runs eagerly and as a replayed HIP graph; each replay's logL and chain are compared with the
oracle on the proposals that replay drew."""

import numpy as np
import pytest

from tests.gpu_common import banner, loglik_tolerance
from tests.test_drivers_cpu import OracleBackend, fisher_sigma_u

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu_backend(api, D, wl, windows, prec_l, prec_g=None):
    ctx = api.context_for(wl.T)
    tab = wl.window_table()[list(windows)].copy()
    blocks_d, blocks_w, off = [], [], 0
    for j, i in enumerate(windows):
        d, ww = wl.window_data(i)
        tab[j, 4] = tab[j, 5] = off
        blocks_d.append(d.ravel())
        blocks_w.append(ww.ravel())
        off += d.size
    d_t = torch.as_tensor(np.concatenate(blocks_d), device="cuda")
    w_t = torch.as_tensor(np.concatenate(blocks_w), device="cuda")
    return D.GpuBackend(ctx, tab, d_t, w_t, prec_l, prec_g), ctx, d_t, w_t, tab


@pytest.fixture(scope="module")
def env(oracle_lib):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_03763_amd import api, drivers as D, inputs as I
    O = oracle_lib
    c1 = I.workload_c1(O.template_fn(), n_cand=4)
    c4 = I.workload_c4(O.template_fn(), n_win=2, n_cand=4)
    return dict(api=api, D=D, I=I, O=O, c1=c1, c4=c4)


def test_de_search_gpu_follows_oracle(env):
    banner("drivers: DE search on two C4 windows, FP64 scoring, GPU vs oracle-driven (host generations)")
    api, D, O, wl = env["api"], env["D"], env["O"], env["c4"]
    be, *_ = _gpu_backend(api, D, wl, [0, 1], api.GB_FP64)
    boxes = [wl.window_box(0), wl.window_box(1)]
    th_g, rho_g, hist_g = D.de_search(be, boxes, np.random.default_rng(7), pop=256, generations=40, keep=4,
                                      on_device=False)
    th_o, rho_o, hist_o = D.de_search(OracleBackend(O, wl, [0, 1]), boxes, np.random.default_rng(7),
                                      pop=256, generations=40, keep=4)
    np.testing.assert_allclose(hist_g, hist_o, rtol=1e-10)
    np.testing.assert_allclose(rho_g, rho_o, rtol=1e-10)
    np.testing.assert_allclose(th_g, th_o, rtol=1e-9)
    be.close()


def test_search_gpu_finds_sources(env):
    banner("drivers: DE + polish on two C4 windows, FP64 logL, mixed gradient")
    api, D, O, wl = env["api"], env["D"], env["O"], env["c4"]
    be, *_ = _gpu_backend(api, D, wl, [0, 1], api.GB_FP64, api.GB_MIXED)
    boxes = [wl.window_box(0), wl.window_box(1)]
    # window 0 holds one weak source (SNR 18) in a wide box: DE with 256 members reaches SNR
    # 6-11 after 120 generations and 14-16 after 600 (host and device generations alike), so
    # the search runs 400 generations and the paper's three restarts
    th, l = D.search(be, boxes, np.random.default_rng(7), pop=256, generations=400, keep=8,
                     polish_iterations=40, n_searches=3)
    for i in range(2):
        one = OracleBackend(O, wl, [i])
        l_or, c_or = one.loglik(th[i][None, :])
        d, ww = wl.window_data(i)
        dd = float(np.sum(ww * np.abs(d) ** 2))
        assert abs(l[i] - l_or[0]) <= loglik_tolerance(dd, c_or[0, 0], c_or[0, 1])
        _, c_src = one.loglik(wl.windows[i].sources)
        rho_src = c_src[:, 0] / np.sqrt(c_src[:, 1])
        assert c_or[0, 0] / np.sqrt(c_or[0, 1]) > 0.8 * rho_src.max()
    be.close()


def test_polish_gpu_mixed_gradient(env):
    banner("drivers: BFGS polish on C1, FP64 logL + mixed gradient")
    api, D, I, O, wl = env["api"], env["D"], env["I"], env["O"], env["c1"]
    be, *_ = _gpu_backend(api, D, wl, [0], api.GB_FP64, api.GB_MIXED)
    src = wl.windows[0].sources[0]
    sig = fisher_sigma_u(O, wl, 0, src)
    th0 = I.from_table1(I.to_table1(src) + 3 * sig * np.random.default_rng(1).standard_normal(8))
    th, hist = D.polish(be, th0, sig, iterations=60)
    one = OracleBackend(O, wl, [0])
    l_end, _ = one.loglik(th[None, :])
    assert hist[-1] == pytest.approx(l_end[0], rel=1e-10)
    _, h_ref = D.polish(one, src, sig, iterations=60)
    # the maximum is reached up to what the mixed gradient resolves (logL is flat there)
    assert l_end[0] == pytest.approx(h_ref[-1], abs=1e-4)
    be.close()


@pytest.mark.parametrize("graph", [False, True])
def test_posterior_stage(env, graph):
    """One MH stage (draw, gb_mh_step, chain) eager and captured in a HIP graph in global capture
    mode, where any unsafe call during the capture fails it."""
    banner(f"drivers: posterior stage on C1, graph={graph}")
    api, D, I, O, wl = env["api"], env["D"], env["I"], env["O"], env["c1"]
    assert D.CAPTURE_MODE == "global"
    n = 4096
    _, ctx, d_t, w_t, tab = _gpu_backend(api, D, wl, [0], api.GB_FP64)
    row = tab[0].copy()
    row[6], row[7] = 0, n
    plan = api.Plan(ctx, row[None, :], api.GB_FP64)
    plan.prepare(d_t, w_t)
    src = wl.windows[0].sources[0]
    lo, hi = I.reduced_box(src, wl.window_box(0), fisher_sigma_u(O, wl, 0, src))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1234)
    temp = 2.0
    st = D.PosteriorStage(plan, lo, hi, temp, gen)
    if graph:
        st.capture()
    one = OracleBackend(O, wl, [0])
    d, ww = wl.window_data(0)
    dd = float(np.sum(ww * np.abs(d) ** 2))
    prev = None
    for _ in range(3):
        if graph:
            st.replay()
        else:
            st.run()
        torch.cuda.synchronize()
        th = st.theta.cpu().numpy()
        u = st.u.cpu().numpy()
        l = st.logL.cpu().numpy()
        uu = I.to_table1(th)
        assert np.all(uu >= lo - 1e-12) and np.all(uu <= hi + 1e-12)
        l_ref, c_ref = one.loglik(th)
        tol = loglik_tolerance(dd, c_ref[:, 0], c_ref[:, 1])
        assert np.all(np.abs(l - l_ref) <= tol), np.max(np.abs(l - l_ref) / tol)
        chain_ref, acc_ref = O.mh_chain(l, np.zeros(n), u, temp)
        np.testing.assert_array_equal(st.chain.cpu().numpy(), chain_ref)
        assert int(st.n_accept.cpu()[0]) == acc_ref
        if prev is not None:
            assert not np.array_equal(prev, th), "each replay draws new proposals"
        prev = th
    plan.close()


def test_tune_on_windows_then_search(env):
    """tune_on_windows tunes the families of the windows it is given (two C4 windows: one (N, C)),
    on per_window candidates each; a DE search on the tuned context still takes the oracle-driven
    run's decisions."""
    banner("drivers: launch shapes tuned on two C4 windows, then the DE search of the first test")
    api, D, O, wl = env["api"], env["D"], env["O"], env["c4"]
    be, ctx, d_t, w_t, tab = _gpu_backend(api, D, wl, [0, 1], api.GB_FP64)
    boxes = [wl.window_box(0), wl.window_box(1)]
    be.close()
    rep = D.tune_on_windows(ctx, tab, d_t, w_t, boxes, per_window=300, rng=np.random.default_rng(1))
    fam = {(int(tab[i, 2]), int(tab[i, 3])) for i in range(2)}
    heads = sorted(l.split(":", 1)[0] for l in rep.splitlines() if l.strip())
    want = sorted(f"{p} N={N} C={C}" for N, C in fam for p in ("fp64  loglik", "mixed loglik", "mixed grad  "))
    assert heads == want, (heads, want)
    assert all("/ 600 (" in l for l in rep.splitlines() if l.strip()), rep
    be = D.GpuBackend(ctx, tab, d_t, w_t, api.GB_FP64)
    th_g, rho_g, hist_g = D.de_search(be, boxes, np.random.default_rng(7), pop=256, generations=40, keep=4,
                                      on_device=False)
    th_o, rho_o, hist_o = D.de_search(OracleBackend(O, wl, [0, 1]), boxes, np.random.default_rng(7),
                                      pop=256, generations=40, keep=4)
    np.testing.assert_allclose(hist_g, hist_o, rtol=1e-10)
    np.testing.assert_allclose(th_g, th_o, rtol=1e-9)
    be.close()
