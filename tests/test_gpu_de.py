"""The differential-evolution step on the GPU (gb_de_trial, gb_de_select) against oracle/de.py on
the same uniforms: trial coordinates and the selection bit-exact (the step's arithmetic is
plain sums, products, an exact remainder and comparisons, rounded the same way on both sides),
the trial parameters to the last bits of arcsin/arccos.  Populations of 4 (the smallest), a
ragged 37 and 512 with 64 windows; mutants far outside the boxes; scores with NaN and inf.
Then ten generations in a row on the likelihood of real windows (the GPU's components feed both
sides), and the device-resident search finding the sources of the C1-like windows."""

import numpy as np
import pytest
import torch

from paper_2307_03763_amd import api
from paper_2307_03763_amd import drivers as D
from paper_2307_03763_amd import inputs as I
from tests.gpu_common import banner, dev

pytestmark = pytest.mark.gpu


def _boxes(rng, n_win):
    lo = np.stack([rng.uniform(1e-3, 5e-3, n_win), rng.uniform(-1e-16, 0, n_win), np.full(n_win, -1.0),
                   np.zeros(n_win), np.full(n_win, -1.0), np.zeros(n_win), np.zeros(n_win)], axis=1)
    hi = lo + np.stack([np.full(n_win, 1e-6), np.full(n_win, 2e-16), np.full(n_win, 2.0), np.full(n_win, 2 * np.pi),
                        np.full(n_win, 2.0), np.full(n_win, np.pi), np.full(n_win, 2 * np.pi)], axis=1)
    return lo, hi


@pytest.mark.parametrize("n_win,pop,best1", [(3, 4, False), (5, 37, False), (64, 512, False), (3, 4, True),
                                             (64, 512, True)])
def test_de_step_matches_oracle(n_win, pop, best1):
    from oracle import de
    banner(f"gb_de_trial / gb_de_select: {n_win} windows x {pop} members, {'best' if best1 else 'rand'}/1")
    rng = np.random.default_rng(n_win * 1000 + pop)
    lo, hi = _boxes(rng, n_win)
    x = lo[:, None, :] + (hi - lo)[:, None, :] * rng.random((n_win, pop, 7))
    x[:, 0, :] = lo                                  # members on the walls
    x[:, -1, :] = hi
    u_idx = rng.random((n_win, pop, 3))
    u_idx[:, 0, :] = 0.0
    u_idx[:, 1, :] = np.nextafter(1.0, 0.0)
    u_cross, u_j = rng.random((n_win, pop, 7)), rng.random((n_win, pop))
    F = rng.uniform(0.5, 2.5, n_win)                 # large steps: many mutants outside the box
    base = rng.integers(0, pop, n_win).astype(np.int32) if best1 else None
    tx, th = api.gb_de_trial(dev(lo), dev(hi), dev(x), dev(u_idx), dev(u_cross), dev(u_j), dev(F), 0.7, 1e-22,
                             base=None if base is None else torch.as_tensor(base, device="cuda"))
    rx, rth = de.trial(lo, hi, x, u_idx, u_cross, u_j, F, 0.7, 1e-22, base=base)
    tx, th = tx.cpu().numpy(), th.cpu().numpy()
    assert np.array_equal(tx, rx)
    plain = [0, 1, 3, 4, 6, 7]
    assert np.array_equal(th[:, plain], rth[:, plain])
    # arcsin / arccos of the same argument: two libraries, each within about an ulp of the
    # result (results up to pi: 4.4e-16 per ulp)
    err = float(np.max(np.abs(th[:, [2, 5]] - rth[:, [2, 5]])))
    banner(f"  arcsin/arccos: largest difference {err:.2e}")
    assert err <= 2e-15, err
    # selection with awkward scores
    comps = np.stack([rng.normal(size=n_win * pop), rng.uniform(0.5, 2.0, n_win * pop)], axis=1)
    comps[::7, 0] = np.nan
    comps[::11, 1] = 0.0
    comps[::13, 1] = -1.0
    s = rng.normal(size=(n_win, pop))
    s[:, ::5] = -np.inf
    s[0, :] = 5.0                                    # a window of ties
    xg, sg = dev(x), dev(s)
    bi = torch.empty(n_win, dtype=torch.int32, device="cuda")
    best = api.gb_de_select(dev(comps), xg, sg, dev(tx), best_idx=bi).cpu().numpy()
    rx2, rs2, rbest, rbi = de.select(comps, x, s, tx)
    assert np.array_equal(xg.cpu().numpy(), rx2) and np.array_equal(sg.cpu().numpy(), rs2)
    assert np.array_equal(best, rbest) and np.array_equal(bi.cpu().numpy(), rbi)


def test_de_generations_on_likelihood(oracle_lib):
    from oracle import de
    banner("ten DE generations (rand/1 and best/1 in turn) on four ragged windows, GPU vs oracle step")
    wl = I.workload_c3(oracle_lib.template_fn(), n_win=4, n_cand=1)
    ctx = api.context_for(wl.T)
    pop = 96
    boxes = [wl.window_box(i) for i in range(wl.n_win)]
    be = D.GpuBackend(ctx, wl.window_table(), dev(wl.data, torch.complex128), dev(wl.weights), api.GB_FP64)
    lo, hi = D._box_arrays(boxes)
    lo, hi = lo[:, list(D.SEARCH_DIMS)], hi[:, list(D.SEARCH_DIMS)]
    rng = np.random.default_rng(8)
    x = lo[:, None, :] + (hi - lo)[:, None, :] * rng.random((wl.n_win, pop, 7))
    plan = be._plan(pop, api.GB_FP64)
    s = np.full((wl.n_win, pop), -np.inf)
    _, c = plan.loglik(dev(de.to_theta(x, D.REF_AMP).reshape(-1, 8)), comps=True)
    xg, sg = dev(x), dev(s)
    bi = torch.empty(wl.n_win, dtype=torch.int32, device="cuda")
    api.gb_de_select(c, xg, sg, xg.clone(), best_idx=bi)
    x, s, _, rbi = de.select(c.cpu().numpy(), x, s, x)
    for g in range(10):
        u_idx, u_cross, u_j = rng.random((wl.n_win, pop, 3)), rng.random((wl.n_win, pop, 7)), rng.random((wl.n_win, pop))
        F = np.full(wl.n_win, rng.uniform(0.5, 1.0))
        use_best = g % 2 == 1                        # alternate the two strategies
        tx, th = api.gb_de_trial(dev(lo), dev(hi), xg, dev(u_idx), dev(u_cross), dev(u_j), dev(F), 0.7, D.REF_AMP,
                                 base=bi if use_best else None)
        _, c = plan.loglik(th, comps=True)
        best = api.gb_de_select(c, xg, sg, tx, best_idx=bi)
        rtx, _ = de.trial(lo, hi, x, u_idx, u_cross, u_j, F, 0.7, D.REF_AMP, base=rbi if use_best else None)
        assert np.array_equal(tx.cpu().numpy(), rtx)
        x, s, rbest, rbi = de.select(c.cpu().numpy(), x, s, rtx)
        assert np.array_equal(xg.cpu().numpy(), x) and np.array_equal(sg.cpu().numpy(), s)
        assert np.array_equal(best.cpu().numpy(), rbest) and np.array_equal(bi.cpu().numpy(), rbi)
    be.close()


def test_device_de_search_finds_sources(oracle_lib):
    banner("device-resident DE search (no host work per generation) on loud windows")
    from tests.test_search_cpu import segments_workload
    wl, seg = segments_workload(oracle_lib)
    ctx = api.context_for(wl.T)
    be = D.GpuBackend(ctx, wl.window_table(), dev(wl.data, torch.complex128), dev(wl.weights), api.GB_FP64)
    boxes = [wl.window_box(i) for i in range(wl.n_win)]
    th, rho, hist = D.de_search(be, boxes, np.random.default_rng(4), pop=256, generations=150, keep=2)
    assert th.shape == (wl.n_win, 2, 8) and hist.shape == (151, wl.n_win)
    assert np.all(np.diff(hist, axis=0) >= 0)                  # greedy: the best never drops
    for i, w in enumerate(wl.windows):
        if len(w.sources):
            assert abs(th[i, 0, 0] - w.sources[0, 0]) * wl.T < 1.0, (i, th[i, 0, 0] * wl.T, w.sources[0, 0] * wl.T)
    be.close()


def test_device_de_convergence_stop(oracle_lib):
    banner("device DE with SciPy's convergence stop: windows leave the batch as they converge")
    from tests.test_search_cpu import segments_workload
    wl, seg = segments_workload(oracle_lib)
    ctx = api.context_for(wl.T)
    be = D.GpuBackend(ctx, wl.window_table(), dev(wl.data, torch.complex128), dev(wl.weights), api.GB_MIXED)
    boxes = [wl.window_box(i) for i in range(wl.n_win)]
    th, rho, hist = D.de_search(be, boxes, np.random.default_rng(5), pop=128, generations=600, keep=2,
                                tol=0.01, check_every=10)
    assert th.shape == (wl.n_win, 2, 8) and hist.shape == (601, wl.n_win)
    assert np.all(np.isfinite(hist)) and np.all(np.diff(hist, axis=0) >= 0)
    # the windows with a loud source converged on it and stopped early: their best rho is flat
    # over the last generations
    for i, w in enumerate(wl.windows):
        if len(w.sources):
            assert abs(th[i, 0, 0] - w.sources[0, 0]) * wl.T < 1.0
            assert hist[-1, i] == hist[-100, i]
    assert np.allclose(rho[:, 0], hist[-1])
    be.close()


def test_device_de_graph_matches_eager(oracle_lib):
    """The device DE replayed from captured HIP graphs against the same DE launched eagerly. Both
    consume the same draws, so populations, scores and the whole history must agree bit for bit,
    over many chunk replays with eager host work (the convergence checks) between them,
    compactions with re-captures, and a partial last chunk run eagerly.  The chunks are captured
    in global mode, where any unsafe call during the capture fails it."""
    banner("device DE: HIP-graph chunks vs eager launches")
    from paper_2307_03763_amd import drivers as D
    assert D.CAPTURE_MODE == "global"
    from tests.test_search_cpu import segments_workload
    wl, seg = segments_workload(oracle_lib)
    ctx = api.context_for(wl.T)
    be = D.GpuBackend(ctx, wl.window_table(), dev(wl.data, torch.complex128), dev(wl.weights), api.GB_MIXED)
    boxes = [wl.window_box(i) for i in range(wl.n_win)]
    out, chunks = [], []
    for graph in (True, False):
        out.append(D.de_search(be, boxes, np.random.default_rng(5), pop=128, generations=205, keep=2, tol=0.01,
                               check_every=10, graph=graph))
        chunks.append(dict(be.de_chunks))
    banner(f"  chunks with graphs: {chunks[0]}; eager: {chunks[1]}")
    assert chunks[0]["replays"] >= 3 and chunks[0]["captures"] >= 1
    assert chunks[1]["replays"] == 0 and chunks[1]["captures"] == 0
    for a, b in zip(*out):
        assert np.array_equal(a, b)
    be.close()
