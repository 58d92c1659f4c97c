"""Drivers around the batched likelihood: the search, polish and posterior stages.

* ``de_search`` -- the differential-evolution search of Algorithm 2 / Sec. III D, run for many
  windows at once: each window has its own population in Table I coordinates without the
  amplitude, every generation of every window is scored in one batched likelihood call by the
  SNR rho = <d|h> / sqrt(<h|h>) (Sec. III SNR equation, independent of the amplitude), and the
  kept members of each window get A_max = A <d|h> / <h|h> (Sec. III amplitude equation).
  Mutation is DE/best/1/bin by default (SciPy's default strategy: mutants around each window's
  best member), or DE/rand/1/bin, with a scale factor dithered per generation.
* ``polish`` -- refinement of many starting points at once by quasi-Newton (BFGS) ascent on
  logL: per iteration one batched gradient call, then one batched line search (all trial step
  lengths of all starts in one likelihood call).
* ``search`` -- DE, then the polish of its best members, with restarts (Sec. III D).
* ``PosteriorStage`` -- one temperature of Algorithm 4: proposals drawn uniformly in a box in
  Table I coordinates (so the proposal density is constant there and cancels), logL of all of
  them in parallel and the independent-proposal chain, in one ``gb_mh_step``; optionally
  captured once in a HIP graph and replayed.

The drivers only choose parameters and keep the best values; every likelihood, gradient and
chain is computed by a backend.  A backend evaluates ``theta`` of shape [n_win * n, 8] laid out
window-major (rows i*n .. i*n+n-1 belong to window i) and returns (logL [n_win*n],
comps [n_win*n, 2]) from ``loglik`` and (logL, grad [n_win*n, 8]) from ``loglik_grad``.
``GpuBackend`` calls the HIP library.
"""

from __future__ import annotations

import math
from typing import Optional

import numpy as np

from . import inputs as I

# Table I coordinates searched by DE: all but log10 A (index 4), which is profiled
SEARCH_DIMS = (0, 1, 2, 3, 5, 6, 7)
PERIODIC = (3, 6, 7)
REF_AMP = 1e-22


class GpuBackend:
    """Batched logL / gradient through the HIP library for the windows of ``table`` (rows as in
    ``Workload.window_table``: k0, W, N, C, data_off, w_off, ...; an optional 9th column holds the
    per-window precision for GB_PER_WINDOW).  The candidate slices are rewritten per call; plans
    are cached per (candidates per window, precision).  The DE search runs on the device with
    this backend (gb_de_trial / gb_de_select; population and scores stay in HBM)."""

    device_de = True

    def __init__(self, ctx, table, d, w, precision_logl: int, precision_grad: Optional[int] = None):
        import torch
        from . import api
        self.api, self.torch = api, torch
        self.ctx = ctx
        t = np.asarray(table, dtype=np.int64)
        self.table = t.reshape(-1, t.shape[-1]).copy()
        self.n_win = len(self.table)
        self.d, self.w = d, w
        self.pl = precision_logl
        self.pg = api.GB_MIXED if precision_grad is None else precision_grad
        self.plans = {}

    def _plan(self, n: int, prec: int):
        key = (n, prec)
        if key not in self.plans:
            t = self.table.copy()
            t[:, 6] = np.arange(self.n_win) * n
            t[:, 7] = n
            p = self.api.Plan(self.ctx, t, prec)
            p.prepare(self.d, self.w)
            self.plans[key] = p
        return self.plans[key]

    def _sub_plan(self, rows, n: int, prec: int):
        """A plan over the windows ``rows`` only, n candidates each (not cached: the caller
        closes it)."""
        t = self.table[np.asarray(rows)].copy()
        t[:, 6] = np.arange(len(t)) * n
        t[:, 7] = n
        p = self.api.Plan(self.ctx, t, prec)
        p.prepare(self.d, self.w)
        return p

    def _n(self, theta) -> int:
        if len(theta) % self.n_win:
            raise ValueError("theta rows must be a multiple of the window count")
        return len(theta) // self.n_win

    def loglik(self, theta: np.ndarray):
        th = self.torch.as_tensor(np.ascontiguousarray(theta, dtype=np.float64), device="cuda")
        l, c = self._plan(self._n(theta), self.pl).loglik(th, comps=True)
        return l.cpu().numpy(), c.cpu().numpy()

    def loglik_grad(self, theta: np.ndarray):
        th = self.torch.as_tensor(np.ascontiguousarray(theta, dtype=np.float64), device="cuda")
        l, g = self._plan(self._n(theta), self.pg).loglik_grad(th)
        return l.cpu().numpy(), g.cpu().numpy()

    def close(self):
        for p in self.plans.values():
            p.close()
        self.plans.clear()


def _snr(comps: np.ndarray) -> np.ndarray:
    with np.errstate(invalid="ignore", divide="ignore"):
        rho = comps[..., 0] / np.sqrt(comps[..., 1])
    return np.where(np.isfinite(rho), rho, -np.inf)


def _box_arrays(boxes) -> tuple:
    if isinstance(boxes, I.PriorBox):
        boxes = [boxes]
    return np.stack([b.lo for b in boxes]), np.stack([b.hi for b in boxes])


def _fold_into_box(m: np.ndarray, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """Periodic angles wrap into [lo, hi); the other coordinates reflect at the walls.
    m: [n_win, pop, 7]; lo, hi: [n_win, 7]."""
    out = m.copy()
    for k, dim_i in enumerate(SEARCH_DIMS):
        lk, hk = lo[:, k, None], hi[:, k, None]
        v = m[..., k]
        if dim_i in PERIODIC:
            out[..., k] = lk + np.mod(v - lk, hk - lk)
        else:
            v = np.where(v < lk, 2 * lk - v, v)
            v = np.where(v > hk, 2 * hk - v, v)
            out[..., k] = np.clip(v, lk, hk)
    return out


def _three_others(rng: np.random.Generator, n_win: int, pop: int) -> np.ndarray:
    """For each member i of each population, three distinct indices, all different from i."""
    idx = rng.integers(0, pop, size=(n_win, pop, 3))
    me = np.arange(pop)[None, :]
    for _ in range(1000):
        bad = ((idx[..., 0] == me) | (idx[..., 1] == me) | (idx[..., 2] == me)
               | (idx[..., 0] == idx[..., 1]) | (idx[..., 0] == idx[..., 2])
               | (idx[..., 1] == idx[..., 2]))
        if not bad.any():
            return idx
        idx[bad] = rng.integers(0, pop, size=(int(bad.sum()), 3))
    raise RuntimeError("population too small for DE/rand/1")


def _to_theta(x: np.ndarray) -> np.ndarray:
    u = np.empty(x.shape[:-1] + (8,))
    u[..., list(SEARCH_DIMS)] = x
    u[..., 4] = math.log10(REF_AMP)
    return I.from_table1(u)


def tune_on_windows(ctx, table, d, w, boxes, per_window: int = 512, rng: Optional[np.random.Generator] = None,
                    reps: int = 2) -> str:
    """Launch shapes of ``ctx`` chosen on the work a search or a posterior gives it: the windows of
    ``table`` on the data d and weights w, with ``per_window`` candidates each drawn uniformly in
    the window's Table I box (as a DE population starts; amplitude at the reference value), timed
    by gb_autotune_windows.  Plans created afterwards use the choice; returns its report."""
    import torch
    from . import api
    rng = np.random.default_rng(0) if rng is None else rng
    lo, hi = _box_arrays(boxes)
    lo, hi = lo[:, list(SEARCH_DIMS)], hi[:, list(SEARCH_DIMS)]
    t = np.asarray(table, dtype=np.int64).reshape(len(table), -1).copy()
    n = len(t)
    x = lo[:, None, :] + rng.random((n, per_window, lo.shape[1])) * (hi - lo)[:, None, :]
    th = torch.as_tensor(_to_theta(x).reshape(-1, 8), dtype=torch.float64, device="cuda")
    t[:, 6] = np.arange(n) * per_window
    t[:, 7] = per_window
    return api.gb_autotune_windows(ctx.handle, t, d, w, th, reps)


def de_search(backend, boxes, rng: np.random.Generator, pop: int = 512, generations: int = 50,
              cr: float = 0.7, f_lo: float = 0.5, f_hi: float = 1.0, init: Optional[np.ndarray] = None,
              keep: int = 1, on_device: Optional[bool] = None, strategy: str = "best1", tol: float = 0.0,
              check_every: int = 50, graph: bool = True):
    """Maximise rho over the seven non-amplitude parameters inside each window's Table I box.

    ``boxes`` is one PriorBox per window of the backend (or a single one for one window);
    ``init`` optionally seeds member 0 of each population ([n_win, 8] or [8]).  With a backend
    that offers it (``device_de``) the generations run on the device (``on_device`` False keeps
    them on the host: the same DE with NumPy's random streams).  ``strategy``: "rand1"
    (DE/rand/1/bin) or "best1" (DE/best/1/bin, SciPy's default: mutants around each window's
    best member).  ``tol`` > 0 stops a window once its population has converged in SciPy's
    sense, std(rho) <= tol |mean(rho)| (SciPy's default tol is 0.01), checked every
    ``check_every`` generations; a stopped window keeps its population (on the device the
    converged windows leave the batch once a quarter of it has converged).  ``graph``: on the
    device, replay each chunk of ``check_every`` generations from one captured HIP graph.
    Returns
    (theta [n_win, keep, 8] of the best ``keep`` members with A = A_max, rho [n_win, keep],
    history [generations + 1, n_win] of the best rho per generation)."""
    lo, hi = _box_arrays(boxes)
    lo, hi = lo[:, list(SEARCH_DIMS)], hi[:, list(SEARCH_DIMS)]
    n_win, dim = lo.shape
    if pop < 4 or not 1 <= keep <= pop:
        raise ValueError("DE needs pop >= 4 and 1 <= keep <= pop")
    if strategy not in ("rand1", "best1"):
        raise ValueError("strategy must be 'rand1' or 'best1'")
    if on_device is None:
        on_device = getattr(backend, "device_de", False)
    if on_device:
        x, s, history = _de_device(backend, lo, hi, rng, pop, generations, cr, f_lo, f_hi, init, strategy == "best1",
                                   tol, check_every, graph)
        return _de_finish(backend, x, s, history, keep)
    x = lo[:, None, :] + (hi - lo)[:, None, :] * rng.random((n_win, pop, dim))
    if init is not None:
        x[:, 0, :] = I.to_table1(np.broadcast_to(init, (n_win, 8)))[:, list(SEARCH_DIMS)]

    def score(xx):
        _, comps = backend.loglik(_to_theta(xx).reshape(n_win * pop, 8))
        return _snr(comps).reshape(n_win, pop)

    s = score(x)
    history = [s.max(axis=1)]
    wi = np.arange(n_win)[:, None]
    stopped = np.zeros(n_win, dtype=bool)
    for g in range(1, generations + 1):
        r = _three_others(rng, n_win, pop)
        fscale = rng.uniform(f_lo, f_hi)
        if strategy == "best1":
            base = x[np.arange(n_win), np.argmax(s, axis=1)][:, None, :]
            mutant = base + fscale * (x[wi, r[..., 0]] - x[wi, r[..., 1]])
        else:
            mutant = x[wi, r[..., 0]] + fscale * (x[wi, r[..., 1]] - x[wi, r[..., 2]])
        mutant = _fold_into_box(mutant, lo, hi)
        cross = rng.random((n_win, pop, dim)) < cr
        cross[wi, np.arange(pop)[None, :], rng.integers(0, dim, (n_win, pop))] = True
        trial = np.where(cross, mutant, x)
        s_trial = score(trial)
        better = (s_trial > s) & ~stopped[:, None]
        x[better] = trial[better]
        s[better] = s_trial[better]
        history.append(s.max(axis=1))
        if tol > 0 and g % check_every == 0:
            with np.errstate(invalid="ignore"):
                stopped |= _de_converged(s, tol)
            if stopped.all():
                history += [history[-1]] * (generations - g)
                break
    return _de_finish(backend, x, s, np.array(history), keep)


def _de_converged(s, tol: float) -> np.ndarray:
    """SciPy's convergence test per window: std(rho) <= tol |mean(rho)| over the population."""
    m = s.mean(axis=1)
    return np.isfinite(m) & (s.std(axis=1) <= tol * np.abs(m))


# Capture mode of every graph the drivers record: "global", so that a call from any thread that
# is unsafe during a capture (an allocation, a free, a synchronisation) is reported at once.
CAPTURE_MODE = "global"


def _capture_graph(torch, gr, stream, body):
    """Record body() into the HIP graph gr on stream, in CAPTURE_MODE.  Plans and contexts
    destroyed while it runs (by the cyclic garbage collector, for instance) free their device
    memory after the capture (api.capturing), not inside it."""
    from . import api
    with api.capturing():
        with torch.cuda.graph(gr, stream=stream, capture_error_mode=CAPTURE_MODE):
            body()


# Share of the device DE batch that must have converged before the converged windows leave it:
# each compaction costs a new plan and a new graph capture, about one eager chunk.
COMPACT_FRACTION = 0.25


def _de_device(backend, lo, hi, rng, pop, generations, cr, f_lo, f_hi, init, best1=False, tol=0.0,
               check_every=50, graph=True):
    """The DE generations with the population, scores and random draws in device memory: per
    generation one gb_de_trial, one gb_loglik of all trials and one gb_de_select, with no copy
    to the host.

    The generations run in chunks of ``check_every``. A chunk's uniforms come from a torch
    generator seeded by ``rng`` and are drawn into fixed buffers before the chunk runs; its F
    values (one per generation, from ``rng`` as in the host loop) are copied in one transfer.
    gb_de_select writes each generation's best rho into the chunk's history rows. With
    ``graph``, the chunk's launches are captured once in a HIP graph and every later chunk of the
    same batch is one replay (the first chunk, and partial chunks, run eagerly); graph and eager
    runs consume the same draws and give identical results.

    With tol > 0, after every chunk the windows whose population has converged (std(rho) <= tol
    |mean(rho)|) are noted. Once a quarter of the batch has converged (or all of it), those
    windows leave the batch (their members are kept) and the rest run on a plan of their own,
    with a new capture (COMPACT_FRACTION). Converged windows that stay in the batch until then
    keep evolving, which greedy selection can only improve. Returns (x, s, history) as NumPy arrays."""
    torch, api = backend.torch, backend.api
    dev = torch.device("cuda")
    f64 = torch.float64
    n_win, dim = lo.shape
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(rng.integers(0, 2 ** 62)))
    lo_t = torch.as_tensor(np.ascontiguousarray(lo), dtype=f64, device=dev)
    hi_t = torch.as_tensor(np.ascontiguousarray(hi), dtype=f64, device=dev)
    x = lo_t[:, None, :] + (hi_t - lo_t)[:, None, :] * torch.rand((n_win, pop, dim), generator=gen, dtype=f64,
                                                                   device=dev)
    if init is not None:
        x0 = I.to_table1(np.broadcast_to(np.asarray(init, dtype=np.float64), (n_win, 8)))[:, list(SEARCH_DIMS)]
        x[:, 0, :] = torch.as_tensor(np.ascontiguousarray(x0), device=dev)
    x = x.contiguous()
    s = torch.full((n_win, pop), -np.inf, dtype=f64, device=dev)
    plan = backend._plan(pop, backend.pl)
    th0 = torch.as_tensor(np.ascontiguousarray(_to_theta(x.cpu().numpy()).reshape(n_win * pop, 8)), device=dev)
    _, comps = plan.loglik(th0, comps=True)
    best_idx = torch.zeros(n_win, dtype=torch.int32, device=dev)
    hist = torch.full((generations + 1, n_win), np.nan, dtype=f64, device=dev)
    hist[0] = api.gb_de_select(comps, x, s, x.clone(), best_idx=best_idx)
    K = max(1, int(check_every))

    def buffers(na):
        return dict(ui=torch.empty((K, na, pop, 3), dtype=f64, device=dev),
                    uc=torch.empty((K, na, pop, dim), dtype=f64, device=dev),
                    uj=torch.empty((K, na, pop), dtype=f64, device=dev),
                    F=torch.empty((K, na), dtype=f64, device=dev),
                    best=torch.empty((K, na), dtype=f64, device=dev),
                    tx=torch.empty((na, pop, dim), dtype=f64, device=dev),
                    tth=torch.empty((na * pop, 8), dtype=f64, device=dev))

    def chunk(B, k):
        for j in range(k):
            api.gb_de_trial(lo_a, hi_a, xa, B["ui"][j], B["uc"][j], B["uj"][j], B["F"][j], cr, REF_AMP, B["tx"],
                            B["tth"], base=ba if best1 else None)
            _, cj = plan_a.loglik(B["tth"], comps=True)
            api.gb_de_select(cj, xa, sa, B["tx"], best=B["best"][j], best_idx=ba)

    def capture(B):
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        gr = torch.cuda.CUDAGraph()
        _capture_graph(torch, gr, side, lambda: chunk(B, K))
        torch.cuda.current_stream().wait_stream(side)
        return gr

    # the active windows' arrays (the whole batch until a compaction)
    act = torch.arange(n_win, device=dev)
    xa, sa, ba, lo_a, hi_a, plan_a, own_plan = x, s, best_idx, lo_t, hi_t, plan, False
    B, gr, eager_chunks, captures, replays = buffers(n_win), None, 0, 0, 0
    g = 1
    while g <= generations:
        na = len(act)
        k = min(K, generations - g + 1)
        B["ui"][:k].uniform_(generator=gen)
        B["uc"][:k].uniform_(generator=gen)
        B["uj"][:k].uniform_(generator=gen)
        Fk = torch.as_tensor(rng.uniform(f_lo, f_hi, k), dtype=f64)
        B["F"][:k].copy_(Fk[:, None].expand(k, na))
        if graph and k == K and eager_chunks > 0:
            if gr is None:
                gr = capture(B)
                captures += 1
            gr.replay()
            replays += 1
        else:
            chunk(B, k)
            eager_chunks += 1
        hist[g:g + k, act] = B["best"][:k]
        g += k
        if tol > 0 and g <= generations:
            m = sa.mean(dim=1)
            conv = torch.isfinite(m) & (sa.std(dim=1, unbiased=False) <= tol * m.abs())
            n_conv = int(conv.sum().item())
            if n_conv and (n_conv == na or n_conv >= COMPACT_FRACTION * na):
                if xa is not x:                        # write the converged windows back
                    x[act[conv]] = xa[conv]
                    s[act[conv]] = sa[conv]
                gr = None                              # the graph refers to the plan and buffers
                if own_plan:
                    plan_a.close()
                if n_conv == na:
                    act = act[:0]
                    break
                keep_w = ~conv
                if xa is x:                            # the first compaction: copy out the active rows
                    xa, sa, ba = x[keep_w].contiguous(), s[keep_w].contiguous(), best_idx[keep_w].contiguous()
                else:
                    xa, sa, ba = xa[keep_w].contiguous(), sa[keep_w].contiguous(), ba[keep_w].contiguous()
                act = act[keep_w]
                lo_a, hi_a = lo_t[act].contiguous(), hi_t[act].contiguous()
                plan_a, own_plan = backend._sub_plan(act.cpu().numpy(), pop, backend.pl), True
                B = buffers(len(act))
    gr = None
    # how the chunks ran (eagerly, captured, replayed), for tests and diagnostics
    backend.de_chunks = dict(eager=eager_chunks, captures=captures, replays=replays)
    if len(act) and xa is not x:
        x[act] = xa
        s[act] = sa
    if own_plan and len(act):
        plan_a.close()
    # a window that left the batch keeps its best value for the remaining generations
    h = hist.cpu().numpy()
    for g in range(1, generations + 1):
        miss = np.isnan(h[g])
        h[g, miss] = h[g - 1, miss]
    return x.cpu().numpy(), s.cpu().numpy(), h


def _de_finish(backend, x, s, history, keep):
    """The best ``keep`` members of every window with A = A_max, their rho, and the history."""
    n_win, pop, _ = x.shape
    wi = np.arange(n_win)[:, None]
    order = np.argsort(-s, axis=1, kind="stable")[:, :keep]
    th = _to_theta(x[wi, order])                               # [n_win, keep, 8]
    # A_max of the kept members: one more batched call, padded to the population size so
    # that the plan of the scoring calls is reused
    pad = np.repeat(th[:, :1, :], pop, axis=1)
    pad[:, :keep, :] = th
    _, comps = backend.loglik(pad.reshape(n_win * pop, 8))
    comps = comps.reshape(n_win, pop, 2)[:, :keep, :]
    th[..., 4] = REF_AMP * comps[..., 0] / comps[..., 1]
    return th, s[wi, order], history


def _table1_jacobian(theta: np.ndarray) -> np.ndarray:
    """d theta / d u for the Table I coordinates u (sin beta, log10 A, cos iota changed)."""
    j = np.ones_like(theta)
    j[..., 2] = 1.0 / np.maximum(np.cos(theta[..., 2]), 1e-12)
    j[..., 4] = theta[..., 4] * math.log(10.0)
    j[..., 5] = -1.0 / np.maximum(np.sin(theta[..., 5]), 1e-12)
    return j


def polish(backend, theta0: np.ndarray, scale: np.ndarray, iterations: int = 20, n_steps: int = 32,
           tol: float = 1e-9):
    """Quasi-Newton (BFGS) ascent on logL from many starts at once.

    ``theta0`` is [n_win, k, 8]: k starts in each window of the backend ([k, 8] or [8] for one
    window).  ``scale`` is the per-coordinate scale s in Table I coordinates, broadcast to
    [n_win, k, 8] (a Fisher sigma is the natural choice, a small fraction of the box widths a
    safe one); the search runs in x = u / s.  Each iteration takes one batched gradient call,
    then evaluates alpha * p along each start's BFGS direction p for alpha in {0} and
    10^-6 .. 10^2 in one batched likelihood call and keeps each start's best.  A start stops
    when no step raises its logL by more than `tol`.
    Returns (theta shaped like theta0, logL history [iterations + 1] + theta0's leading shape)."""
    th0 = np.asarray(theta0, dtype=np.float64)
    shape = th0.shape
    th = th0.reshape((-1,) + shape[-2:]) if th0.ndim == 3 else th0.reshape(1, -1, 8)
    n_win, k, _ = th.shape
    s = np.broadcast_to(np.asarray(scale, dtype=np.float64), (n_win, k, 8)).copy()
    alphas = np.concatenate([[0.0], np.logspace(-6, 2, n_steps - 1)])
    na = len(alphas)
    H = np.broadcast_to(np.eye(8), (n_win, k, 8, 8)).copy()
    active = np.ones((n_win, k), dtype=bool)
    wi, ki = np.arange(n_win)[:, None], np.arange(k)[None, :]

    def grad_x(t):
        _, g = backend.loglik_grad(t.reshape(n_win * k, 8))
        return g.reshape(n_win, k, 8) * _table1_jacobian(t) * s

    # logL values come from the likelihood calls (the precision chosen for scoring); the
    # gradient calls only supply directions and curvature pairs
    gx = grad_x(th)
    l0, _ = backend.loglik(th.reshape(n_win * k, 8))
    cur = l0.reshape(n_win, k)
    hist = [cur.copy()]
    x = I.to_table1(th) / s
    for _ in range(iterations):
        if not active.any():
            hist.append(cur.copy())
            continue
        p = np.matmul(H, gx[..., None])[..., 0]
        bad = np.sum(p * gx, axis=-1) <= 0.0
        if bad.any():                                           # not an ascent direction
            H[bad] = np.eye(8)
            p[bad] = gx[bad]
        pn = np.linalg.norm(p, axis=-1, keepdims=True)
        p = np.where(pn > 0, p / np.where(pn > 0, pn, 1.0), 0.0)
        p[~active] = 0.0
        trial_u = (x[:, :, None, :] + alphas[None, None, :, None] * p[:, :, None, :]) * s[:, :, None, :]
        trial_u[..., 2] = np.clip(trial_u[..., 2], -1.0, 1.0)
        trial_u[..., 5] = np.clip(trial_u[..., 5], -1.0, 1.0)
        trial = I.from_table1(trial_u)                          # [n_win, k, na, 8]
        lt, _ = backend.loglik(trial.reshape(n_win * k * na, 8))
        lt = lt.reshape(n_win, k, na)
        lt = np.where(np.isfinite(lt), lt, -np.inf)
        j = np.argmax(lt, axis=-1)
        best = lt[wi, ki, j]
        move = active & (j > 0) & (best - cur > tol)
        active = move
        th_new = np.where(move[..., None], trial[wi, ki, j], th)
        x_new = I.to_table1(th_new) / s
        gx_new = grad_x(th_new)
        sk, yk = x_new - x, gx - gx_new                         # curvature pairs of -logL
        sy = np.sum(sk * yk, axis=-1)
        upd = move & (sy > 1e-12 * np.linalg.norm(sk, axis=-1) * np.linalg.norm(yk, axis=-1))
        if upd.any():
            r = 1.0 / sy[upd]
            su, yu = sk[upd], yk[upd]
            V = np.eye(8)[None] - r[:, None, None] * (su[:, :, None] * yu[:, None, :])
            H[upd] = (np.matmul(np.matmul(V, H[upd]), V.transpose(0, 2, 1))
                      + r[:, None, None] * (su[:, :, None] * su[:, None, :]))
        cur = np.where(move, best, cur)
        th, x, gx = th_new, x_new, gx_new
        hist.append(cur.copy())
    return th.reshape(shape), np.array(hist).reshape((iterations + 1,) + shape[:-1])


def search(backend, boxes, rng: np.random.Generator, pop: int = 512, generations: int = 50,
           keep: int = 8, polish_iterations: int = 20, scale_frac: float = 1e-3, n_searches: int = 1,
           strategy: str = "best1", tol: float = 0.0):
    """Maximum-likelihood search of Sec. III D for every window of the backend: DE over the box,
    then the BFGS polish of the ``keep`` best members (scale: ``scale_frac`` of the box widths),
    repeated ``n_searches`` times from fresh populations in case a search ends at a local
    optimum.  Returns (theta [n_win, 8], logL [n_win]) of the best polished point per window."""
    lo, hi = _box_arrays(boxes)
    n_win = len(lo)
    best_th = np.full((n_win, 8), np.nan)
    best_l = np.full(n_win, -np.inf)
    scale = (scale_frac * (hi - lo))[:, None, :]
    for _ in range(n_searches):
        th, _, _ = de_search(backend, boxes, rng, pop=pop, generations=generations, keep=keep, strategy=strategy,
                             tol=tol)
        th, hist = polish(backend, th, scale, iterations=polish_iterations)
        l_end = hist[-1]                                       # [n_win, keep]
        j = np.argmax(l_end, axis=1)
        cand_l = l_end[np.arange(n_win), j]
        better = cand_l > best_l
        best_th[better] = th[np.arange(n_win), j][better]
        best_l[better] = cand_l[better]
    return best_th, best_l


class PosteriorStage:
    """One temperature of Algorithm 4 on the single window of a prepared plan whose window holds
    n candidates: n proposals uniform in the box [lo, hi] (Table I coordinates, so log g = 0),
    their logL and the independent-proposal chain, all in one ``gb_mh_step``.  ``run()`` launches
    the stage eagerly on the current stream; ``capture()`` records it once in a HIP graph (the
    draws come from ``generator``, which every replay advances) and ``replay()`` re-launches it.
    After either, the buffers theta, u, logL, chain and n_accept hold the stage's result."""

    def __init__(self, plan, box_lo: np.ndarray, box_hi: np.ndarray, temperature: float, generator=None):
        import torch
        self.torch = torch
        if plan.n_win != 1:
            raise ValueError("PosteriorStage drives a plan of one window")
        dev = torch.device("cuda")
        self.plan, self.T = plan, float(temperature)
        self.gen = generator if generator is not None else torch.cuda.default_generators[torch.cuda.current_device()]
        self.n = int(plan.table[0, 7])
        self.lo = torch.as_tensor(np.asarray(box_lo, dtype=np.float64), device=dev)
        self.hi = torch.as_tensor(np.asarray(box_hi, dtype=np.float64), device=dev)
        rows = plan.rows
        self.r = torch.empty((rows, 8), dtype=torch.float64, device=dev)
        self.theta = torch.zeros((rows, 8), dtype=torch.float64, device=dev)
        self.u = torch.empty(rows, dtype=torch.float64, device=dev)
        self.log_g = torch.zeros(rows, dtype=torch.float64, device=dev)
        self.logL = torch.empty(rows, dtype=torch.float64, device=dev)
        self.chain = torch.empty(rows, dtype=torch.int32, device=dev)
        self.n_accept = torch.empty(1, dtype=torch.int64, device=dev)
        self.graph = None

    def _body(self, stream):
        torch = self.torch
        from . import api
        self.r.uniform_(generator=self.gen)
        v = self.lo + (self.hi - self.lo) * self.r
        th = self.theta
        th.copy_(v)
        th[:, 2] = torch.asin(v[:, 2].clamp(-1.0, 1.0))
        th[:, 4] = torch.pow(10.0, v[:, 4])
        th[:, 5] = torch.acos(v[:, 5].clamp(-1.0, 1.0))
        self.u.uniform_(generator=self.gen)
        api.gb_mh_step(self.plan.handle, self.plan.d, self.plan.w, th, self.log_g, self.u, self.T,
                       self.logL, self.chain, self.n_accept, stream)

    def run(self):
        self._body(self.torch.cuda.current_stream())

    def capture(self):
        torch = self.torch
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self._body(s)                # warm-up outside the capture
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        if self.gen is not torch.cuda.default_generators[torch.cuda.current_device()]:
            self.graph.register_generator_state(self.gen)   # the default one is registered by torch
        _capture_graph(torch, self.graph, s, lambda: self._body(s))
        torch.cuda.synchronize()

    def replay(self):
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()


# ---------------------------------------------------------------------------------------------
# Annealed posterior (Algorithm 4 with the proposal updates of Sec. III G)

KDE_PAIRS = ((4, 5), (3, 2), (0, 1))   # (log10 A, cos iota), (lambda, sin beta), (f0, fdot)
UNIFORM_DIMS = (6, 7)                   # psi, phi0: kept in their narrow reduced-box ranges


class UniformBox:
    """Proposals uniform in a box of Table I coordinates (log g constant, taken as 0)."""

    def __init__(self, lo, hi):
        self.lo, self.hi = np.asarray(lo, dtype=np.float64), np.asarray(hi, dtype=np.float64)

    def draw(self, rng, n, backend=None):
        u = self.lo + (self.hi - self.lo) * rng.random((n, 8))
        return u, np.zeros(n)


class PairKDE:
    """Proposal distribution of the later annealing stages: a weighted 2-D Gaussian KDE of the
    previous chain for each of the pairs (A, iota), (lambda, beta), (f, fdot) in Table I
    coordinates, and uniform psi, phi0 in the reduced box.  The kernel points are the chain's
    distinct states weighted by how often the chain holds them; bandwidth by Scott's rule,
    H = n_eff^(-1/3) * (weighted covariance of the pair).  Draws outside the prior box are drawn
    again (the truncation changes g only by a constant, which cancels in the acceptance ratio)."""

    def __init__(self, states_u, lo_prior, hi_prior, lo_box, hi_box):
        uniq, counts = np.unique(states_u, axis=0, return_counts=True)
        self.pts = uniq
        self.w = counts / counts.sum()
        n_eff = 1.0 / np.sum(self.w ** 2)
        self.chol = []
        for a, b in KDE_PAIRS:
            xy = uniq[:, [a, b]]
            mu = self.w @ xy
            d = xy - mu
            cov = (self.w[:, None] * d).T @ d / max(1e-300, 1.0 - np.sum(self.w ** 2))
            cov = cov + np.diag(1e-12 * np.maximum(np.abs(np.diag(cov)), 1e-300))
            H = cov * n_eff ** (-1.0 / 3.0)
            L = np.linalg.cholesky(H)
            self.chol.append([L[0, 0], L[1, 0], L[1, 1]])
        self.chol = np.array(self.chol)
        self.lo_p, self.hi_p = np.asarray(lo_prior), np.asarray(hi_prior)
        self.lo_b, self.hi_b = np.asarray(lo_box), np.asarray(hi_box)

    def draw(self, rng, n, backend):
        out = np.empty((n, 8))
        filled = 0
        for _ in range(1000):
            if filled >= n:
                break
            k = 2 * (n - filled) + 16
            u = np.empty((k, 8))
            for p, (a, b) in enumerate(KDE_PAIRS):
                j = rng.choice(len(self.pts), size=k, p=self.w)
                L = np.array([[self.chol[p, 0], 0.0], [self.chol[p, 1], self.chol[p, 2]]])
                u[:, [a, b]] = self.pts[j][:, [a, b]] + rng.standard_normal((k, 2)) @ L.T
            for d in UNIFORM_DIMS:
                u[:, d] = self.lo_b[d] + (self.hi_b[d] - self.lo_b[d]) * rng.random(k)
            # periodic angles (lambda, psi, phi0) are not bounded by the prior box
            ok = np.all((u[:, [0, 1, 2, 4, 5]] >= self.lo_p[[0, 1, 2, 4, 5]]) &
                        (u[:, [0, 1, 2, 4, 5]] <= self.hi_p[[0, 1, 2, 4, 5]]), axis=1)
            take = u[ok][: n - filled]
            out[filled:filled + len(take)] = take
            filled += len(take)
        if filled < n:
            raise RuntimeError("KDE proposals keep leaving the prior box")
        x = np.stack([out[:, [a, b]] for a, b in KDE_PAIRS], axis=1)          # [n, 3, 2]
        pts = np.stack([self.pts[:, [a, b]] for a, b in KDE_PAIRS], axis=0)   # [3, m, 2]
        wts = np.broadcast_to(self.w, (len(KDE_PAIRS), len(self.w)))
        log_g = backend.kde_logpdf(pts, np.ascontiguousarray(wts), self.chol, x)
        return out, log_g


def annealed_posterior(backend, theta_mle, box: I.PriorBox, rng: np.random.Generator,
                       temps=(15.0, 10.0, 5.0, 3.0, 2.0, 1.0), n: int = 10000, fd_step: float = 1e-9):
    """Algorithm 4 for one source: the Fisher matrix at theta_mle (finite differences with steps
    of ``fd_step`` of the Table I widths) gives sigma and the reduced box (Sec. III G); then for
    every temperature n proposals (uniform in the reduced box first, then from the pairwise KDE
    of the previous chain), their logL in parallel and the independent-proposal chain.
    Returns (per-stage list of dicts with T, states (theta of the chain, [n, 8]), n_accept,
    logL of the states; the reduced box (lo, hi); sigma in Table I coordinates)."""
    theta_mle = np.asarray(theta_mle, dtype=np.float64)
    F = backend.fisher(theta_mle[None, :], (fd_step * box.width)[None, :])[0]
    sigma = np.sqrt(np.diag(np.linalg.inv(F)))
    lo, hi = I.reduced_box(theta_mle, box, sigma)
    sampler = UniformBox(lo, hi)
    stages = []
    for T in temps:
        props_u, log_g = sampler.draw(rng, n, backend)
        props = I.from_table1(props_u)
        uni = rng.random(n)
        logL, chain, nacc = backend.mh(props, log_g, uni, T)
        states_u = props_u[chain]
        stages.append({"T": float(T), "states": props[chain], "n_accept": int(nacc), "logL": logL[chain]})
        sampler = PairKDE(states_u, box.lo, box.hi, lo, hi)
    return stages, (lo, hi), sigma


class GpuPosteriorBackend:
    """The library calls of the annealed posterior for one window: gb_fisher, gb_mh_step and
    gb_kde_logpdf (plans cached per proposal count)."""

    def __init__(self, ctx, window_row, d, w):
        import torch
        from . import api
        self.api, self.torch = api, torch
        self.ctx = ctx
        self.row = np.asarray(window_row, dtype=np.int64).copy()
        self.d, self.w = d, w
        self.plans = {}

    def _dev(self, a):
        return self.torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")

    def fisher(self, theta, steps):
        rows = np.repeat(self.row[None, :], len(theta), axis=0)
        return self.api.gb_fisher(self.ctx.handle, self._dev(theta), self._dev(steps), rows, self.w).cpu().numpy()

    def mh(self, theta, log_g, u, T):
        n = len(theta)
        if n not in self.plans:
            row = self.row.copy()
            row[6], row[7] = 0, n
            p = self.api.Plan(self.ctx, row[None, :], self.api.GB_FP64)
            p.prepare(self.d, self.w)
            self.plans[n] = p
        l, ch, na = self.plans[n].mh_step(self._dev(theta), self._dev(log_g), self._dev(u), T)
        return l.cpu().numpy(), ch.cpu().numpy(), int(na.cpu()[0])

    def kde_logpdf(self, pts, wts, chol, x):
        return self.api.gb_kde_logpdf(self._dev(pts), self._dev(wts), self._dev(chol), self._dev(x)).cpu().numpy()


# ---------------------------------------------------------------------------------------------
# Search within frequency segments (Algorithm 2), for many segments at once

def local_search(backend, seg_edges, rng: np.random.Generator, n_signals: int, rho_threshold: float = 9.0,
                 n_searches: int = 3, pop: int = 512, generations: int = 50, keep: int = 8,
                 polish_iterations: int = 20, scale_frac: float = 1e-3, joint_sweeps: int = 2, progress=None,
                 strategy: str = "best1", tol: float = 0.0):
    """Algorithm 2 for every window of the backend at once (each window = one padded segment;
    seg_edges [n_win, 2] = the unpadded segment's edges in Hz).  Per signal: n_searches DE +
    polish searches on the residual (the first one ends the window when rho on the analysed data
    is at most rho_threshold - 2), the best of them by rho on the residual ends the window when
    its rho on the analysed data is at most rho_threshold; a signal inside the unpadded segment
    joins theta_in, one outside joins theta_out; then theta_in is refined jointly on the data
    minus theta_out (block-coordinate polish: each source on the data minus all other found
    sources, ``joint_sweeps`` sweeps), and the residual becomes the data minus all found
    signals.  ``progress(message)``, if given, hears of every signal step.  Returns (theta_in,
    theta_out): per window a list of parameter vectors."""
    n_win = backend.n_win
    seg = np.asarray(seg_edges, dtype=np.float64)
    boxes = backend.boxes
    widths = np.stack([b.width for b in boxes])
    found_in = [[] for _ in range(n_win)]
    found_out = [[] for _ in range(n_win)]
    active = np.ones(n_win, dtype=bool)
    backend.set_residual(found_in, found_out)
    for step in range(n_signals):
        if not active.any():
            break
        if progress:
            progress(f"signal {step + 1}: {int(active.sum())} of {n_win} segments still searching, "
                     f"{sum(len(f) for f in found_in)} found")
        best_th = np.zeros((n_win, 8))
        best_rho = np.full(n_win, -np.inf)
        best_rho_an = np.full(n_win, -np.inf)
        for j in range(n_searches):
            th, _ = search(backend, boxes, rng, pop=pop, generations=generations, keep=keep,
                           polish_iterations=polish_iterations, scale_frac=scale_frac, strategy=strategy,
                           tol=tol)
            rho_res = _snr(backend.loglik(th)[1])
            rho_an = backend.rho_analyze(th)
            if j == 0:
                active &= ~(rho_an <= rho_threshold - 2.0)
            better = rho_res > best_rho
            best_th[better], best_rho[better], best_rho_an[better] = th[better], rho_res[better], rho_an[better]
        active &= ~(best_rho_an <= rho_threshold)
        for i in np.nonzero(active)[0]:
            inside = seg[i, 0] <= best_th[i, 0] < seg[i, 1]
            (found_in if inside else found_out)[i].append(best_th[i].copy())
        # joint refinement of the sources inside, each on the data minus all other found sources
        k_max = max((len(f) for f in found_in), default=0)
        for _ in range(joint_sweeps if k_max else 0):
            for k in range(k_max):
                has = np.array([len(found_in[i]) > k for i in range(n_win)]) & active
                if not has.any():
                    continue
                backend.set_residual([[t for m, t in enumerate(found_in[i]) if m != k or not has[i]]
                                      for i in range(n_win)], found_out)
                start = np.stack([found_in[i][k] if has[i] else _box_centre(boxes[i]) for i in range(n_win)])
                th, _ = polish(backend, start[:, None, :], (scale_frac * widths)[:, None, :],
                               iterations=polish_iterations)
                for i in np.nonzero(has)[0]:
                    found_in[i][k] = th[i, 0].copy()
        backend.set_residual(found_in, found_out)
    return found_in, found_out


def _box_centre(box: I.PriorBox) -> np.ndarray:
    return I.from_table1(0.5 * (box.lo + box.hi))


class GpuSearchBackend(GpuBackend):
    """The library calls of local_search for the windows of ``table``: likelihoods and gradients
    on the current residual (data minus the sources found so far, formed by gb_add_templates),
    and rho on the analysed data itself.  noise="psd" keeps the given weights; noise="median"
    follows the paper's dynamic local estimate: after every change of the residual, each
    window's weights become 4 / (T S) with S its median periodogram (gb_noise_estimate), and
    both the residual's and the analysed data's scalar products use them."""

    def __init__(self, ctx, table, d, w, boxes, precision_logl: int, precision_grad: Optional[int] = None,
                 noise: str = "psd"):
        if noise not in ("psd", "median"):
            raise ValueError("noise must be 'psd' or 'median'")
        self.noise = noise
        w_own = w.clone() if noise == "median" else w
        super().__init__(ctx, table, d.clone(), w_own, precision_logl, precision_grad)
        self.d_analyze = d
        self.boxes = list(boxes)
        self.analyze = GpuBackend(ctx, table, d, w_own, self.api.GB_FP64)

    def set_residual(self, *lists):
        theta, src = [], []
        for lst in lists:
            for i, srcs in enumerate(lst):
                for t in srcs:
                    theta.append(t)
                    src.append(i)
        th = self.torch.as_tensor(np.array(theta).reshape(-1, 8), dtype=self.torch.float64, device="cuda")
        self.api.gb_add_templates(self.ctx.handle, self.table, th, src, -1.0, self.d_analyze, self.d)
        if self.noise == "median":
            self.api.gb_noise_estimate(self.table, self.d, self.ctx.T, self.w)
            for p in self.analyze.plans.values():
                p.prepare(self.d_analyze, self.w)
        for p in self.plans.values():
            p.prepare(self.d, self.w)

    def rho_analyze(self, theta):
        return _snr(self.analyze.loglik(theta)[1])

    def close(self):
        super().close()
        self.analyze.close()


# ---------------------------------------------------------------------------------------------
# The global search over many segments (Algorithm 3 with the three runs of Table II)

def overlapping_windows(table, sources: np.ndarray, T: float) -> tuple:
    """(source index, window index) pairs: every window whose bins meet the N bins of the
    source's template at that window's N (first bin floor(f0 T) - N/2)."""
    t = np.asarray(table, dtype=np.int64)
    k0, W, N = t[:, 0], t[:, 1], t[:, 2]
    si, wi = [], []
    for s, th in enumerate(np.atleast_2d(sources)):
        q = int(np.floor(th[0] * T))
        first = q - N // 2
        hit = np.nonzero((first < k0 + W) & (first + N > k0))[0]
        si += [s] * len(hit)
        wi += list(hit)
    return np.array(si, dtype=np.int64), np.array(wi, dtype=np.int32)


def global_search(backend_factory, table, T: float, seg_edges, d, rng: np.random.Generator,
                  subtract, runs=((0, 3), (1, 10), (0, 10)), **search_kw):
    """Algorithm 3 over all segments: segments alternate even/odd by index; each run is
    local_search over the segments of one parity (all at once) on the data minus the sources the
    previous run found (Table II: even segments with n_signals = 3 on d, odd segments with 10 on
    d minus the even results, even segments again with 10 on d minus the odd results).
    ``backend_factory(rows, d_analyze)`` builds a search backend for a subset of windows;
    ``subtract(d, sources, src_win)`` returns d minus the listed templates (each in the windows
    given).  Returns (recovered parameter vectors [n, 8], index of the segment of each)."""
    t = np.asarray(table, dtype=np.int64)
    seg = np.asarray(seg_edges, dtype=np.float64)
    results = {}
    d_run = d
    progress = search_kw.get("progress")
    for parity, n_signals in runs:
        rows = np.arange(parity, len(t), 2)
        if progress:
            progress(f"run over the {'odd' if parity else 'even'} segments, up to {n_signals} signals each")
        be = backend_factory(rows, d_run)
        found_in, _ = local_search(be, seg[rows], rng, n_signals, **search_kw)
        if hasattr(be, "close"):
            be.close()
        results[parity] = [(rows[i], th) for i in range(len(rows)) for th in found_in[i]]
        srcs = np.array([th for _, th in results[parity]]).reshape(-1, 8)
        si, wi = overlapping_windows(t, srcs, T)
        d_run = subtract(d, srcs[si], wi) if len(si) else d
    rec = results.get(0, []) + results.get(1, [])
    if not rec:
        return np.zeros((0, 8)), np.zeros(0, dtype=np.int64)
    return np.array([th for _, th in rec]), np.array([r for r, _ in rec], dtype=np.int64)


def _from_table1_t(u):
    """Table I coordinates back to parameters, on tensors (as inputs.from_table1)."""
    import torch
    th = u.clone()
    th[..., 2] = torch.asin(u[..., 2].clamp(-1.0, 1.0))
    th[..., 4] = torch.pow(10.0, u[..., 4])
    th[..., 5] = torch.acos(u[..., 5].clamp(-1.0, 1.0))
    return th


class PairKDEBatch:
    """PairKDE for S sources at once, on tensors (on the backend's device): the proposals u
    [S, n, 8] (Table I coordinates) of a stage and its chains [S, n] (indices into them).  The
    kernel points of source s are its chain's distinct states weighted by how often the chain
    holds them, padded with zero weights to the largest count over the sources; bandwidths by
    Scott's rule as in PairKDE.  A kernel point of a pair is drawn by picking a uniform position
    of the chain (the same distribution as drawing a distinct state by its weight)."""

    def __init__(self, u, chain, lo_prior, hi_prior, lo_box, hi_box):
        import torch
        self.torch = torch
        S, n = chain.shape
        dev = u.device
        chain = chain.long()
        flat = (chain + n * torch.arange(S, device=dev)[:, None]).reshape(-1)
        counts = torch.bincount(flat, minlength=S * n).reshape(S, n).to(torch.float64)
        held = counts > 0
        m = int(held.sum(dim=1).max().item())
        order = torch.sort((~held).to(torch.int8), dim=1, stable=True).indices[:, :m]
        self.w = torch.gather(counts, 1, order) / n                               # [S, m]
        self.pts = torch.gather(u, 1, order[:, :, None].expand(S, m, 8))          # [S, m, 8]
        sw2 = (self.w * self.w).sum(dim=1)
        n_eff = 1.0 / sw2
        chol = []
        for a, b in KDE_PAIRS:
            xy = self.pts[:, :, [a, b]]
            mu = (self.w[:, :, None] * xy).sum(dim=1)
            d = xy - mu[:, None, :]
            wd = self.w[:, :, None] * d
            c00 = (wd[:, :, 0] * d[:, :, 0]).sum(dim=1)
            c01 = (wd[:, :, 0] * d[:, :, 1]).sum(dim=1)
            c11 = (wd[:, :, 1] * d[:, :, 1]).sum(dim=1)
            den = (1.0 - sw2).clamp(min=1e-300)
            c00, c01, c11 = c00 / den, c01 / den, c11 / den
            c00 = c00 + 1e-12 * c00.abs().clamp(min=1e-300)
            c11 = c11 + 1e-12 * c11.abs().clamp(min=1e-300)
            f = n_eff ** (-1.0 / 3.0)
            h00, h01, h11 = c00 * f, c01 * f, c11 * f
            l00 = torch.sqrt(h00)
            l10 = h01 / l00
            l11 = torch.sqrt((h11 - l10 * l10).clamp(min=0.0))
            l11 = torch.where(l11 > 0, l11, torch.sqrt(h11) * 1e-6)
            chol.append(torch.stack([l00, l10, l11], dim=1))
        self.chol = torch.stack(chol, dim=1)                                       # [S, 3, 3]
        self.u, self.chain = u, chain
        self.lo_p, self.hi_p = lo_prior, hi_prior
        self.lo_b, self.hi_b = lo_box, hi_box

    def _candidates(self, sel, k, gen):
        torch = self.torch
        S_a = len(sel)
        n = self.chain.shape[1]
        dev = self.u.device
        cand = torch.empty((S_a, k, 8), dtype=torch.float64, device=dev)
        u_a, ch_a = self.u[sel], self.chain[sel]
        for p, (a, b) in enumerate(KDE_PAIRS):
            t = torch.randint(0, n, (S_a, k), generator=gen, device=dev)
            j = torch.gather(ch_a, 1, t)
            base = torch.gather(u_a, 1, j[:, :, None].expand(S_a, k, 8))
            z = torch.randn((S_a, k, 2), generator=gen, dtype=torch.float64, device=dev)
            L = self.chol[sel, p]
            cand[:, :, a] = base[:, :, a] + z[:, :, 0] * L[:, None, 0]
            cand[:, :, b] = base[:, :, b] + z[:, :, 0] * L[:, None, 1] + z[:, :, 1] * L[:, None, 2]
        for dd in UNIFORM_DIMS:
            r = torch.rand((S_a, k), generator=gen, dtype=torch.float64, device=dev)
            lo, hi = self.lo_b[sel, dd], self.hi_b[sel, dd]
            cand[:, :, dd] = lo[:, None] + (hi - lo)[:, None] * r
        bd = [0, 1, 2, 4, 5]      # lambda, psi, phi0 are periodic: not bounded by the prior box
        ok = ((cand[:, :, bd] >= self.lo_p[sel][:, None, bd]) & (cand[:, :, bd] <= self.hi_p[sel][:, None, bd])).all(dim=2)
        return cand, ok

    def draw(self, gen, n, backend):
        torch = self.torch
        S = self.chain.shape[0]
        dev = self.u.device
        out = torch.empty((S, n, 8), dtype=torch.float64, device=dev)
        filled = torch.zeros(S, dtype=torch.int64, device=dev)
        for _ in range(200):
            sel = torch.nonzero(filled < n).reshape(-1)
            if len(sel) == 0:
                break
            need = n - filled[sel]
            k = 2 * int(need.max().item()) + 16
            cand, ok = self._candidates(sel, k, gen)
            rank = torch.cumsum(ok.to(torch.int64), dim=1)
            take = ok & (rank <= need[:, None])
            got = take.sum(dim=1)
            # rows of cand that are taken go to out[s, filled[s] + rank - 1]
            s_idx, c_idx = torch.nonzero(take, as_tuple=True)
            dst = filled[sel][s_idx] + rank[s_idx, c_idx] - 1
            out[sel[s_idx], dst] = cand[s_idx, c_idx]
            filled[sel] += got
        # a source whose KDE keeps proposing outside the prior box (its chain pressed against a
        # wall) falls back to proposals uniform in its reduced box for this stage
        fallback = filled < n
        if bool(fallback.any().item()):
            fb = torch.nonzero(fallback).reshape(-1)
            r = torch.rand((len(fb), n, 8), generator=gen, dtype=torch.float64, device=dev)
            out[fb] = self.lo_b[fb][:, None, :] + (self.hi_b[fb] - self.lo_b[fb])[:, None, :] * r
        x = torch.stack([out[:, :, [a, b]] for a, b in KDE_PAIRS], dim=2)                   # [S, n, 3, 2]
        pts = torch.stack([self.pts[:, :, [a, b]] for a, b in KDE_PAIRS], dim=1)            # [S, 3, m, 2]
        wts = self.w[:, None, :].expand(S, len(KDE_PAIRS), self.w.shape[1]).contiguous()
        log_g = backend.kde_logpdf(pts.contiguous(), wts, self.chol.contiguous(), x.contiguous())
        log_g[fallback] = 0.0
        self.fallback = fallback
        return out, log_g


def annealed_posterior_batch(backend, theta_mle: np.ndarray, boxes, seed: int,
                             temps=(15.0, 10.0, 5.0, 3.0, 2.0, 1.0), n: int = 10000, fd_step: float = 1e-9):
    """Algorithm 4 for S sources at once (Algorithm 5 runs it for every recovered source): one
    gb_fisher call gives every source's sigma and reduced box; each temperature draws n
    proposals per source (uniform in the reduced box first, then from the source's pairwise KDE
    of its previous chain), and one gb_mh_step resolves all S chains.  The draws stay on the
    backend's device (a torch generator seeded with ``seed``).  Returns (per-stage list of
    dicts with T, states [S, n, 8], n_accept [S], logL of the states [S, n]; the reduced boxes
    (lo, hi) [S, 8]; sigma [S, 8])."""
    import torch
    theta_mle = np.atleast_2d(np.asarray(theta_mle, dtype=np.float64))
    S = len(theta_mle)
    dev = backend.device
    widths = np.stack([b.width for b in boxes])
    F = backend.fisher(theta_mle, fd_step * widths)
    lo, hi, sigma = np.empty((S, 8)), np.empty((S, 8)), np.empty((S, 8))
    for k in range(S):
        try:
            sg = np.sqrt(np.diag(np.linalg.inv(F[k])))
        except np.linalg.LinAlgError:
            sg = np.full(8, np.nan)
        sigma[k] = sg if np.all(np.isfinite(sg)) else 1e-3 * widths[k]
        lo[k], hi[k] = I.reduced_box(theta_mle[k], boxes[k], sigma[k])
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    lo_t, hi_t = t(lo), t(hi)
    lo_p, hi_p = t(np.stack([b.lo for b in boxes])), t(np.stack([b.hi for b in boxes]))
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed))
    u = lo_t[:, None, :] + (hi_t - lo_t)[:, None, :] * torch.rand((S, n, 8), generator=gen, dtype=torch.float64,
                                                                   device=dev)
    log_g = torch.zeros((S, n), dtype=torch.float64, device=dev)
    stages = []
    for i, T in enumerate(temps):
        props = _from_table1_t(u)
        uni = torch.rand((S, n), generator=gen, dtype=torch.float64, device=dev)
        logL, chain, nacc = backend.mh(props.reshape(S * n, 8), log_g.reshape(-1), uni.reshape(-1), float(T))
        chain = chain.reshape(S, n).long()
        states = torch.gather(props, 1, chain[:, :, None].expand(S, n, 8))
        stages.append({"T": float(T), "states": states, "n_accept": nacc,
                       "logL": torch.gather(logL.reshape(S, n), 1, chain)})
        if i + 1 < len(temps):
            u, log_g = PairKDEBatch(u, chain, lo_p, hi_p, lo_t, hi_t).draw(gen, n, backend)
    return stages, (lo, hi), sigma


class GpuPosteriorBatchBackend:
    """The library calls of annealed_posterior_batch: S sources, each with its own copy of its
    window holding d_posterior = d_residual + s(theta_MLE) (Algorithm 5); gb_fisher over the
    S windows, gb_mh_step with n proposals per window, gb_kde_logpdf with one set per source."""

    def __init__(self, ctx, table, d_residual, w, sources, rows, precision: Optional[int] = None):
        import torch
        from . import api
        self.api, self.torch = api, torch
        self.precision = api.GB_FP64 if precision is None else precision
        self.device = torch.device("cuda")
        self.ctx = ctx
        t = np.asarray(table, dtype=np.int64)
        rows = np.asarray(rows, dtype=np.int64)
        tab = t[rows].copy()
        sizes = tab[:, 3] * tab[:, 1]
        offs = np.concatenate([[0], np.cumsum(sizes)[:-1]])
        gather = np.concatenate([np.arange(t[r, 4], t[r, 4] + sz) for r, sz in zip(rows, sizes)])
        gi = torch.as_tensor(gather, device=self.device)
        self.d = d_residual.index_select(0, gi).contiguous()
        self.w = w.index_select(0, gi).contiguous()
        tab[:, 4] = offs
        tab[:, 5] = offs
        self.tab = tab
        th = torch.as_tensor(np.atleast_2d(np.asarray(sources, dtype=np.float64)), device=self.device)
        api.gb_add_templates(ctx.handle, tab, th, np.arange(len(tab), dtype=np.int32), 1.0, self.d, self.d)
        self.plans = {}

    def fisher(self, theta, steps):
        t = lambda a: self.torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=self.device)
        return self.api.gb_fisher(self.ctx.handle, t(theta), t(steps), self.tab, self.w).cpu().numpy()

    def mh(self, theta, log_g, u, T):
        n = len(theta) // len(self.tab)
        if n not in self.plans:
            tab = self.tab.copy()
            tab[:, 6] = np.arange(len(tab)) * n
            tab[:, 7] = n
            p = self.api.Plan(self.ctx, tab, self.precision)
            p.prepare(self.d, self.w)
            self.plans[n] = p
        return self.plans[n].mh_step(theta.contiguous(), log_g.contiguous(), u.contiguous(), T)

    def kde_logpdf(self, pts, wts, chol, x):
        return self.api.gb_kde_logpdf(pts, wts, chol, x)

    def close(self):
        for p in self.plans.values():
            p.close()
        self.plans = {}


def posterior_batch(ctx, table, T: float, d_residual, w, sources, seg_rows, boxes, seed: int,
                    n: int = 10000, temps=(15.0, 10.0, 5.0, 3.0, 2.0, 1.0), fd_step: float = 1e-9,
                    chunk: int = 256, precision: Optional[int] = None):
    """Algorithm 5's posterior step for every recovered source: ``d_residual`` is the data minus
    all recovered sources (window layout of ``table``), ``seg_rows`` the window of each source;
    the sources run through annealed_posterior_batch ``chunk`` at a time, each on its window
    plus its own template; ``precision`` is the likelihood's (FP64 by default; the Fisher
    matrix always uses FP64 templates).  Returns (final-stage states [n_src, n, 8] (numpy),
    accepted proposals per stage [n_src, n_stages], logL of the final states [n_src, n])."""
    src = np.atleast_2d(np.asarray(sources, dtype=np.float64))
    rows = np.asarray(seg_rows, dtype=np.int64)
    states, accepted, logL = [], [], []
    for c0 in range(0, len(src), chunk):
        sl = slice(c0, min(len(src), c0 + chunk))
        be = GpuPosteriorBatchBackend(ctx, table, d_residual, w, src[sl], rows[sl], precision)
        stages, _, _ = annealed_posterior_batch(be, src[sl], [boxes[r] for r in rows[sl]], seed + c0,
                                                temps=temps, n=n, fd_step=fd_step)
        states.append(stages[-1]["states"].cpu().numpy())
        logL.append(stages[-1]["logL"].cpu().numpy())
        accepted.append(np.stack([s["n_accept"].cpu().numpy() for s in stages], axis=1))
        be.close()
    if not states:
        return np.zeros((0, n, 8)), np.zeros((0, len(temps)), dtype=np.int64), np.zeros((0, n))
    return np.concatenate(states), np.concatenate(accepted), np.concatenate(logL)


def match_delta(ctx, table, T: float, w, recovered, rec_rows, injected, n_near: int = 3) -> np.ndarray:
    """Scaled error of Sec. IV (matching recovered signals), delta = <s_rec - s_inj | s_rec - s_inj> / <s_rec | s_rec>, of every
    recovered source against the ``n_near`` injected sources nearest in frequency, in the
    recovered source's window; returns the smallest delta of each (inf with no injected source),
    the index of the injected source that gives it (-1 with none), and the largest overlap
    O = <s_rec | s_inj> / sqrt(<s_rec | s_rec> <s_inj | s_inj>) over the same candidates (the
    other match metric of Sec. IV; -inf with none).
    One window per (recovered, injected) pair holds the injected template as data, so the
    likelihood kernel's components give delta = -2 logL / <h|h>."""
    import torch
    from . import api
    dev = torch.device("cuda")
    rec = np.atleast_2d(np.asarray(recovered, dtype=np.float64))
    inj = np.atleast_2d(np.asarray(injected, dtype=np.float64))
    if len(rec) == 0 or len(inj) == 0:
        return np.full(len(rec), np.inf), np.full(len(rec), -1, dtype=np.int64), np.full(len(rec), -np.inf)
    t = np.asarray(table, dtype=np.int64)
    order = np.argsort(inj[:, 0])
    f_sorted = inj[order, 0]
    pairs = []
    for k in range(len(rec)):
        c = np.searchsorted(f_sorted, rec[k, 0])
        near = sorted(range(max(0, c - n_near), min(len(inj), c + n_near)),
                      key=lambda j: abs(f_sorted[j] - rec[k, 0]))[:n_near]
        pairs += [(k, int(order[j])) for j in near]
    tab = t[np.asarray(rec_rows)[[k for k, _ in pairs]]].copy()
    sizes = tab[:, 3] * tab[:, 1]
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    gather = np.concatenate([np.arange(t[r, 4], t[r, 4] + s) for r, s in
                             zip(np.asarray(rec_rows)[[k for k, _ in pairs]], sizes)])
    w_p = w.index_select(0, torch.as_tensor(gather, device=dev)).contiguous()
    tab[:, 4] = offs
    tab[:, 5] = offs
    tab[:, 6] = np.arange(len(pairs))
    tab[:, 7] = 1
    d0 = torch.zeros(int(sizes.sum()), dtype=torch.complex128, device=dev)
    d_p = api.gb_add_templates(ctx.handle, tab, torch.as_tensor(inj[[j for _, j in pairs]], device=dev),
                               np.arange(len(pairs), dtype=np.int32), 1.0, d0)
    plan = api.Plan(ctx, tab, api.GB_FP64)
    plan.prepare(d_p, w_p)
    l, c = plan.loglik(torch.as_tensor(rec[[k for k, _ in pairs]], device=dev), comps=True)
    plan.close()
    l, c = l.cpu().numpy(), c.cpu().numpy()
    # <s_inj|s_inj> = -2 logL + 2 <s_inj|s_rec> - <s_rec|s_rec>; a recovered template with no
    # power in its window gives no match (delta not a number)
    ii = -2.0 * l + 2.0 * c[:, 0] - c[:, 1]
    with np.errstate(invalid="ignore", divide="ignore"):
        delta = (-2.0 * l) / c[:, 1]
        ov = c[:, 0] / np.sqrt(c[:, 1] * ii)
    best = np.full(len(rec), np.inf)
    which = np.full(len(rec), -1, dtype=np.int64)
    best_ov = np.full(len(rec), -np.inf)
    for (k, j), dl, o in zip(pairs, delta, ov):
        if dl < best[k]:
            best[k], which[k] = dl, j
        if o > best_ov[k]:
            best_ov[k] = o
    return best, which, best_ov
