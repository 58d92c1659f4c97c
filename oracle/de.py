"""Plain reference of one differential-evolution generation -- TEST INFRASTRUCTURE ONLY.

The paper's search step (Sec. III, Algorithm 2) maximises the SNR with differential evolution
(Storn and Price), strategies DE/rand/1/bin and DE/best/1/bin.  Written from that definition,
with every random number given as an input:

* donors       -- for member i, three members a, b, c distinct from i and from each other, each
                  uniform over the members still free: a = floor(u0 (pop - 1)), b = floor(u1
                  (pop - 2)), c = floor(u2 (pop - 3)), each then stepped past the indices
                  already taken, in increasing order;
* trial        -- mutant x_a + F (x_b - x_c) (DE/rand/1), or x_best + F (x_a - x_b) with the
                  window's best member as the base (DE/best/1, SciPy's default strategy; each
                  product and sum rounded on its own), brought
                  back into the window's box (lambda, psi, phi0 wrap around their range, the
                  other coordinates reflect once at a wall and are clipped), then binomial
                  crossover: coordinate k comes from the mutant when u_cross_k < cr or
                  k = floor(u_j 7), else from x_i; and the trial's physical parameters;
* select       -- greedy replacement by rho = <d|h> / sqrt(<h|h>) (not a finite number:
                  -inf), the best rho of each window and the first member holding it.
Coordinates: f0, fdot, sin(beta), lambda, cos(iota), psi, phi0 (Table I without the
amplitude, on which the SNR does not depend).
Only tests/, the smoke check and the benchmark's CPU-baseline leg may use this module.
"""

from __future__ import annotations

import numpy as np

DIM = 7
PERIODIC = (3, 5, 6)   # lambda, psi, phi0 among the seven coordinates


def _pick(u: np.ndarray, n: int) -> np.ndarray:
    return np.clip(np.floor(u * n).astype(np.int64), 0, n - 1)


def donors(u_idx: np.ndarray, pop: int) -> np.ndarray:
    """u_idx [n_win, pop, 3] -> donor indices [n_win, pop, 3]."""
    i = np.broadcast_to(np.arange(pop)[None, :], u_idx.shape[:2])
    a = _pick(u_idx[..., 0], pop - 1)
    a = a + (a >= i)
    b = _pick(u_idx[..., 1], pop - 2)
    lo_ia, hi_ia = np.minimum(i, a), np.maximum(i, a)
    b = b + (b >= lo_ia)
    b = b + (b >= hi_ia)
    taken = np.sort(np.stack([i, a, b], axis=-1), axis=-1)
    c = _pick(u_idx[..., 2], pop - 3)
    for t in range(3):
        c = c + (c >= taken[..., t])
    return np.stack([a, b, c], axis=-1)


def fold(m: np.ndarray, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """Bring mutants [n_win, pop, 7] into the boxes lo, hi [n_win, 7]."""
    out = np.empty_like(m)
    for k in range(DIM):
        v = m[..., k]
        lk, hk = lo[:, k, None], hi[:, k, None]
        if k in PERIODIC:
            wd = hk - lk
            r = np.fmod(v - lk, wd)
            r = np.where((r != 0.0) & ((r < 0.0) != (wd < 0.0)), r + wd, r)
            out[..., k] = lk + r
        else:
            v = np.where(v < lk, 2.0 * lk - v, v)
            v = np.where(v > hk, 2.0 * hk - v, v)
            out[..., k] = np.minimum(np.maximum(v, lk), hk)
    return out


def to_theta(x: np.ndarray, amp: float) -> np.ndarray:
    """Seven searched coordinates -> the eight parameters (amplitude amp)."""
    th = np.empty(x.shape[:-1] + (8,))
    th[..., 0], th[..., 1], th[..., 3] = x[..., 0], x[..., 1], x[..., 3]
    th[..., 2] = np.arcsin(np.clip(x[..., 2], -1.0, 1.0))
    th[..., 4] = amp
    th[..., 5] = np.arccos(np.clip(x[..., 4], -1.0, 1.0))
    th[..., 6], th[..., 7] = x[..., 5], x[..., 6]
    return th


def trial(lo, hi, x, u_idx, u_cross, u_j, F, cr: float, amp: float, base=None):
    """One DE/rand/1/bin trial per member (DE/best/1/bin with base [n_win], the index of each
    window's best member).  Returns (trial_x [n_win, pop, 7], trial_theta [n_win * pop, 8])."""
    n_win, pop, _ = x.shape
    d = donors(u_idx, pop)
    w = np.arange(n_win)[:, None]
    if base is None:
        xa, xb, xc = x[w, d[..., 0]], x[w, d[..., 1]], x[w, d[..., 2]]
    else:
        xa = np.broadcast_to(x[np.arange(n_win), np.asarray(base)][:, None, :], x.shape)
        xb, xc = x[w, d[..., 0]], x[w, d[..., 1]]
    diff = xb - xc
    step = np.asarray(F)[:, None, None] * diff
    m = fold(xa + step, lo, hi)
    take = (u_cross < cr) | (np.arange(DIM)[None, None, :] == _pick(u_j, DIM)[..., None])
    tx = np.where(take, m, x)
    return tx, to_theta(tx, amp).reshape(n_win * pop, 8)


def rho_of(comps: np.ndarray) -> np.ndarray:
    with np.errstate(invalid="ignore", divide="ignore"):
        r = comps[..., 0] / np.sqrt(comps[..., 1])
    return np.where(np.isfinite(r), r, -np.inf)


def select(comps, x, s, trial_x):
    """Greedy selection; returns new (x, s, best [n_win], index of the first best member)."""
    n_win, pop, _ = x.shape
    r = rho_of(np.asarray(comps).reshape(n_win, pop, 2))
    better = r > s
    x2 = np.where(better[..., None], trial_x, x)
    s2 = np.where(better, r, s)
    return x2, s2, s2.max(axis=1), np.argmax(s2, axis=1)
