"""Pins of the differential-evolution reference in oracle/de.py (CPU).

* Donors: distinct and different from the member for every uniform; for a population of four
  they are exactly the three others; swept over an even grid of uniforms each free index comes
  up equally often (a over the pop - 1 others, b over the pop - 2 left given a, c over the
  pop - 3 left given a and b), i.e. the mapping is uniform.
* Folding: reflection at either wall, wrapping of periodic coordinates, points inside kept.
* Crossover: with cr = 0 exactly the forced coordinate comes from the mutant; with cr = 1 all;
  F = 0 makes the mutant the first donor.
* Selection: strictly larger rho replaces; NaN never does; best is the maximum, held first by
  the reported member.
* The whole step maximises a known function: rho = -|x - x*|^2 (fed in as comps = (rho, 1))
  reaches x* from a uniform start, with DE/rand/1 and with DE/best/1.
"""

import numpy as np


def _de():
    from oracle import de
    return de


def test_donors_distinct_and_pop4():
    de = _de()
    rng = np.random.default_rng(1)
    for pop in (4, 5, 17, 512):
        u = rng.random((3, pop, 3))
        u[0, :, :] = 0.0
        u[1, :, :] = np.nextafter(1.0, 0.0)
        d = de.donors(u, pop)
        i = np.arange(pop)[None, :]
        assert np.all((d >= 0) & (d < pop))
        assert np.all((d[..., 0] != i) & (d[..., 1] != i) & (d[..., 2] != i))
        assert np.all((d[..., 0] != d[..., 1]) & (d[..., 0] != d[..., 2]) & (d[..., 1] != d[..., 2]))
        if pop == 4:
            assert np.all(np.sort(d, axis=-1) == np.array([[sorted(set(range(4)) - {k}) for k in range(4)]]))


def test_donor_mapping_is_uniform():
    de = _de()
    pop, m = 10, 7
    i = 3
    # a: an even grid over [0, 1) hits each of the 9 others m times
    g = (np.arange((pop - 1) * m) + 0.5) / ((pop - 1) * m)
    u = np.zeros((1, pop, 3))
    counts = np.zeros(pop, dtype=int)
    for v in g:
        u[0, i, 0] = v
        counts[de.donors(u, pop)[0, i, 0]] += 1
    assert counts[i] == 0 and np.all(np.delete(counts, i) == m)
    # b given a; c given a and b
    u[0, i, 0] = 0.05                     # a = 0
    a = de.donors(u, pop)[0, i, 0]
    g = (np.arange((pop - 2) * m) + 0.5) / ((pop - 2) * m)
    counts[:] = 0
    for v in g:
        u[0, i, 1] = v
        counts[de.donors(u, pop)[0, i, 1]] += 1
    assert counts[i] == 0 and counts[a] == 0 and np.all(np.delete(counts, [i, a]) == m)
    u[0, i, 1] = 0.999                    # b = the largest free index
    b = de.donors(u, pop)[0, i, 1]
    g = (np.arange((pop - 3) * m) + 0.5) / ((pop - 3) * m)
    counts[:] = 0
    for v in g:
        u[0, i, 2] = v
        counts[de.donors(u, pop)[0, i, 2]] += 1
    assert counts[i] == counts[a] == counts[b] == 0 and np.all(np.delete(counts, [i, a, b]) == m)


def test_fold():
    de = _de()
    lo = np.array([[0.0, -1.0, -1.0, 0.0, -1.0, 0.0, 0.0]])
    hi = np.array([[1.0, 1.0, 1.0, 2 * np.pi, 1.0, np.pi, 2 * np.pi]])
    m = np.array([[[-0.25, 1.5, 0.3, -0.5, 0.99, np.pi + 0.5, 4 * np.pi + 1.0]]])
    f = de.fold(m, lo, hi)[0, 0]
    assert f[0] == 0.25 and f[1] == 0.5 and f[2] == 0.3 and f[4] == 0.99
    assert abs(f[3] - (2 * np.pi - 0.5)) < 1e-15 and abs(f[5] - 0.5) < 1e-15 and abs(f[6] - 1.0) < 1e-14
    # far outside: reflected at the first wall (and then at the other if still beyond it), then
    # clipped: -5 in [0, 1] -> 5 -> -3 -> 0; 7 in [-1, 1] -> -5 -> -1
    m2 = np.array([[[-5.0, 7.0, 0.0, 0.0, 0.0, 0.0, 0.0]]])
    f2 = de.fold(m2, lo, hi)[0, 0]
    assert f2[0] == 0.0 and f2[1] == -1.0


def test_crossover_and_F():
    de = _de()
    rng = np.random.default_rng(2)
    n_win, pop = 2, 9
    lo, hi = np.full((n_win, 7), -10.0), np.full((n_win, 7), 10.0)
    x = rng.uniform(-1, 1, (n_win, pop, 7))
    u_idx, u_cross, u_j = rng.random((n_win, pop, 3)), rng.random((n_win, pop, 7)), rng.random((n_win, pop))
    F = np.array([0.7, 0.7])
    t0, _ = de.trial(lo, hi, x, u_idx, u_cross, u_j, F, 0.0, 1e-22)
    jr = np.floor(u_j * 7).astype(int)
    diff = t0 != x
    assert np.all(diff.sum(axis=-1) <= 1)
    assert np.all(~diff | (np.arange(7)[None, None, :] == jr[..., None]))
    t1, th = de.trial(lo, hi, x, u_idx, u_cross, u_j, np.zeros(2), 1.0, 1e-22)
    d = de.donors(u_idx, pop)
    xa = x[np.arange(n_win)[:, None], d[..., 0]]
    flat = [0, 1, 2, 4]                     # periodic coordinates pass through l + (v - l): rounding
    assert np.array_equal(t1[..., flat], xa[..., flat])
    assert np.allclose(t1, xa, rtol=0, atol=1e-14)
    assert th.shape == (n_win * pop, 8) and np.all(th[:, 4] == 1e-22)


def test_select():
    de = _de()
    x = np.zeros((1, 4, 7))
    tx = np.ones((1, 4, 7))
    s = np.array([[1.0, 1.0, 1.0, -np.inf]])
    comps = np.array([[2.0, 1.0], [1.0, 1.0], [np.nan, 1.0], [1.0, 0.0]])   # rho 2, 1 (tie), NaN, inf
    x2, s2, best, bi = de.select(comps, x, s, tx)
    assert np.array_equal(s2, np.array([[2.0, 1.0, 1.0, -np.inf]]))
    assert np.all(x2[0, 0] == 1.0) and np.all(x2[0, 1:] == 0.0)
    assert best[0] == 2.0 and bi[0] == 0
    # ties: the first member holding the best value
    _, _, _, bi = de.select(np.array([[0.0, 1.0]] * 4), np.zeros((1, 4, 7)), np.array([[1.0, 3.0, 3.0, 0.0]]),
                            np.ones((1, 4, 7)))
    assert bi[0] == 1


def test_de_maximises_known_function():
    de = _de()
    rng = np.random.default_rng(3)
    n_win, pop = 3, 40
    lo, hi = np.full((n_win, 7), -1.0), np.full((n_win, 7), 1.0)
    lo[:, [3, 5, 6]], hi[:, [3, 5, 6]] = 0.0, 2 * np.pi
    target = rng.uniform(-0.8, 0.8, (n_win, 7))
    target[:, [3, 5, 6]] = rng.uniform(0.5, 5.5, (n_win, 3))
    x = lo[:, None, :] + (hi - lo)[:, None, :] * rng.random((n_win, pop, 7))

    def comps_of(xx):
        r = -np.sum((xx - target[:, None, :]) ** 2, axis=-1)
        return np.stack([r.ravel(), np.ones(r.size)], axis=1)

    x0 = x
    for strategy in ("rand1", "best1"):
        x = x0.copy()
        s = np.full((n_win, pop), -np.inf)
        x, s, best, bi = de.select(comps_of(x), x, s, x)
        for _ in range(300):
            tx, _ = de.trial(lo, hi, x, rng.random((n_win, pop, 3)), rng.random((n_win, pop, 7)),
                             rng.random((n_win, pop)), np.full(n_win, rng.uniform(0.5, 1.0)), 0.7, 1e-22,
                             base=bi if strategy == "best1" else None)
            x, s, best, bi = de.select(comps_of(tx), x, s, tx)
        top = x[np.arange(n_win), bi]
        assert np.max(np.abs(top - target)) < 1e-3 and np.all(best > -1e-6), strategy
