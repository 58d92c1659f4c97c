"""Pins of the local noise estimate in oracle/noise.py (CPU).

* A hand-computed case: three bins, T = 2 -> periodogram (2, 4, 9), median 4; an even count
  takes the mean of the two middle values.
* The periodogram of PSD noise is unbiased: its mean over 2e5 bins is S within 1.5%.
* Its values are exponentially distributed (two Gaussian components per bin), so the median of
  pure noise is S ln 2 (within 2% at 2e5 bins), and with 5% of the bins made very loud the
  median moves to the 0.5 / 0.95 quantile, -ln(1 - 0.5 / 0.95) S.
* The weights are 4 / (T S) per channel, as the scalar product's with the true PSD.
"""

import math

import numpy as np

from paper_2307_03763_amd import inputs as I


def _noise():
    from oracle import noise
    return noise


def test_hand_case():
    nz = _noise()
    d = np.array([[1 + 1j, 2.0, 3j]])
    assert np.array_equal(nz.periodogram(d, 2.0), np.array([[2.0, 4.0, 9.0]]))
    assert nz.local_noise(d, 2.0)[0] == 4.0
    d4 = np.array([[1 + 1j, 2.0, 3j, 0.5]])       # periodogram (2, 4, 9, 0.25): median (2 + 4) / 2
    assert nz.local_noise(d4, 2.0)[0] == 3.0
    assert np.array_equal(nz.local_weights(d, 2.0), np.full((1, 3), 4.0 / (2.0 * 4.0)))


def test_unbiased_and_median_of_noise():
    nz = _noise()
    rng = np.random.default_rng(5)
    T, S0 = I.T1, 3.0e-40
    n = 200_000
    psd = np.full((2, n), S0)
    d = I.draw_noise(rng, psd, T)
    P = nz.periodogram(d, T)
    assert abs(P.mean() / S0 - 1.0) < 0.015
    med = nz.local_noise(d, T)
    assert np.all(np.abs(med / (S0 * math.log(2.0)) - 1.0) < 0.02)
    w = nz.local_weights(d, T)
    assert np.allclose(w, (4.0 / (T * med))[:, None], rtol=0, atol=0)


def test_median_with_loud_bins():
    nz = _noise()
    rng = np.random.default_rng(6)
    T, S0 = I.T1, 1.0e-40
    n = 200_000
    d = I.draw_noise(rng, np.full((1, n), S0), T)
    loud = rng.choice(n, n // 20, replace=False)
    d[0, loud] *= 1e4
    q = -math.log(1.0 - 0.5 / 0.95)
    assert abs(nz.local_noise(d, T)[0] / (S0 * q) - 1.0) < 0.02
