"""Plain references for the noise estimates -- TEST INFRASTRUCTURE ONLY.

* periodogram   -- the one-sided PSD estimate of every frequency bin (Sec. III, noise within a
                   frequency segment): the paper's 2 |A(f)|^2 / (N f_sample) of a DFT A of N time
                   samples.  The data here are continuous-transform values d = dt * A and
                   T = N dt, so the same estimate reads 2 |d|^2 / T.
* local_noise   -- the constant noise level of one padded window and channel: the median of the
                   periodogram over the window's bins (the paper takes the median to damp loud
                   signals inside the window).
* local_weights -- the scalar product's weights 4 / (T S) from that level, for every bin.
Only tests/, the smoke check and the benchmark's CPU-baseline leg may use this module.
"""

from __future__ import annotations

import numpy as np


def periodogram(d: np.ndarray, T: float) -> np.ndarray:
    """2 |d_k|^2 / T for every element of d (complex)."""
    d = np.asarray(d, dtype=np.complex128)
    return 2.0 * (d.real * d.real + d.imag * d.imag) / T


def local_noise(block: np.ndarray, T: float) -> np.ndarray:
    """Median over the bins of each channel of a window block [C, W] -> [C]."""
    return np.median(periodogram(block, T), axis=1)


def local_weights(block: np.ndarray, T: float) -> np.ndarray:
    """Weights 4 / (T S_c) of a window block [C, W], constant along each channel."""
    S = local_noise(block, T)
    return np.repeat((4.0 / (T * S))[:, None], block.shape[1], axis=1)
