"""Plain reference of the global noise estimate -- TEST INFRASTRUCTURE ONLY.

Sec. III F (global noise estimate) and Sec. III G (partial residual): from a residual
d_residual = d - sum s(theta) (or the partial residual d - s_partial sum s(theta)), per channel

  1. the residual as a time series: the one-sided spectrum of the band, assembled from the
     frequency segments (each bin from the segment that owns it; zero outside every segment),
     transformed back with the inverse of the Fourier convention x~_k = dt sum_n x_n e^{-2 pi i k n / M}:
     x_n = (1 / T) sum_k x~_k e^{2 pi i k n / M} over the Hermitian extension, T = M dt;
  2. Welch's method with Hann windows: segments of L samples, 50% overlap, K = 2 M / L - 1 of them
     (511 for L = 2^14 at M = 2^22: the paper's "500 windows"), periodic Hann window
     w_n = 1/2 - 1/2 cos(2 pi n / L), the one-sided density
     P_j = 2 dt / (sum_n w_n^2) * mean_s |sum_n w_n x_{a_s + n} e^{-2 pi i j n / L}|^2
     (DC and the Nyquist bin not doubled), at f_j = j / (L dt);
  3. the median clip: windows of 30 Welch bins shifted by 15, in order, each on the values the
     previous ones left; in each, values above twice the window's median are set to twice the
     median (the reading of the paper's "values above the window's median ... twice the median");
  4. a Savitzky-Golay filter of order 1, window length 10 below 0.8 mHz and 70 above (T of 1 or
     2 years);
  5. a cubic spline through the smoothed curve, evaluated at every bin where an estimate is
     wanted.
Steps 3-5 run over the channel's band only: the Welch bins whose frequency lies inside the
segments that hold the channel (outside it the assembled spectrum is zero, and smoothing across
its edge would mix those zeros in).  Outside the band the spline is held at its end values.

Each step is written out plainly; library routines serve only as the FFT (numpy.fft) and the
median (numpy.median).  Only tests/, the smoke check and the benchmark's CPU-baseline leg may use
this module.
"""

from __future__ import annotations

import math

import numpy as np


# ------------------------------------------------------------------ 1. time series
def assemble(d: np.ndarray, seg, windows, data_off, M: int, c: int) -> np.ndarray:
    """One-sided spectrum [M/2 + 1] of channel c: bin k of segment i (seg[i] = [lo, hi) absolute
    bins) taken from window i's data block (k0, W, C); zero where no segment with channel c is."""
    X = np.zeros(M // 2 + 1, dtype=np.complex128)
    for i, (k0, W, C) in enumerate(windows):
        if c >= C:
            continue
        lo, hi = int(seg[i][0]), int(seg[i][1])
        block = d[int(data_off[i]) + c * W: int(data_off[i]) + (c + 1) * W]
        X[lo:hi] = block[lo - k0:hi - k0]
    return X


def time_series(X: np.ndarray, M: int, dt: float) -> np.ndarray:
    """x_n = (1/T) sum_k x~_k e^{2 pi i k n/M} over the Hermitian extension of the one-sided X."""
    return np.fft.irfft(X, n=M) / dt   # irfft carries the 1/M; 1/T = 1/(M dt)


# ------------------------------------------------------------------ 2. Welch
def hann(L: int) -> np.ndarray:
    n = np.arange(L, dtype=np.float64)
    return 0.5 - 0.5 * np.cos(2.0 * math.pi * n / L)


def welch(x: np.ndarray, dt: float, L: int):
    """Welch's one-sided PSD density of x with periodic Hann windows of L samples and 50%
    overlap: returns (f [L/2 + 1], P [L/2 + 1])."""
    M = len(x)
    w = hann(L)
    K = 2 * M // L - 1
    acc = np.zeros(L // 2 + 1)
    for s in range(K):
        seg = x[s * (L // 2): s * (L // 2) + L] * w
        Y = np.fft.rfft(seg)
        acc += Y.real ** 2 + Y.imag ** 2
    P = acc / K * (2.0 * dt / np.sum(w * w))
    P[0] *= 0.5
    P[-1] *= 0.5
    f = np.arange(L // 2 + 1) / (L * dt)
    return f, P


# ------------------------------------------------------------------ 3. median clip
def median_clip(P: np.ndarray, width: int = 30, stride: int = 15) -> np.ndarray:
    """Windows [s, s + width) for s = 0, stride, 2 stride, ... while s < len(P) (the last ones cut
    at the end), in order: values above twice the window's median become twice the median."""
    out = np.array(P, dtype=np.float64, copy=True)
    for s in range(0, len(out), stride):
        win = out[s:s + width]
        m = float(np.median(win))
        win[win > 2.0 * m] = 2.0 * m
    return out


# ------------------------------------------------------------------ 4. Savitzky-Golay, order 1
def savgol1(y: np.ndarray, wl: int) -> np.ndarray:
    """Least-squares line over each window of wl points, evaluated at the window's output point.
    Interior point i: the window y[i - (wl-1)//2 .. i + wl//2], where the line's value at i is the
    window mean (the positions are symmetric about i for odd wl; for even wl the output point is
    the lower of the two middle ones, and the line's value there is still the mean because its
    uniform weights come out of the fit for that position).  The first and last wl//2 outputs
    come from the line fitted to the first and last wl points, evaluated at their own positions."""
    y = np.asarray(y, dtype=np.float64)
    n = len(y)
    if n < wl:
        raise ValueError("fewer points than the filter window")
    h = wl // 2
    out = np.empty(n)
    for i in range(h, n - h):
        out[i] = np.mean(y[i - (wl - 1) // 2: i + wl // 2 + 1])
    pos = np.arange(wl, dtype=np.float64)

    def line(seg):
        pm = pos.mean()
        slope = np.sum((pos - pm) * (seg - seg.mean())) / np.sum((pos - pm) ** 2)
        return seg.mean() + slope * (pos - pm)

    out[:h] = line(y[:wl])[:h]
    out[n - h:] = line(y[n - wl:])[wl - h:]
    return out


def smooth(f: np.ndarray, P: np.ndarray, f_switch: float = 0.8e-3, wl_short: int = 10, wl_long: int = 70):
    """The two-length Savitzky-Golay of the paper: wl_short below f_switch, wl_long above (each
    filter runs over the whole array; the output takes from each its own frequency range)."""
    a = savgol1(P, wl_short)
    b = savgol1(P, wl_long)
    return np.where(f < f_switch, a, b)


# ------------------------------------------------------------------ 5. cubic spline
def natural_spline(y: np.ndarray) -> np.ndarray:
    """Second derivatives m of the natural cubic spline through (j, y_j), j = 0..n-1 (unit
    spacing): m_{j-1} + 4 m_j + m_{j+1} = 6 (y_{j+1} - 2 y_j + y_{j-1}), m_0 = m_{n-1} = 0,
    solved by forward elimination and back substitution (Thomas)."""
    y = np.asarray(y, dtype=np.float64)
    n = len(y)
    m = np.zeros(n)
    if n < 3:
        return m
    k = n - 2
    rhs = 6.0 * (y[2:] - 2.0 * y[1:-1] + y[:-2])
    diag = np.full(k, 4.0)
    for i in range(1, k):
        r = 1.0 / diag[i - 1]
        diag[i] -= r
        rhs[i] -= r * rhs[i - 1]
    sol = np.zeros(k)
    sol[-1] = rhs[-1] / diag[-1]
    for i in range(k - 2, -1, -1):
        sol[i] = (rhs[i] - sol[i + 1]) / diag[i]
    m[1:-1] = sol
    return m


def spline_eval(y: np.ndarray, m: np.ndarray, t: np.ndarray) -> np.ndarray:
    """The spline at positions t (in units of the grid), held at its end values outside
    [0, n-1]."""
    n = len(y)
    t = np.clip(np.asarray(t, dtype=np.float64), 0.0, n - 1.0)
    i = np.minimum(np.floor(t).astype(np.int64), n - 2)
    u = t - i
    v = 1.0 - u
    return v * y[i] + u * y[i + 1] + ((v ** 3 - v) * m[i] + (u ** 3 - u) * m[i + 1]) / 6.0


# ------------------------------------------------------------------ the whole estimate
def band(seg, windows, c: int):
    """[lo, hi) absolute bins spanned by the segments whose windows hold channel c."""
    idx = [i for i, (_, _, C) in enumerate(windows) if c < C]
    if not idx:
        return None
    return min(int(seg[i][0]) for i in idx), max(int(seg[i][1]) for i in idx)


def global_noise(d: np.ndarray, seg, windows, data_off, T: float, dt: float, L: int = 1 << 14,
                 width: int = 30, stride: int = 15, f_switch: float = 0.8e-3, wl_short: int = 10,
                 wl_long: int = 70, clip: bool = True):
    """The noise PSD at every bin of every window (the layout of the data), from the residual d.
    Returns (S like d's real layout, per-channel Welch P [3][L/2+1], per-channel smoothed curve
    [3][L/2+1] with zeros outside the band).  clip=False leaves the median clip out (to measure
    what it does)."""
    M = int(round(T / dt))
    S = np.zeros(len(d))
    welch_all = np.zeros((3, L // 2 + 1))
    smooth_all = np.zeros((3, L // 2 + 1))
    for c in range(3):
        b = band(seg, windows, c)
        if b is None:
            continue
        x = time_series(assemble(d, seg, windows, data_off, M, c), M, dt)
        f, P = welch(x, dt, L)
        welch_all[c] = P
        # Welch bins inside the band: j L / M in [lo, hi - 1] fine bins
        j_lo = -(-b[0] * L // M)
        j_hi = ((b[1] - 1) * L) // M
        Pc = median_clip(P[j_lo:j_hi + 1], width, stride) if clip else P[j_lo:j_hi + 1]
        Sc = smooth(f[j_lo:j_hi + 1], Pc, f_switch, wl_short, wl_long)
        smooth_all[c, j_lo:j_hi + 1] = Sc
        m = natural_spline(Sc)
        for i, (k0, W, C) in enumerate(windows):
            if c >= C:
                continue
            k = k0 + np.arange(W)
            o = int(data_off[i]) + c * W
            S[o:o + W] = spline_eval(Sc, m, k * L / M - j_lo)
    return S, welch_all, smooth_all


def weights(S: np.ndarray, T: float) -> np.ndarray:
    """The scalar product's weights 4 / (T S) from a noise estimate."""
    return 4.0 / (T * S)
