"""Seeded synthetic inputs shaped like the paper's workloads.

This module is shared by the test oracle and the HIP path, so it holds none of the
method's arithmetic: no waveform, no response, no inner product, no likelihood.  It
provides

* the analytic instrument-noise PSD of the A, E, T channels and the weights
  ``w = 4 / (T S)`` that the discrete inner product uses,
* Gaussian frequency-domain noise drawn from that PSD,
* the Table I prior box and draws in its coordinates (sin beta, log A, cos iota),
* the frequency-derivative formula and the segment widths of Sec. III A together
  with Algorithm 1 (``segmenting``),
* the window layouts and candidate batches of five synthetic workloads.

Injected signals are produced by a caller-supplied ``template_fn`` (the oracle in
tests, the HIP path in the benchmark), so this file never computes one itself.

Parameter order everywhere: (f0, fdot, beta, lambda, amplitude, iota, psi, phi0).
"""

from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Sequence

import numpy as np

# ---------------------------------------------------------------------------------
# constants of the synthetic setting
# ---------------------------------------------------------------------------------
C_LIGHT = 299792458.0            # m/s
AU = 1.495978707e11              # m
ARM_L = 2.5e9                    # m; f*/2 = 1/(4 pi L) = 9.55 mHz (Sec. II, T-channel rule)
YEAR = 31558149.76               # s, sidereal year (orbital period of the guiding centre)
DT = 15.0                        # s, sampling cadence (f_Nyquist = 33.3 mHz, Sec. IV)
T1 = 2 ** 21 * DT                # s, ~1 yr
T2 = 2 ** 22 * DT                # s, ~2 yr
GMSUN_C3 = 4.925490947e-6        # s, G M_sun / c^3
F_STAR = C_LIGHT / (2.0 * math.pi * ARM_L)
F_T_CHANNEL = F_STAR / 2.0       # T channel used at and above this frequency (Sec. II)
SEED_BASE = 20230707

PARAM_NAMES = ("f0", "fdot", "beta", "lam", "amp", "iota", "psi", "phi0")
# coordinates in which Table I states the prior box
TABLE1_NAMES = ("f0", "fdot", "sin_beta", "lam", "log10_amp", "cos_iota", "psi", "phi0")


# ---------------------------------------------------------------------------------
# noise model
# ---------------------------------------------------------------------------------
def keplerian_orbits(t, P_orb: float = YEAR, L: float = ARM_L, AU_: float = AU) -> np.ndarray:
    """Spacecraft positions [3, len(t), 3] (m, ecliptic frame) on exact Keplerian ellipses: the
    orbits whose first-order expansion in the eccentricity is the classic rigid-triangle
    formula (shared mean longitude 2 pi t / P_orb, perihelion longitudes 2 pi i / 3,
    e = L / (2 sqrt3 AU), each orbit plane tilted about the axis perpendicular to its apsides
    by sin eps = sqrt3 e).  Kept to all orders, the arms breathe (about +-0.24% at the default
    sizes) and the centroid leaves the ecliptic (about 9,000 km): an input for the unequal-arm
    model, sampled on a grid by orbit_grid."""
    t = np.asarray(t, dtype=np.float64)
    lam = 2.0 * math.pi * t / P_orb
    e = L / (2.0 * math.sqrt(3.0) * AU_)
    eps = math.asin(math.sqrt(3.0) * e)
    out = np.empty((3,) + t.shape + (3,))
    for i in range(3):
        w = 2.0 * math.pi * i / 3.0
        M = lam - w
        E = M.copy()
        for _ in range(40):                      # Kepler's equation E - e sin E = M (Newton)
            E = E - (E - e * np.sin(E) - M) / (1.0 - e * np.cos(E))
        u = AU_ * (np.cos(E) - e)                # along the apsidal line
        v = AU_ * math.sqrt(1.0 - e * e) * np.sin(E)
        xp, zp = u * math.cos(eps), -u * math.sin(eps)
        out[i, ..., 0] = xp * math.cos(w) - v * math.sin(w)
        out[i, ..., 1] = xp * math.sin(w) + v * math.cos(w)
        out[i, ..., 2] = zp
    return out


def orbit_grid(positions_fn, T: float, n: int = 4097) -> tuple:
    """Positions on the uniform grid t_j = t0 + j dt, j < n, covering [-dt, T + dt] (so that the
    four-point interpolation of the library and of the oracle has a centred stencil at both
    ends): returns (pos [n, 3, 3] as spacecraft, xyz; t0; dt)."""
    dt = T / (n - 3)
    t0 = -dt
    t = t0 + dt * np.arange(n, dtype=np.float64)
    x = positions_fn(t)                          # [3, n, 3]
    return np.ascontiguousarray(np.transpose(x, (1, 0, 2))), t0, dt


def psd_single_link(f):
    """Acceleration and optical-metrology noise in fractional-frequency units.

    Returns (S_acc, S_oms) per link at frequency f (Hz).  Levels 3e-15 m s^-2/sqrt(Hz)
    and 15 pm/sqrt(Hz) with the usual low- and high-frequency reddening.
    """
    f = np.asarray(f, dtype=np.float64)
    s_acc = (3e-15) ** 2 * (1.0 + (0.4e-3 / f) ** 2) * (1.0 + (f / 8e-3) ** 4)
    s_oms = (15e-12) ** 2 * (1.0 + (2e-3 / f) ** 4)
    s_acc_ff = s_acc / (2.0 * math.pi * f * C_LIGHT) ** 2
    s_oms_ff = s_oms * (2.0 * math.pi * f / C_LIGHT) ** 2
    return s_acc_ff, s_oms_ff


def psd_aet(f, arm_length: float = ARM_L, tdi: int = 1):
    """One-sided noise PSDs (S_A = S_E, S_T) of the equal-arm A, E, T of TDI generation 1 or 2.

    Link noises are independent; the A/E/T combinations of Sec. II diagonalise their
    covariance.  With x = 2 pi f L / c, first generation:
      S_A = 8 sin^2 x [(2 + cos x) S_oms + 2 (3 + 2 cos x + cos 2x) S_acc]
      S_T = 32 sin^2 x sin^2(x/2) [S_oms + 4 sin^2(x/2) S_acc]
    The second-generation combinations with equal arms are the first-generation ones minus
    their copy delayed by four arm lengths, which multiplies both PSDs by |1 - e^{-4ix}|^2
    = 4 sin^2(2x).
    """
    f = np.asarray(f, dtype=np.float64)
    s_acc, s_oms = psd_single_link(f)
    x = 2.0 * math.pi * f * arm_length / C_LIGHT
    sx2 = np.sin(x) ** 2
    s_a = 8.0 * sx2 * ((2.0 + np.cos(x)) * s_oms + 2.0 * (3.0 + 2.0 * np.cos(x) + np.cos(2 * x)) * s_acc)
    sh2 = np.sin(x / 2.0) ** 2
    s_t = 32.0 * sx2 * sh2 * (s_oms + 4.0 * sh2 * s_acc)
    if tdi == 2:
        g2 = 4.0 * np.sin(2.0 * x) ** 2
        s_a, s_t = s_a * g2, s_t * g2
    return s_a, s_t


def channel_psd(k0: int, W: int, C: int, T: float, arm_length: float = ARM_L, tdi: int = 1) -> np.ndarray:
    """PSD per channel and window bin, shape [C, W]; bins k0..k0+W-1 at f = k / T."""
    f = (k0 + np.arange(W, dtype=np.float64)) / T
    s_a, s_t = psd_aet(f, arm_length, tdi)
    rows = [s_a, s_a] + ([s_t] if C == 3 else [])
    return np.stack(rows[:C])


def inner_product_weights(psd: np.ndarray, T: float) -> np.ndarray:
    """Weights w = 4 df / S with df = 1/T, the discretised factor of the scalar product."""
    return 4.0 / (T * psd)


def draw_noise(rng: np.random.Generator, psd: np.ndarray, T: float) -> np.ndarray:
    """Gaussian FD noise: Re and Im i.i.d. N(0, T S / 4) per bin and channel."""
    sd = np.sqrt(T * psd / 4.0)
    return sd * rng.standard_normal(psd.shape) + 1j * sd * rng.standard_normal(psd.shape)


def channels_for(f: float) -> int:
    """Paper rule (Sec. II): A, E below f*/2, A, E, T at and above."""
    return 3 if f >= F_T_CHANNEL else 2


# ---------------------------------------------------------------------------------
# frequency derivative, signal widths, segments (Sec. III A)
# ---------------------------------------------------------------------------------
def chirp_mass(m1: float, m2: float) -> float:
    return (m1 * m2) ** 0.6 / (m1 + m2) ** 0.2


def fdot_gr(f, mc_sun):
    """fdot = 96/5 pi^(8/3) (G Mc / c^3)^(5/3) f^(11/3)  (Sec. III A, with G, c restored)."""
    m = np.asarray(mc_sun, dtype=np.float64) * GMSUN_C3
    return 96.0 / 5.0 * math.pi ** (8.0 / 3.0) * m ** (5.0 / 3.0) * np.asarray(f, dtype=np.float64) ** (11.0 / 3.0)


MC_CHANDRASEKHAR = chirp_mass(1.4, 1.4)


def b_max(f, T: float):
    """Broadest expected signal width B_max = B_F + 2 B_O + 2 B_C (Sec. III A)."""
    b_f = fdot_gr(f, MC_CHANDRASEKHAR) * T
    b_o = 1e-4 * np.asarray(f, dtype=np.float64)
    b_c = 4.0 / YEAR
    return b_f + 2.0 * b_o + 2.0 * b_c


def segmenting(f_min: float, f_max: float, T: float, kappa: float = 1.0) -> List[tuple]:
    """Algorithm 1: consecutive segments [f, f + 2 B_max(f)] from f_min until f >= f_max.

    ``kappa`` scales B_max (1 = the paper's rule)."""
    out = []
    f = f_min
    while f < f_max:
        f_next = f + 2.0 * kappa * float(b_max(f, T))
        out.append((f, f_next))
        f = f_next
    return out


def a_of_rho(rho, f, T: float, psd_value):
    """A(rho) = 2 rho (S / (T sin^2(f / f*)))^(1/2)  (Sec. III B)."""
    return 2.0 * rho * np.sqrt(psd_value / (T * np.sin(f / F_STAR) ** 2))


# ---------------------------------------------------------------------------------
# Table I prior box and coordinate changes
# ---------------------------------------------------------------------------------
@dataclasses.dataclass
class PriorBox:
    """Table I bounds in Table I coordinates, arrays of length 8 (TABLE1_NAMES)."""
    lo: np.ndarray
    hi: np.ndarray

    @property
    def width(self) -> np.ndarray:
        return self.hi - self.lo


def table1_box(f_seg_lo: float, f_seg_hi: float, T: float) -> PriorBox:
    """Table I for one segment; f is padded by a quarter of the segment width on each side."""
    pad = (f_seg_hi - f_seg_lo) / 4.0
    f_lo, f_hi = f_seg_lo - pad, f_seg_hi + pad
    fc = 0.5 * (f_seg_lo + f_seg_hi)
    s_a, _ = psd_aet(fc)
    lo = np.array([f_lo, -5e-6 * fc ** (13.0 / 3.0), -1.0, -math.pi,
                   math.log10(a_of_rho(7.0, fc, T, s_a)), -1.0, 0.0, 0.0])
    hi = np.array([f_hi, 1.02e-6 * fc ** (11.0 / 3.0), 1.0, math.pi,
                   math.log10(a_of_rho(1000.0, fc, T, s_a)), 1.0, math.pi, 2.0 * math.pi])
    return PriorBox(lo, hi)


def to_table1(theta: np.ndarray) -> np.ndarray:
    th = np.asarray(theta, dtype=np.float64)
    u = th.copy()
    u[..., 2] = np.sin(th[..., 2])
    u[..., 4] = np.log10(th[..., 4])
    u[..., 5] = np.cos(th[..., 5])
    return u


def from_table1(u: np.ndarray) -> np.ndarray:
    uu = np.asarray(u, dtype=np.float64)
    th = uu.copy()
    th[..., 2] = np.arcsin(np.clip(uu[..., 2], -1.0, 1.0))
    th[..., 4] = 10.0 ** uu[..., 4]
    th[..., 5] = np.arccos(np.clip(uu[..., 5], -1.0, 1.0))
    return th


def draw_uniform_box(rng: np.random.Generator, lo: np.ndarray, hi: np.ndarray, n: int) -> np.ndarray:
    """n points uniform in a box given in Table I coordinates; returned in natural ones."""
    u = lo + (hi - lo) * rng.random((n, 8))
    return from_table1(u)


def draw_gaussian_around(rng: np.random.Generator, theta0: np.ndarray, box: PriorBox,
                         rel_sigma: float, n: int) -> np.ndarray:
    """n Gaussian draws around theta0 in Table I coordinates with sigma = rel_sigma * box width.
    Only the bounded coordinates (sin beta, cos iota in [-1, 1]) are truncated, by redrawing;
    the others may leave the box (an injected source need not lie inside Table I's amplitude
    range, and the angles are periodic)."""
    u0 = to_table1(theta0)
    sig = rel_sigma * box.width
    out = np.empty((n, 8))
    filled = 0
    for _ in range(10000):
        if filled >= n:
            break
        cand = u0 + sig * rng.standard_normal((2 * (n - filled) + 8, 8))
        ok = (np.abs(cand[:, 2]) <= 1.0) & (np.abs(cand[:, 5]) <= 1.0)
        cand = cand[ok][: n - filled]
        out[filled:filled + len(cand)] = cand
        filled += len(cand)
    if filled < n:
        raise ValueError("draw_gaussian_around: centre too far outside the bounded coordinates")
    return from_table1(out)


def random_angles(rng: np.random.Generator, n: int) -> np.ndarray:
    """beta, lambda, iota, psi, phi0 uniform in Table I coordinates; shape [n, 5]."""
    sb = rng.uniform(-1, 1, n)
    lam = rng.uniform(-math.pi, math.pi, n)
    ci = rng.uniform(-1, 1, n)
    psi = rng.uniform(0, math.pi, n)
    phi0 = rng.uniform(0, 2 * math.pi, n)
    return np.stack([np.arcsin(sb), lam, np.arccos(ci), psi, phi0], axis=1)


def make_theta(f0, fdot, amp, angles) -> np.ndarray:
    f0 = np.atleast_1d(np.asarray(f0, dtype=np.float64))
    n = len(f0)
    th = np.empty((n, 8))
    th[:, 0] = f0
    th[:, 1] = fdot
    th[:, 2] = angles[:, 0]
    th[:, 3] = angles[:, 1]
    th[:, 4] = amp
    th[:, 5] = angles[:, 2]
    th[:, 6] = angles[:, 3]
    th[:, 7] = angles[:, 4]
    return th


# ---------------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------------
# template_fn(theta[n, 8], N, C, T) -> (h[n, C, N] complex128, first_bin[n] int64):
# the frequency-domain template on bins first_bin .. first_bin + N - 1.
TemplateFn = Callable[[np.ndarray, int, int, float], tuple]


@dataclasses.dataclass
class WindowSpec:
    k0: int
    W: int
    N: int
    C: int
    f_lo: float                # unpadded segment (or window) edges, Hz
    f_hi: float
    sources: np.ndarray        # injected theta [n_src, 8]
    target: int = 0            # index of the source the candidates are drawn around


@dataclasses.dataclass
class Workload:
    name: str
    T: float
    windows: List[WindowSpec]
    theta: np.ndarray          # [sum n_cand, 8], candidates of all windows, concatenated
    n_cand: np.ndarray         # [n_win]
    cand_off: np.ndarray       # [n_win]
    data: Optional[np.ndarray] = None      # complex128, concatenated [C][W] blocks
    weights: Optional[np.ndarray] = None   # float64, same layout
    data_off: Optional[np.ndarray] = None  # [n_win] offsets (in elements) into data/weights
    psd: Optional[np.ndarray] = None
    tdi: int = 1                           # TDI generation of the data (noise PSD and injections)

    @property
    def n_win(self) -> int:
        return len(self.windows)

    def window_table(self) -> np.ndarray:
        """int64 table [n_win, 8]: k0, W, N, C, data_off, w_off, cand_off, n_cand."""
        t = np.zeros((self.n_win, 8), dtype=np.int64)
        for i, w in enumerate(self.windows):
            t[i] = (w.k0, w.W, w.N, w.C, self.data_off[i], self.data_off[i],
                    self.cand_off[i], self.n_cand[i])
        return t

    def window_data(self, i: int):
        w = self.windows[i]
        o = int(self.data_off[i])
        d = self.data[o:o + w.C * w.W].reshape(w.C, w.W)
        ww = self.weights[o:o + w.C * w.W].reshape(w.C, w.W)
        return d, ww

    def window_theta(self, i: int) -> np.ndarray:
        o = int(self.cand_off[i])
        return self.theta[o:o + int(self.n_cand[i])]

    def window_box(self, i: int) -> "PriorBox":
        """Table I box of window i: the window's bins less W/6 on each side (the padding)."""
        w = self.windows[i]
        return table1_box(w.f_lo + w.W / 6 / self.T, w.f_hi - w.W / 6 / self.T, self.T)


def add_templates(data_cw: np.ndarray, k0: int, h: np.ndarray, first_bin: np.ndarray, sign: float = 1.0):
    """Add templates h[n, C, N] (bins first_bin..) into a window block data_cw[C, W] (bins k0..),
    clipped to the window.  Pure index bookkeeping."""
    C, W = data_cw.shape
    for j in range(h.shape[0]):
        lo = int(first_bin[j])
        N = h.shape[2]
        a = max(lo, k0)
        b = min(lo + N, k0 + W)
        if a < b:
            data_cw[:, a - k0:b - k0] += sign * h[j, :C, a - lo:b - lo]


def finalize_data(wl: Workload, template_fn: Optional[TemplateFn], rng_noise, noise: bool = True,
                  subtract_others: bool = False):
    """Fill data = sum of injections (via template_fn) + PSD noise, and weights."""
    offs = []
    blocks_d, blocks_w, blocks_s = [], [], []
    o = 0
    for w in wl.windows:
        psd = channel_psd(w.k0, w.W, w.C, wl.T, tdi=wl.tdi)
        d = np.zeros((w.C, w.W), dtype=np.complex128)
        if template_fn is not None and len(w.sources):
            srcs = w.sources
            if subtract_others:
                srcs = srcs[w.target:w.target + 1]
            h, fb = template_fn(srcs, w.N, w.C, wl.T)
            add_templates(d, w.k0, h, fb)
        if noise:
            d += draw_noise(rng_noise, psd, wl.T)
        blocks_d.append(d.ravel())
        blocks_w.append(inner_product_weights(psd, wl.T).ravel())
        blocks_s.append(psd.ravel())
        offs.append(o)
        o += w.C * w.W
    wl.data = np.concatenate(blocks_d)
    wl.weights = np.concatenate(blocks_w)
    wl.psd = np.concatenate(blocks_s)
    wl.data_off = np.asarray(offs, dtype=np.int64)
    return wl


def _streams(cfg: int):
    ss = np.random.SeedSequence(SEED_BASE + cfg)
    inj, noise, prop, de = ss.spawn(4)
    return (np.random.default_rng(inj), np.random.default_rng(noise),
            np.random.default_rng(prop), np.random.default_rng(de))


def _concat(wins: List[WindowSpec], thetas: List[np.ndarray], name: str, T: float) -> Workload:
    n_cand = np.array([len(t) for t in thetas], dtype=np.int64)
    cand_off = np.concatenate([[0], np.cumsum(n_cand)[:-1]]).astype(np.int64)
    theta = np.concatenate(thetas) if thetas else np.zeros((0, 8))
    return Workload(name=name, T=T, windows=wins, theta=theta, n_cand=n_cand, cand_off=cand_off)


def workload_c1(template_fn: Optional[TemplateFn], n_cand: int = 1000, noise: bool = True) -> Workload:
    """Plain single window: f0 = 3 mHz, W = 128, N = 128, C = 2, T ~ 1 yr; one injection
    (fdot = 1e-17 Hz/s, A = 1e-22); candidates Gaussian around the truth (1e-4 of the
    Table I widths)."""
    r_inj, r_noise, r_prop, _ = _streams(1)
    T = T1
    f0 = 3.000e-3
    q = int(math.floor(f0 * T))
    ang = random_angles(r_inj, 1)
    src = make_theta([f0], 1e-17, 1e-22, ang)
    w = WindowSpec(k0=q - 64, W=128, N=128, C=2, f_lo=(q - 64) / T, f_hi=(q + 64) / T, sources=src)
    box = table1_box(w.f_lo + (w.f_hi - w.f_lo) / 6, w.f_hi - (w.f_hi - w.f_lo) / 6, T)
    cands = draw_gaussian_around(r_prop, src[0], box, 1e-4, n_cand)
    wl = _concat([w], [cands], "C1 plain FP64: 1 window, 128 bins at 3 mHz, N=128, T=2^21*15 s", T)
    return finalize_data(wl, template_fn, r_noise, noise)


def c2_sources(r_inj) -> tuple:
    T = T2
    qc = int(math.floor(8.0e-3 * T))
    offs = np.array([0.0, 7.3, 18.6])
    f0 = (qc + offs + 0.37) / T
    amp = 10.0 ** r_inj.uniform(-23, -21, 3)
    mc = r_inj.uniform(0.1, 1.0, 3)
    ang = random_angles(r_inj, 3)
    src = make_theta(f0, fdot_gr(f0, mc), amp, ang)
    return qc, src


def workload_c2(template_fn: Optional[TemplateFn], n_cand: int = 10000, noise: bool = True,
                subtract_others: bool = True, sigma: Optional[np.ndarray] = None) -> Workload:
    """Single window of 512 bins at 8 mHz, N = 256, C = 2, T ~ 2 yr, three overlapping
    injections; candidates uniform in the reduced box around source 1 (Sec. III G):
    +-4 sigma, f +-1 sigma, fdot over the full prior, psi +-pi/1000, phi0 +-2pi/1000.
    ``sigma`` (Table I coordinates) comes from a Fisher matrix computed by the caller;
    without it, 1e-3 of the prior widths is used."""
    r_inj, r_noise, r_prop, _ = _streams(2)
    T = T2
    qc, src = c2_sources(r_inj)
    w = WindowSpec(k0=qc - 256, W=512, N=256, C=2, f_lo=(qc - 256) / T, f_hi=(qc + 256) / T,
                   sources=src, target=0)
    box = table1_box(w.f_lo + 512 / 6 / T, w.f_hi - 512 / 6 / T, T)
    lo, hi = reduced_box(src[0], box, sigma)
    cands = draw_uniform_box(r_prop, lo, hi, n_cand)
    wl = _concat([w], [cands], "C2: 1 window, 512 bins at 8 mHz, N=256, T=2^22*15 s, 3 overlapping GBs", T)
    wl.box_lo, wl.box_hi = lo, hi
    return finalize_data(wl, template_fn, r_noise, noise, subtract_others=subtract_others)


def reduced_box(theta_mle: np.ndarray, box: PriorBox, sigma: Optional[np.ndarray]):
    """Theta_reduced of Sec. III G in Table I coordinates, intersected with the prior box.  The
    maximum is first brought into the prior box in its bounded coordinates (an unconstrained
    polish can end just outside it), so that the reduced box is never empty."""
    u = to_table1(theta_mle)
    for i in (0, 1, 2, 4, 5):
        u[i] = min(max(u[i], box.lo[i]), box.hi[i])
    s = sigma if sigma is not None else 1e-3 * box.width
    lo = u - 4 * s
    hi = u + 4 * s
    lo[0], hi[0] = u[0] - s[0], u[0] + s[0]
    lo[1], hi[1] = box.lo[1], box.hi[1]
    lo[6], hi[6] = u[6] - math.pi / 1000, u[6] + math.pi / 1000
    lo[7], hi[7] = u[7] - 2 * math.pi / 1000, u[7] + 2 * math.pi / 1000
    for i in (0, 2, 3, 4, 5):
        lo[i] = max(lo[i], box.lo[i])
        hi[i] = min(hi[i], box.hi[i])
    return lo, hi


def _source_bandwidth_bins(f0, fdot, T):
    return (np.abs(fdot) * T + 2e-4 * f0 + 8.0 / YEAR) * T


def workload_c3(template_fn: Optional[TemplateFn], n_win: int = 256, n_cand: int = 10000,
                noise: bool = True) -> Workload:
    """Ragged batch: windows with f0 log-uniform in 0.3-20 mHz, W = 64 * 2^round(5 s),
    N = 64 * 2^round(3 s), s = log(f0 / 0.3 mHz) / log(20 / 0.3); 1-4 injections per window
    (A log-uniform 1e-23..1e-21, fdot from chirp masses 0.1-1 Msun); C by the paper rule;
    candidates Gaussian around the loudest source (1e-4 of the Table I widths)."""
    r_inj, r_noise, r_prop, _ = _streams(3)
    T = T1
    wins, thetas = [], []
    rejected = 0
    total = 0
    fc_all = np.exp(r_inj.uniform(math.log(0.3e-3), math.log(20e-3), n_win))
    for fc in fc_all:
        s = math.log(fc / 0.3e-3) / math.log(20 / 0.3)
        W = 64 * 2 ** int(round(5 * s))
        N = 64 * 2 ** int(round(3 * s))
        q = int(math.floor(fc * T))
        k0 = q - W // 2
        C = channels_for(fc)
        n_src = int(r_inj.integers(1, 5))
        srcs = []
        while len(srcs) < n_src:
            f0 = (q + r_inj.uniform(-W / 4, W / 4)) / T
            mc = r_inj.uniform(0.1, 1.0)
            fd = float(fdot_gr(f0, mc))
            total += 1
            if _source_bandwidth_bins(f0, fd, T) > N - 16:
                rejected += 1
                continue
            amp = 10.0 ** r_inj.uniform(-23, -21)
            ang = random_angles(r_inj, 1)
            srcs.append(make_theta([f0], fd, amp, ang)[0])
        srcs = np.array(srcs)
        s_a, _ = psd_aet(srcs[:, 0])
        loud = int(np.argmax(srcs[:, 4] / np.sqrt(s_a) * np.abs(np.sin(srcs[:, 0] / F_STAR))))
        w = WindowSpec(k0=k0, W=W, N=N, C=C, f_lo=k0 / T, f_hi=(k0 + W) / T, sources=srcs, target=loud)
        box = table1_box(w.f_lo + W / 6 / T, w.f_hi - W / 6 / T, T)
        wins.append(w)
        thetas.append(draw_gaussian_around(r_prop, srcs[loud], box, 1e-4, n_cand))
    wl = _concat(wins, thetas, f"C3 ragged: {n_win} windows, f0 0.3-20 mHz, W 64-2048, N 64-512, "
                               f"{n_cand} candidates per window, T=2^21*15 s", T)
    wl.rejected = (rejected, total)
    return finalize_data(wl, template_fn, r_noise, noise)


def workload_c4(template_fn: Optional[TemplateFn], n_win: int = 64, n_cand: int = 4096,
                noise: bool = True) -> Workload:
    """Gradient workload: windows with f0 log-uniform in 1-10 mHz, W = 256/512/1024 by band,
    N = 256, C = 2, 1-2 injections, candidates uniform over the Table I box."""
    r_inj, r_noise, r_prop, _ = _streams(4)
    T = T1
    wins, thetas = [], []
    fc_all = np.exp(r_inj.uniform(math.log(1e-3), math.log(10e-3), n_win))
    for fc in fc_all:
        W = 256 if fc < 2.15e-3 else (512 if fc < 4.64e-3 else 1024)
        N = 256
        q = int(math.floor(fc * T))
        k0 = q - W // 2
        n_src = int(r_inj.integers(1, 3))
        srcs = []
        while len(srcs) < n_src:
            f0 = (q + r_inj.uniform(-W / 4, W / 4)) / T
            fd = float(fdot_gr(f0, r_inj.uniform(0.1, 1.0)))
            if _source_bandwidth_bins(f0, fd, T) > N - 16:
                continue
            amp = 10.0 ** r_inj.uniform(-23, -21)
            srcs.append(make_theta([f0], fd, amp, random_angles(r_inj, 1))[0])
        srcs = np.array(srcs)
        w = WindowSpec(k0=k0, W=W, N=N, C=2, f_lo=k0 / T, f_hi=(k0 + W) / T, sources=srcs)
        box = table1_box(w.f_lo + W / 6 / T, w.f_hi - W / 6 / T, T)
        # fdot prior: keep the Table I range; frequencies restricted to the unpadded window
        wins.append(w)
        thetas.append(draw_uniform_box(r_prop, box.lo, box.hi, n_cand))
    wl = _concat(wins, thetas, f"C4 gradient: {n_win} windows, f0 1-10 mHz, W 256-1024, N=256, "
                               f"{n_cand} candidates per window, T=2^21*15 s", T)
    return finalize_data(wl, template_fn, r_noise, noise)


W_MAX = 4096  # the widest padded window (the per-segment median sorts a window's channel in LDS)


def split_wide(segs, T: float, w_max: int = W_MAX) -> List[tuple]:
    """Segments whose padded window (1.5 times the segment) would exceed ``w_max`` bins, cut into
    the fewest equal parts whose windows fit; the others unchanged."""
    out = []
    for fa, fb in segs:
        n = max(1, math.ceil(1.5 * (fb - fa) * T / w_max))
        step = (fb - fa) / n
        out += [(fa + i * step, fa + (i + 1) * step if i + 1 < n else fb) for i in range(n)]
    return out


def workload_c5_windows(n_target: int = 4000, T: float = T2, f_min: float = 0.3e-3,
                        f_max: float = 30e-3) -> tuple:
    """Full-band windows: Algorithm 1 with B_max scaled by kappa, its segments wider than a
    4096-bin padded window allows split into equal parts (split_wide: above about 18 mHz
    Algorithm 1's segments outgrow the window, which would leave their outer bins outside every
    window), kappa chosen by bisection so that ``n_target`` segments result in all; padded
    W = 1.5 x segment, in [64, 4096]."""
    lo_k, hi_k = 0.05, 20.0
    for _ in range(60):
        mid = math.sqrt(lo_k * hi_k)
        n = len(split_wide(segmenting(f_min, f_max, T, mid), T))
        if n > n_target:
            lo_k = mid
        else:
            hi_k = mid
    kappa = hi_k
    # the split makes the count step unevenly with kappa: take the nearest kappa (steps of 1e-4
    # relative) that gives exactly n_target segments, if one is close
    for j in sorted(range(-300, 301), key=abs):
        k = hi_k * (1.0 + 1e-4 * j)
        if len(split_wide(segmenting(f_min, f_max, T, k), T)) == n_target:
            kappa = k
            break
    segs = split_wide(segmenting(f_min, f_max, T, kappa), T)
    return kappa, segs


def nextpow2(x: int) -> int:
    return 1 << max(0, int(math.ceil(math.log2(max(1, x)))))


def workload_c5(template_fn: Optional[TemplateFn], n_target: int = 4000, n_gb: int = 20000, pop: int = 512,
                noise: bool = True, T: float = T2, segments: Optional[tuple] = None) -> Workload:
    """Full band: the windows of Algorithm 1 over 0.3-30 mHz with B_max scaled so that
    ``n_target`` segments result, the widest split to fit (workload_c5_windows); each padded by
    a quarter of its width on both sides (W = 1.5 x segment bins, in [64, 4096]).  ``n_gb`` GBs: f0 log-uniform
    0.3-30 mHz, A log-uniform 1e-23..1e-21, fdot from chirp masses 0.1-1 Msun, sources wider than
    1024 - 16 bins rejected (as C3).  Every GB is injected into every window its band overlaps;
    N = nextpow2(widest overlapping band + 16) clamped to [64, 1024]; C by the paper rule at the
    window centre.  Candidates: a DE population of ``pop`` per window, uniform over the window's
    Table I box.  ``segments`` = (i0, i1) keeps the contiguous segments i0 .. i1-1 only (the GB
    population is the same; the sources overlapping the kept windows are injected)."""
    r_inj, r_noise, r_prop, _ = _streams(5)
    kappa, segs = workload_c5_windows(n_target, T)
    if segments is not None:
        segs = segs[segments[0]:segments[1]]
    f_min, f_max = 0.3e-3, 30e-3
    gbs, bw = [], []
    rejected = 0
    while len(gbs) < n_gb:
        f0 = math.exp(r_inj.uniform(math.log(f_min), math.log(f_max)))
        fd = float(fdot_gr(f0, r_inj.uniform(0.1, 1.0)))
        b = _source_bandwidth_bins(f0, fd, T)
        if b > 1024 - 16:
            rejected += 1
            continue
        amp = 10.0 ** r_inj.uniform(-23, -21)
        gbs.append(make_theta([f0], fd, amp, random_angles(r_inj, 1))[0])
        bw.append(b)
    gbs = np.array(gbs)
    bw = np.array(bw)
    q = np.floor(gbs[:, 0] * T)
    order = np.argsort(q)
    gbs, bw, q = gbs[order], bw[order], q[order]
    lo_bin, hi_bin = q - bw / 2 - 1, q + bw / 2 + 1
    wins, thetas = [], []
    for fa, fb in segs:
        fc = 0.5 * (fa + fb)
        W = int(min(4096, max(64, round(1.5 * (fb - fa) * T))))
        k0 = int(math.floor(fc * T)) - W // 2
        i0 = int(np.searchsorted(hi_bin, k0 - 1024))
        sel = [j for j in range(i0, len(gbs)) if lo_bin[j] < k0 + W and hi_bin[j] >= k0 and q[j] < k0 + W + 1024]
        srcs = gbs[sel] if sel else np.zeros((0, 8))
        widest = float(bw[sel].max()) if sel else 0.0
        N = int(min(1024, max(64, nextpow2(int(math.ceil(widest)) + 16))))
        w = WindowSpec(k0=k0, W=W, N=N, C=channels_for(fc), f_lo=k0 / T, f_hi=(k0 + W) / T, sources=srcs)
        wins.append(w)
        box = table1_box(w.f_lo + W / 6 / T, w.f_hi - W / 6 / T, T)
        thetas.append(draw_uniform_box(r_prop, box.lo, box.hi, pop))
    wl = _concat(wins, thetas, f"C5 full band: {len(wins)} windows 0.3-30 mHz (kappa {kappa:.3f}), "
                               f"{n_gb} GBs, DE population {pop} per window, T=2^22*15 s", T)
    wl.rejected = (rejected, rejected + n_gb)
    wl.kappa = kappa
    wl.segments = np.array(segs)
    wl.population = gbs
    return finalize_data(wl, template_fn, r_noise, noise)
