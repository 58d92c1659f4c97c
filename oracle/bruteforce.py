"""Brute-force time-domain TDI (test infrastructure): the definition the fast/slow model approximates.
First- and second-generation Michelson combinations, with equal arms (the analytic orbits) or
with one light time per arm (any positions, tdi_xyz_positions).

For tiny cases (M <= 2^18 samples) the TDI X, Y, Z are evaluated at every sample time
directly from the plane-wave field, with every retardation and delay taken exactly, and
then transformed with a full-length FFT: x~_k = dt * sum_n x_n e^{-2 pi i k n / M}.
Nothing here uses the slow series, the N-point DFT or the sinc form of the oracle, and the
orbits come from the classic first-order heliocentric formula rather than the rigid-triangle
construction used there.  This module is the independent pin of the oracle's model.

Geometry modes
  G1 -- every position and arm vector is taken at the TDI output time t (also inside the
        delayed terms); only the wave's time arguments are retarded.  This is the
        approximation the fast/slow form makes, so it must agree to rounding when the slow
        series is exactly band-limited (periodic orbit, fdot = 0, integer f0 T).
  G2 -- emitter position at the emission time, receiver position at the reception time,
        each delayed term with its own geometry.  Measures the frozen-arm approximation.
"""

from __future__ import annotations

import math

import numpy as np

C_LIGHT = 299792458.0


def orbits(t, P_orb, L, AU):
    """Spacecraft positions, shape [3, len(t), 3] (m): first-order eccentric heliocentric orbits
    x_i = R cos a + e R/2 (cos(2a - b_i) - 3 cos b_i), y_i = R sin a + e R/2 (sin(2a - b_i) - 3 sin b_i),
    z_i = -sqrt3 e R cos(a - b_i), with e = L / (2 sqrt3 R), a = 2 pi t / P, b_i = 2 pi i / 3."""
    t = np.asarray(t, dtype=np.float64)
    a = 2.0 * math.pi * t / P_orb
    e = L / (2.0 * math.sqrt(3.0) * AU)
    out = np.empty((3,) + t.shape + (3,))
    for i in range(3):
        b = 2.0 * math.pi * i / 3.0
        out[i, ..., 0] = AU * np.cos(a) + 0.5 * e * AU * (np.cos(2 * a - b) - 3.0 * math.cos(b))
        out[i, ..., 1] = AU * np.sin(a) + 0.5 * e * AU * (np.sin(2 * a - b) - 3.0 * math.sin(b))
        out[i, ..., 2] = -math.sqrt(3.0) * e * AU * np.cos(a - b)
    return out


def polarisation(theta):
    """Propagation direction k and the psi-rotated tensors e+, ex (3x3) of one source."""
    f0, fdot, beta, lam, amp, iota, psi, phi0 = [float(x) for x in theta]
    k = -np.array([math.cos(beta) * math.cos(lam), math.cos(beta) * math.sin(lam), math.sin(beta)])
    u = np.array([math.sin(beta) * math.cos(lam), math.sin(beta) * math.sin(lam), -math.cos(beta)])
    v = np.array([math.sin(lam), -math.cos(lam), 0.0])
    ep0 = np.outer(u, u) - np.outer(v, v)
    ec0 = np.outer(u, v) + np.outer(v, u)
    ep = math.cos(2 * psi) * ep0 + math.sin(2 * psi) * ec0
    ec = -math.sin(2 * psi) * ep0 + math.cos(2 * psi) * ec0
    ap = amp * (1.0 + math.cos(iota) ** 2)
    ac = -2.0 * amp * math.cos(iota)
    return k, ep, ec, ap, ac


def _phase(theta, tau):
    """Phi(tau) = 2 pi f0 tau + pi fdot tau^2 + phi0, reduced in cycles before the 2 pi."""
    f0, fdot, phi0 = float(theta[0]), float(theta[1]), float(theta[7])
    cyc = f0 * tau + 0.5 * fdot * tau * tau
    cyc = cyc - np.round(cyc)
    return 2.0 * math.pi * cyc + phi0


def _nHn(theta, pol, n, tau):
    """n . H(tau) . n for arm unit vectors n [..., 3] and times tau [...]:
    H = A+ cos(Phi) e+ + Ax sin(Phi) ex."""
    k, ep, ec, ap, ac = pol
    fp = np.einsum("...i,ij,...j->...", n, ep, n)
    fc = np.einsum("...i,ij,...j->...", n, ec, n)
    ph = _phase(theta, tau)
    return ap * np.cos(ph) * fp + ac * np.sin(ph) * fc


def link(theta, pol, t, r, s, delay, P_orb, L, AU, mode="G1"):
    """y_rs(t - delay L/c): light emitted at s, received at r (0-based spacecraft indices).
    y = [n.H(t_emit - k.x_s/c).n - n.H(t_recv - k.x_r/c).n] / (2 (1 - k.n)), n = (x_r - x_s)/|.|."""
    k = pol[0]
    t_recv = t - delay * L / C_LIGHT
    t_emit = t_recv - L / C_LIGHT
    if mode == "G1":
        x = orbits(t, P_orb, L, AU)
        xr, xs = x[r], x[s]
    else:
        xr = orbits(t_recv, P_orb, L, AU)[r]
        xs = orbits(t_emit, P_orb, L, AU)[s]
    sep = xr - xs
    n = sep / np.linalg.norm(sep, axis=-1, keepdims=True)
    kn = n @ k
    h_emit = _nHn(theta, pol, n, t_emit - (xs @ k) / C_LIGHT)
    h_recv = _nHn(theta, pol, n, t_recv - (xr @ k) / C_LIGHT)
    return (h_emit - h_recv) / (2.0 * (1.0 - kn))


def tdi_xyz(theta, t, P_orb, L, AU, mode="G1", generation=1):
    """Equal-arm Michelson X, Y, Z at times t (arrays), Y and Z by the cyclic relabelling
    1 -> 2 -> 3 -> 1.  First generation (eight links):
      X1 = y13 + y31(t-L) + y12(t-2L) + y21(t-3L) - y12 - y21(t-L) - y13(t-2L) - y31(t-3L).
    Second generation (sixteen links; every delay operator is one arm length here):
      X2 = y13 + y31(t-L) + y12(t-2L) + y21(t-3L) + y12(t-4L) + y21(t-5L) + y13(t-6L) + y31(t-7L)
         - y12 - y21(t-L) - y13(t-2L) - y31(t-3L) - y13(t-4L) - y31(t-5L) - y12(t-6L) - y21(t-7L)."""
    pol = polarisation(theta)

    def y(r, s, j):
        return link(theta, pol, t, r - 1, s - 1, j, P_orb, L, AU, mode)

    def michelson(a, b, c):
        x = (y(a, c, 0) + y(c, a, 1) + y(a, b, 2) + y(b, a, 3)
             - y(a, b, 0) - y(b, a, 1) - y(a, c, 2) - y(c, a, 3))
        if generation == 2:
            x = x + (y(a, b, 4) + y(b, a, 5) + y(a, c, 6) + y(c, a, 7)
                     - y(a, c, 4) - y(c, a, 5) - y(a, b, 6) - y(b, a, 7))
        return x

    X = michelson(1, 2, 3)
    Y = michelson(2, 3, 1)
    Z = michelson(3, 1, 2)
    return X, Y, Z


def tdi_xyz_positions(theta, t, positions, generation=1):
    """Michelson X, Y, Z with one light time per arm, G1 geometry: every position, arm vector
    and arm length at the output time t, from positions(t) -> [3, len(t), 3] (m); only the
    wave's time arguments are retarded, each link by its own light time L_rs(t)/c.  With
    Lc = arm 12 and Lb = arm 31 (light times at t):
      X1 = y13 + y31(t-Lb) + y12(t-2Lb) + y21(t-2Lb-Lc) - y12 - y21(t-Lc) - y13(t-2Lc) - y31(t-2Lc-Lb),
      X2 = X1(t) - X1(t - 2Lb - 2Lc)  (the frozen arms' delays commute),
    Y and Z by the cyclic relabelling 1 -> 2 -> 3 -> 1."""
    pol = polarisation(theta)
    k = pol[0]
    t = np.asarray(t, dtype=np.float64)
    x = positions(t)

    def light(r, s):
        return np.linalg.norm(x[r] - x[s], axis=-1) / C_LIGHT

    def y(r, s, tau):
        sep = x[r] - x[s]
        lrs = np.linalg.norm(sep, axis=-1)
        n = sep / lrs[..., None]
        kn = n @ k
        t_recv = t - tau
        t_emit = t_recv - lrs / C_LIGHT
        h_emit = _nHn(theta, pol, n, t_emit - (x[s] @ k) / C_LIGHT)
        h_recv = _nHn(theta, pol, n, t_recv - (x[r] @ k) / C_LIGHT)
        return (h_emit - h_recv) / (2.0 * (1.0 - kn))

    def michelson(a, b, c, extra):
        lab, lac = light(a, b), light(a, c)
        return (y(a, c, extra) + y(c, a, extra + lac) + y(a, b, extra + 2 * lac) + y(b, a, extra + 2 * lac + lab)
                - y(a, b, extra) - y(b, a, extra + lab) - y(a, c, extra + 2 * lab) - y(c, a, extra + 2 * lab + lac))

    out = []
    for a, b, c in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
        X = michelson(a, b, c, np.zeros_like(t))
        if generation == 2:
            X = X - michelson(a, b, c, 2.0 * (light(a, b) + light(a, c)))
        out.append(X)
    return tuple(out)


def spectrum_positions(theta, M, dt, positions, chunk=1 << 15, generation=1):
    """Full-length spectra of A, E, T (as spectrum) for the unequal-arm Michelson combinations of
    tdi_xyz_positions."""
    series = np.empty((3, M))
    for a in range(0, M, chunk):
        t = dt * np.arange(a, min(M, a + chunk), dtype=np.float64)
        X, Y, Z = tdi_xyz_positions(theta, t, positions, generation)
        series[0, a:a + len(t)] = (Z - X) / math.sqrt(2.0)
        series[1, a:a + len(t)] = (X - 2.0 * Y + Z) / math.sqrt(6.0)
        series[2, a:a + len(t)] = (X + Y + Z) / math.sqrt(3.0)
    return dt * np.fft.fft(series, axis=1), series


def tdi_aet(theta, t, P_orb, L, AU, mode="G1", generation=1):
    X, Y, Z = tdi_xyz(theta, t, P_orb, L, AU, mode, generation)
    A = (Z - X) / math.sqrt(2.0)
    E = (X - 2.0 * Y + Z) / math.sqrt(6.0)
    T = (X + Y + Z) / math.sqrt(3.0)
    return A, E, T


def spectrum(theta, M, dt, P_orb, L, AU, mode="G1", chunk=1 << 15, generation=1):
    """Full-length spectra x~_k = dt FFT(x) of A, E, T sampled at t_n = n dt, n < M; [3, M]."""
    series = np.empty((3, M))
    for a in range(0, M, chunk):
        t = dt * np.arange(a, min(M, a + chunk), dtype=np.float64)
        A, E, T = tdi_aet(theta, t, P_orb, L, AU, mode, generation)
        series[0, a:a + len(t)] = A
        series[1, a:a + len(t)] = E
        series[2, a:a + len(t)] = T
    return dt * np.fft.fft(series, axis=1), series
