"""Plain references for the posterior stage's helpers -- TEST INFRASTRUCTURE ONLY.

* fisher_fd   -- the Fisher information matrix F_ij = <d_i h | d_j h> (Sec. III G FIM
                 equation) in Table I coordinates, with the derivatives taken the way the paper
                 states: second-order forward finite differences of the template, steps given
                 per parameter (the paper uses 1e-9 of the prior widths).  Templates from the
                 FP64 oracle; the scalar product over the window's bins and channels.
* fisher_u    -- the same matrix from the oracle's exact (dual-number) template derivatives,
                 carried to Table I coordinates by the chain rule; pins fisher_fd.
* kde_logpdf  -- log of a weighted 2-D Gaussian kernel density estimate, summed over parameter
                 pairs, by its definition (log-sum-exp over the kernel points).
Only tests/, the smoke check and the benchmark's CPU-baseline leg may use this module.
"""

from __future__ import annotations

import math

import numpy as np

from paper_2307_03763_amd import inputs as I

from . import oracle as O


def _placed(h, fb, k0, W):
    """A template [C][N] at first bin fb, as a [C][W] block of the window starting at k0."""
    C, N = h.shape
    out = np.zeros((C, W), dtype=np.complex128)
    for i in range(N):
        k = fb + i
        if k0 <= k < k0 + W:
            out[:, k - k0] = h[:, i]
    return out


def fisher_fd(theta, k0, W, N, C, w, g, steps) -> np.ndarray:
    """F in Table I coordinates by d_i h = (-3 h(u) + 4 h(u + e_i) - h(u + 2 e_i)) / (2 e_i)."""
    w = np.asarray(w, dtype=np.float64).reshape(C, W)
    u0 = I.to_table1(np.asarray(theta, dtype=np.float64))
    pts = [u0]
    for i in range(8):
        for k in (1, 2):
            u = u0.copy()
            u[i] += k * steps[i]
            pts.append(u)
    th = I.from_table1(np.array(pts))
    h, fb = O.waveform(th, N, C, g)
    blocks = [_placed(h[j], int(fb[j]), k0, W) for j in range(len(th))]
    D = []
    for i in range(8):
        if steps[i] == 0:
            D.append(np.zeros((C, W), dtype=np.complex128))
            continue
        D.append((-3.0 * blocks[0] + 4.0 * blocks[1 + 2 * i] - blocks[2 + 2 * i]) / (2.0 * steps[i]))
    F = np.zeros((8, 8))
    for i in range(8):
        for j in range(i, 8):
            F[i, j] = F[j, i] = float(np.sum(w * (D[i] * np.conj(D[j])).real))
    return F


def table1_jacobian(theta) -> np.ndarray:
    """d theta / d u for the Table I coordinates (diagonal)."""
    th = np.asarray(theta, dtype=np.float64)
    j = np.ones(8)
    j[2] = 1.0 / math.cos(th[2])
    j[4] = th[4] * math.log(10.0)
    j[5] = -1.0 / math.sin(th[5])
    return j


def fisher_u(theta, k0, W, N, C, w, g) -> np.ndarray:
    """The exact Fisher matrix (oracle, dual numbers) in Table I coordinates."""
    F = O.fisher(theta, k0, W, N, C, np.asarray(w, dtype=np.float64).ravel(), g)
    J = table1_jacobian(theta)
    return F * np.outer(J, J)


def kde_logpdf(pts, wts, chol, x) -> np.ndarray:
    """sum_p log sum_j wts[p, j] N(x[:, p]; pts[p, j], L_p L_p^T), L_p from chol[p] = (l00, l10, l11)."""
    pts, wts, chol, x = (np.asarray(a, dtype=np.float64) for a in (pts, wts, chol, x))
    out = np.zeros(x.shape[0])
    for p in range(pts.shape[0]):
        L = np.array([[chol[p, 0], 0.0], [chol[p, 1], chol[p, 2]]])
        H = L @ L.T
        Hi = np.linalg.inv(H)
        with np.errstate(divide="ignore"):
            lw = np.log(wts[p])[None, :]
        for a in range(0, x.shape[0], 512):                                # queries in chunks
            d = x[a:a + 512, p, None, :] - pts[p][None, :, :]              # [q, m, 2]
            quad = np.einsum("qmi,ij,qmj->qm", d, Hi, d)
            e = lw - 0.5 * quad
            mx = np.max(e, axis=1, keepdims=True)
            out[a:a + 512] += (mx[:, 0] + np.log(np.sum(np.exp(e - mx), axis=1))
                               - math.log(2.0 * math.pi) - 0.5 * math.log(np.linalg.det(H)))
    return out
