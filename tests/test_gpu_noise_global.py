"""The global noise estimate on the GPU (gb_noise_global) against oracle/noise_global.py, stage by
stage (Welch curve, smoothed curve, the estimate at every window bin and the weights), on PSD
noise with loud narrow lines over Algorithm 1's segments of 0.3-30 mHz: at 2^20 samples with
8192-sample Welch segments, and at the full-band size (2^22 samples, 4930 segments, 16384-sample
Welch segments: 511 of them).  All FP64: bars 1e-11 relative (the sums of the two sides are taken
in different orders)."""

import numpy as np
import pytest
import torch

from paper_2307_03763_amd import api
from paper_2307_03763_amd import inputs as I
from tests.gpu_common import banner, dev
from tests.test_oracle_noise_global import _band_setting

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))


@pytest.mark.parametrize("log2M,L", [(20, 8192), (22, 16384)])
def test_global_noise_matches_oracle(log2M, L):
    from oracle import noise_global as ng
    T = 2 ** log2M * I.DT
    d, seg, windows, offs = _band_setting(T, lines=40, amp=30.0)
    banner(f"gb_noise_global: M = 2^{log2M}, L = {L}, {len(windows)} windows")
    S_o, P_o, Sm_o = ng.global_noise(d, seg, windows, offs, T, I.DT, L=L)
    table = np.array([[k0, W, 64, C, o, 0, 0, 0] for (k0, W, C), o in zip(windows, offs)], dtype=np.int64)
    w, S, P, Sm = api.gb_noise_global(table, seg, dev(d, torch.complex128), T, I.DT, nperseg=L, stages=True)
    torch.cuda.synchronize()
    w, S, P, Sm = (t.cpu().numpy() for t in (w, S, P, Sm))
    # Welch curve: relative where it holds power (1e-6 of its channel's peak and above); the bins
    # outside the band hold only leakage and round-off, bounded against the channel's peak
    scale = np.max(np.abs(P_o), axis=1, keepdims=True)
    big = np.abs(P_o) >= 1e-6 * scale
    e_p = _rel(P[big], P_o[big])
    e_floor = float(np.max(np.abs(P - P_o) / scale))
    e_s, e_S = _rel(Sm, Sm_o), _rel(S, S_o)
    banner(f"  max relative differences: Welch {e_p:.1e} (out of band {e_floor:.1e} of the peak), "
           f"smoothed {e_s:.1e}, estimate {e_S:.1e}")
    assert e_p <= 1e-11 and e_floor <= 1e-13 and e_s <= 1e-11 and e_S <= 1e-11
    np.testing.assert_allclose(w, ng.weights(S_o, T), rtol=1e-11)


def test_global_noise_refuses_bad_settings():
    banner("gb_noise_global: bad settings refused on the host")
    T = 2 ** 20 * I.DT
    table = np.array([[1000, 64, 64, 2, 0, 0, 0, 0]], dtype=np.int64)
    d = torch.zeros(128, dtype=torch.complex128, device="cuda")
    with pytest.raises(api.GbxError, match="power of two"):
        api.gb_noise_global(table, [[1010, 1050]], d, T * 1.5, I.DT)
    with pytest.raises(api.GbxError, match="segment"):
        api.gb_noise_global(table, [[990, 1050]], d, T, I.DT)
    with pytest.raises(api.GbxError, match="fewer than the filter window"):
        api.gb_noise_global(table, [[1010, 1050]], d, T, I.DT, nperseg=8192)
