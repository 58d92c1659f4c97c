"""Python binding of libgbx.so: argument marshalling only.

Every function has the name of the C entry point it calls (include/gbx.h).  Device memory
and streams come from torch; all arithmetic runs in the library's HIP kernels.  There is no
fallback: if the library is missing or no HIP device is present the calls raise.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgbx.so")

GB_OK, GB_EINVAL, GB_EHIP, GB_ENOMEM, GB_EUNSUPPORTED = 0, -1, -2, -3, -4
GB_FP64, GB_MIXED, GB_PER_WINDOW = 0, 1, 2
PRECISION = {"fp64": GB_FP64, "mixed": GB_MIXED, "per_window": GB_PER_WINDOW}

EXPORTS = ("gb_create", "gb_destroy", "gb_last_error", "gb_waveform", "gb_channels", "gb_set_orbit", "gb_plan_create",
           "gb_plan_destroy", "gb_plan_info", "gb_window_prepare", "gb_loglik", "gb_loglik_grad", "gb_mh_step",
           "gb_autotune", "gb_autotune_windows", "gb_select_variant", "gb_fisher", "gb_kde_logpdf", "gb_add_templates",
           "gb_noise_estimate", "gb_noise_estimate_noalloc", "gb_noise_global", "gb_de_trial", "gb_de_select")


class GbxError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where} failed with status {status}: {msg}")
        self.status = status


class gb_config(ctypes.Structure):
    _fields_ = [("T", ctypes.c_double), ("orbit_period", ctypes.c_double),
                ("arm_length", ctypes.c_double), ("au", ctypes.c_double),
                ("tdi_generation", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class gb_noise_global_config(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("f_switch", ctypes.c_double), ("nperseg", ctypes.c_int32),
                ("clip_width", ctypes.c_int32), ("clip_stride", ctypes.c_int32), ("sg_short", ctypes.c_int32),
                ("sg_long", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class gb_window(ctypes.Structure):
    _fields_ = [("k0", ctypes.c_int64), ("W", ctypes.c_int32), ("N", ctypes.c_int32),
                ("C", ctypes.c_int32), ("precision", ctypes.c_int32), ("data_off", ctypes.c_int64),
                ("cand_off", ctypes.c_int64), ("n_cand", ctypes.c_int64)]


_lib = None
_vp = ctypes.c_void_p


def lib():
    """Load libgbx.so (built in-tree by paper_2307_03763_amd/build.py); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2307_03763_amd/build.py "
                              "(there is no non-HIP fallback)")
        L = ctypes.CDLL(LIB_PATH)
        i, i64, d, st = ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_int
        L.gb_create.argtypes = [ctypes.POINTER(gb_config), ctypes.POINTER(_vp)]
        L.gb_create.restype = st
        L.gb_destroy.argtypes = [_vp]
        L.gb_destroy.restype = None
        L.gb_last_error.argtypes = []
        L.gb_last_error.restype = ctypes.c_char_p
        L.gb_waveform.argtypes = [_vp, _vp, i64, i, i, i, _vp, _vp, _vp]
        L.gb_waveform.restype = st
        L.gb_channels.argtypes = [_vp, i64, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        L.gb_channels.restype = st
        L.gb_set_orbit.argtypes = [_vp, _vp, ctypes.c_int32, d, d]
        L.gb_set_orbit.restype = st
        L.gb_plan_create.argtypes = [_vp, ctypes.POINTER(gb_window), i, i, ctypes.POINTER(_vp)]
        L.gb_plan_create.restype = st
        L.gb_plan_destroy.argtypes = [_vp]
        L.gb_plan_destroy.restype = None
        L.gb_plan_info.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int),
                                   ctypes.POINTER(ctypes.c_int64)]
        L.gb_plan_info.restype = st
        L.gb_window_prepare.argtypes = [_vp, _vp, _vp, _vp]
        L.gb_window_prepare.restype = st
        L.gb_loglik.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]
        L.gb_loglik.restype = st
        L.gb_loglik_grad.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]
        L.gb_loglik_grad.restype = st
        L.gb_mh_step.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, d, _vp, _vp, _vp, _vp]
        L.gb_mh_step.restype = st
        L.gb_autotune.argtypes = [_vp, i, ctypes.c_char_p, ctypes.c_size_t]
        L.gb_autotune.restype = st
        L.gb_autotune_windows.argtypes = [_vp, _vp, i, _vp, _vp, _vp, i, ctypes.c_char_p, ctypes.c_size_t]
        L.gb_autotune_windows.restype = st
        L.gb_select_variant.argtypes = [_vp, i, i, i, i, i, i, i]
        L.gb_select_variant.restype = st
        L.gb_fisher.argtypes = [_vp, _vp, _vp, i, ctypes.POINTER(gb_window), _vp, _vp, _vp]
        L.gb_fisher.restype = st
        L.gb_kde_logpdf.argtypes = [_vp, _vp, i, i, i64, _vp, _vp, i64, _vp, _vp]
        L.gb_kde_logpdf.restype = st
        L.gb_noise_estimate.argtypes = [ctypes.POINTER(gb_window), i, _vp, d, _vp, _vp, _vp]
        L.gb_noise_estimate.restype = st
        L.gb_noise_estimate_noalloc.argtypes = [ctypes.POINTER(gb_window), i, _vp, d, _vp, _vp, _vp]
        L.gb_noise_estimate_noalloc.restype = st
        L.gb_noise_global.argtypes = [ctypes.POINTER(gb_window), ctypes.POINTER(ctypes.c_int64), i, _vp, d,
                                      ctypes.POINTER(gb_noise_global_config), _vp, _vp, _vp, _vp, _vp]
        L.gb_noise_global.restype = st
        L.gb_de_trial.argtypes = [i, i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, d, d, _vp, _vp, _vp]
        L.gb_de_trial.restype = st
        L.gb_de_select.argtypes = [i, i, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
        L.gb_de_select.restype = st
        L.gb_add_templates.argtypes = [_vp, ctypes.POINTER(gb_window), i, _vp, ctypes.POINTER(ctypes.c_int32), i, d,
                                       _vp, _vp, _vp]
        L.gb_add_templates.restype = st
        _lib = L
    return _lib


def _check(status: int, where: str):
    if status != GB_OK:
        raise GbxError(status, where, lib().gb_last_error().decode())


def _stream(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _dev(t: torch.Tensor, dtype, name: str) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a HIP device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def _real_view(t: torch.Tensor) -> torch.Tensor:
    return torch.view_as_real(t) if t.is_complex() else t


# ------------------------------------------------------------------------------------------
def gb_create(T: float, orbit_period: float, arm_length: float, au: float, tdi: int = 1) -> int:
    cfg = gb_config(T, orbit_period, arm_length, au, int(tdi), 0)
    out = _vp()
    _check(lib().gb_create(ctypes.byref(cfg), ctypes.byref(out)), "gb_create")
    return out.value


def gb_destroy(ctx: int):
    lib().gb_destroy(ctx)


def gb_waveform(ctx: int, theta: torch.Tensor, N: int, C: int, precision: int = GB_FP64, stream=None):
    """Templates [B, C, N] complex128 and first bins [B] int64 (see include/gbx.h)."""
    if theta.dim() != 2 or theta.shape[1] != 8:
        raise ValueError(f"theta must be [B, 8], got {list(theta.shape)}")
    B = theta.shape[0]
    h = torch.empty((B, C, N), dtype=torch.complex128, device=theta.device)
    fb = torch.empty((B,), dtype=torch.int64, device=theta.device)
    _check(lib().gb_waveform(ctx, _dev(theta, torch.float64, "theta"), B, N, C, precision,
                             _real_view(h).data_ptr(), fb.data_ptr(), _stream(stream)), "gb_waveform")
    return h, fb


def windows_array(table) -> ctypes.Array:
    """gb_window[] from rows (k0, W, N, C, data_off, w_off(unused), cand_off, n_cand[, precision])."""
    rows = np.asarray(table, dtype=np.int64).reshape(len(table), -1)
    arr = (gb_window * len(rows))()
    for i, r in enumerate(rows):
        prec = int(r[8]) if len(r) > 8 else GB_FP64
        arr[i] = gb_window(int(r[0]), int(r[1]), int(r[2]), int(r[3]), prec, int(r[4]), int(r[6]), int(r[7]))
    return arr


def gb_channels(ctx: int, k0: int, W: int) -> int:
    """Channel count of the rule of Sec. II for a window (what C = 0 resolves to in a plan)."""
    C = ctypes.c_int32()
    _check(lib().gb_channels(ctx, int(k0), int(W), ctypes.byref(C)), "gb_channels")
    return C.value


def gb_set_orbit(ctx: int, pos=None, t0: float = 0.0, dt: float = 0.0):
    """Numerical orbits for the context: positions pos [n, 3, 3] (spacecraft, xyz; m) at
    t_j = t0 + j dt (see include/gbx.h); pos None returns to the analytic orbits."""
    if pos is None:
        _check(lib().gb_set_orbit(ctx, None, 0, 0.0, 0.0), "gb_set_orbit")
        return
    a = np.ascontiguousarray(pos, dtype=np.float64)
    if a.ndim != 3 or a.shape[1:] != (3, 3):
        raise ValueError("pos must be [n, 3, 3]")
    _check(lib().gb_set_orbit(ctx, a.ctypes.data, a.shape[0], float(t0), float(dt)), "gb_set_orbit")


def gb_plan_create(ctx: int, table, precision: int) -> int:
    arr = windows_array(table)
    out = _vp()
    _check(lib().gb_plan_create(ctx, arr, len(arr), precision, ctypes.byref(out)), "gb_plan_create")
    return out.value


def gb_plan_destroy(plan: int):
    lib().gb_plan_destroy(plan)


def gb_plan_info(plan: int):
    """(rows, n_win, data_len) of a plan: the sizes its calls read and write."""
    rows, n_win, data_len = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int64()
    _check(lib().gb_plan_info(plan, ctypes.byref(rows), ctypes.byref(n_win), ctypes.byref(data_len)), "gb_plan_info")
    return rows.value, n_win.value, data_len.value


def _data_len(wins) -> int:
    """Elements of d and w that a window list reads: the largest data_off + C W."""
    return max((int(w.data_off) + int(w.C) * int(w.W) for w in wins), default=0)


def _check_len(t: torch.Tensor, n: int, name: str):
    """The kernels index raw pointers: a tensor shorter than what the call reads or writes would
    be an out-of-bounds device access, so it is refused before any launch."""
    if t.numel() < n:
        raise ValueError(f"{name} has {t.numel()} elements; the call reads or writes {n}")


def _check_rows(t: torch.Tensor, rows: int, width: int, name: str):
    if width == 1:
        ok = t.dim() == 1 and t.shape[0] >= rows
    else:
        ok = t.dim() == 2 and t.shape[1] == width and t.shape[0] >= rows
    if not ok:
        shape = f"[>= {rows}]" if width == 1 else f"[>= {rows}, {width}]"
        raise ValueError(f"{name} must be {shape}, got {list(t.shape)}")


def _check_data(plan: int, d: torch.Tensor, w: torch.Tensor):
    _, _, n = gb_plan_info(plan)
    _check_len(_real_view(d), 2 * n, "d (as float64 pairs)")
    _check_len(w, n, "w")


def _check_cand(plan: int, theta: torch.Tensor, outs):
    rows, _, _ = gb_plan_info(plan)
    _check_rows(theta, rows, 8, "theta")
    for t, width, name in outs:
        if t is not None:
            _check_rows(t, rows, width, name)


def gb_window_prepare(plan: int, d: torch.Tensor, w: torch.Tensor, stream=None):
    _check_data(plan, d, w)
    _check(lib().gb_window_prepare(plan, _dev(_real_view(d), torch.float64, "d"),
                                   _dev(w, torch.float64, "w"), _stream(stream)), "gb_window_prepare")


def gb_loglik(plan: int, d, w, theta, logL, comps=None, stream=None):
    _check_data(plan, d, w)
    _check_cand(plan, theta, [(logL, 1, "logL"), (comps, 2, "comps")])
    _check(lib().gb_loglik(plan, _dev(_real_view(d), torch.float64, "d"), _dev(w, torch.float64, "w"), _dev(theta, torch.float64, "theta"),
                           _dev(logL, torch.float64, "logL"),
                           None if comps is None else _dev(comps, torch.float64, "comps"),
                           _stream(stream)), "gb_loglik")


def gb_loglik_grad(plan: int, d, w, theta, logL, grad, stream=None):
    _check_data(plan, d, w)
    _check_cand(plan, theta, [(logL, 1, "logL"), (grad, 8, "grad")])
    _check(lib().gb_loglik_grad(plan, _dev(_real_view(d), torch.float64, "d"), _dev(w, torch.float64, "w"),
                                _dev(theta, torch.float64, "theta"), _dev(logL, torch.float64, "logL"),
                                _dev(grad, torch.float64, "grad"), _stream(stream)), "gb_loglik_grad")


def gb_mh_step(plan: int, d, w, theta, log_g, u, temperature: float, logL, chain, n_accept, stream=None):
    _check_data(plan, d, w)
    _check_cand(plan, theta, [(log_g, 1, "log_g"), (u, 1, "u"), (logL, 1, "logL"), (chain, 1, "chain")])
    _, n_win, _ = gb_plan_info(plan)
    _check_rows(n_accept, n_win, 1, "n_accept")
    _check(lib().gb_mh_step(plan, _dev(_real_view(d), torch.float64, "d"), _dev(w, torch.float64, "w"), _dev(theta, torch.float64, "theta"),
                            _dev(log_g, torch.float64, "log_g"), _dev(u, torch.float64, "u"),
                            float(temperature), _dev(logL, torch.float64, "logL"),
                            _dev(chain, torch.int32, "chain"), _dev(n_accept, torch.int64, "n_accept"),
                            _stream(stream)), "gb_mh_step")


def gb_autotune(ctx: int, reps: int = 5) -> str:
    buf = ctypes.create_string_buffer(16384)
    _check(lib().gb_autotune(ctx, reps, buf, len(buf)), "gb_autotune")
    return buf.value.decode()


def gb_autotune_windows(ctx: int, table, d: torch.Tensor, w: torch.Tensor, theta: torch.Tensor, reps: int = 3) -> str:
    """Launch shapes timed on the windows of `table` with their own data d, weights w and
    candidates theta [rows, 8]; returns the report of the families it tuned."""
    arr = windows_array(table)
    plan = gb_plan_create(ctx, table, GB_FP64)   # the sizes the windows need (C = 0 resolved)
    try:
        _check_data(plan, d, w)
        _check_cand(plan, theta, [])
    finally:
        gb_plan_destroy(plan)
    buf = ctypes.create_string_buffer(16384)
    _check(lib().gb_autotune_windows(ctx, arr, len(arr), _dev(_real_view(d), torch.float64, "d"),
                                     _dev(w, torch.float64, "w"), _dev(theta, torch.float64, "theta"), reps,
                                     buf, len(buf)), "gb_autotune_windows")
    return buf.value.decode()


def merge_tuning(base: str, override: str) -> str:
    """A tuning report with the lines of `override` in place of `base`'s lines for the same
    (precision, mode, N, C) family."""
    head = lambda line: line.split(":", 1)[0]
    over = {head(l): l for l in override.splitlines() if l.strip()}
    out = [over.pop(head(l), l) for l in base.splitlines() if l.strip()]
    return "\n".join(out + list(over.values())) + "\n"


def gb_select_variant(ctx: int, precision: int, mode: int, N: int, C: int, lanes_per_template: int,
                      waves_per_block: int, min_waves_per_simd: int):
    _check(lib().gb_select_variant(ctx, precision, mode, N, C, lanes_per_template, waves_per_block,
                                   min_waves_per_simd), "gb_select_variant")


def gb_fisher(ctx: int, theta: torch.Tensor, steps: torch.Tensor, table, w: torch.Tensor, stream=None) -> torch.Tensor:
    """Fisher matrices [n, 8, 8] of the sources theta [n, 8] in Table I coordinates; table: one
    window row per source (as Workload.window_table)."""
    n = theta.shape[0]
    wins = windows_array(table)
    if len(wins) != n:
        raise ValueError("gb_fisher: one window row per source")
    _check_rows(theta, n, 8, "theta")
    _check_rows(steps, n, 8, "steps")
    _check_len(w, _data_len(wins), "w")
    F = torch.empty((n, 8, 8), dtype=torch.float64, device=theta.device)
    _check(lib().gb_fisher(ctx, _dev(theta, torch.float64, "theta"), _dev(steps, torch.float64, "steps"), n, wins,
                           _dev(w, torch.float64, "w"), _dev(F, torch.float64, "F"), _stream(stream)), "gb_fisher")
    return F


def gb_kde_logpdf(pts: torch.Tensor, wts: torch.Tensor, chol: torch.Tensor, x: torch.Tensor, stream=None) -> torch.Tensor:
    """Sum over parameter pairs of the log KDE density: pts [P, m, 2], wts [P, m], chol [P, 3],
    x [q, P, 2] -> [q]; or S independent sets: pts [S, P, m, 2], wts [S, P, m], chol [S, P, 3],
    x [S, q, P, 2] -> [S, q]."""
    one = pts.dim() == 3
    S = 1 if one else int(pts.shape[0])
    P, m = int(pts.shape[-3]), int(pts.shape[-2])
    q = int(x.shape[-3])
    if (tuple(wts.shape[-2:]) != (P, m) or tuple(chol.shape[-2:]) != (P, 3) or tuple(x.shape[-2:]) != (P, 2)
            or (not one and (wts.shape[0] != S or chol.shape[0] != S or x.shape[0] != S))):
        raise ValueError("gb_kde_logpdf: inconsistent shapes")
    out = torch.empty((q,) if one else (S, q), dtype=torch.float64, device=x.device)
    _check(lib().gb_kde_logpdf(_dev(pts, torch.float64, "pts"), _dev(wts, torch.float64, "wts"), S, P, m,
                               _dev(chol, torch.float64, "chol"), _dev(x, torch.float64, "x"), q,
                               _dev(out, torch.float64, "out"), _stream(stream)), "gb_kde_logpdf")
    return out


def gb_noise_estimate(table, d: torch.Tensor, T: float, w: Optional[torch.Tensor] = None, stream=None):
    """Median-periodogram noise level of every window and channel of ``table`` from the data d,
    and the weights 4 / (T S) written into w (a copy of d's layout, new unless given).  Returns
    (w, S [n_win, 3])."""
    wins = windows_array(table)
    _check_len(d, _data_len(wins), "d")
    if w is None:
        w = torch.zeros(d.shape, dtype=torch.float64, device=d.device)
    _check_len(w, _data_len(wins), "w")
    S = torch.zeros((len(wins), 3), dtype=torch.float64, device=d.device)
    _check(lib().gb_noise_estimate(wins, len(wins), _dev(d, torch.complex128, "d"), float(T),
                                   _dev(w, torch.float64, "w"), _dev(S, torch.float64, "S"), _stream(stream)),
           "gb_noise_estimate")
    return w, S


def gb_noise_estimate_noalloc(table, d: torch.Tensor, T: float, w: torch.Tensor, S: Optional[torch.Tensor] = None,
                              stream=None):
    """gb_noise_estimate into caller-supplied w (d's layout) and S [n_win, 3] (or None): the
    library allocates no device memory (its window list is staged in a fixed device array;
    at most 16384 windows)."""
    wins = windows_array(table)
    _check_len(d, _data_len(wins), "d")
    _check_len(w, _data_len(wins), "w")
    if S is not None and tuple(S.shape) != (len(wins), 3):
        raise ValueError("gb_noise_estimate_noalloc: S must be [n_win, 3]")
    _check(lib().gb_noise_estimate_noalloc(wins, len(wins), _dev(d, torch.complex128, "d"), float(T),
                                           _dev(w, torch.float64, "w"),
                                           None if S is None else _dev(S, torch.float64, "S"), _stream(stream)),
           "gb_noise_estimate_noalloc")


def gb_noise_global(table, seg, d: torch.Tensor, T: float, dt: float = 15.0, nperseg: int = 16384,
                    clip_width: int = 30, clip_stride: int = 15, sg_short: int = 10, sg_long: int = 70,
                    f_switch: float = 0.8e-3, w: Optional[torch.Tensor] = None, S: bool = True,
                    stages: bool = False, stream=None):
    """Global noise estimate of the residual d (window layout of ``table``) over the segments
    ``seg`` ([n_win, 2] absolute bins [lo, hi) per window).  Returns (w, S or None, welch or None,
    smooth or None): the weights 4 / (T S) and the estimate S in d's layout, and with
    ``stages`` the Welch and smoothed curves [3, nperseg/2 + 1]."""
    wins = windows_array(table)
    sg = np.ascontiguousarray(np.asarray(seg, dtype=np.int64).reshape(len(wins), 2))
    n = _data_len(wins)
    _check_len(d, n, "d")
    if w is None:
        w = torch.zeros(d.shape, dtype=torch.float64, device=d.device)
    _check_len(w, n, "w")
    s_t = torch.zeros(d.shape, dtype=torch.float64, device=d.device) if S else None
    nb = nperseg // 2 + 1
    wl = torch.zeros((3, nb), dtype=torch.float64, device=d.device) if stages else None
    sm = torch.zeros((3, nb), dtype=torch.float64, device=d.device) if stages else None
    cfg = gb_noise_global_config(float(dt), float(f_switch), int(nperseg), int(clip_width), int(clip_stride),
                                 int(sg_short), int(sg_long), 0)
    opt = lambda t, name: None if t is None else _dev(t, torch.float64, name)
    _check(lib().gb_noise_global(wins, sg.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(wins),
                                 _dev(d, torch.complex128, "d"), float(T), ctypes.byref(cfg),
                                 _dev(w, torch.float64, "w"), opt(s_t, "S"), opt(wl, "welch"), opt(sm, "smooth"),
                                 _stream(stream)), "gb_noise_global")
    return w, s_t, wl, sm


def gb_de_trial(lo: torch.Tensor, hi: torch.Tensor, x: torch.Tensor, u_idx: torch.Tensor, u_cross: torch.Tensor,
                u_j: torch.Tensor, F: torch.Tensor, cr: float, amp: float, trial_x: Optional[torch.Tensor] = None,
                trial_theta: Optional[torch.Tensor] = None, base: Optional[torch.Tensor] = None, stream=None):
    """DE/rand/1/bin trials of every member (DE/best/1/bin with base [n_win] int32, the best
    member of each window): x [n_win, pop, 7], lo/hi [n_win, 7], u_idx [n_win, pop, 3],
    u_cross [n_win, pop, 7], u_j [n_win, pop], F [n_win] -> (trial_x [n_win, pop, 7],
    trial_theta [n_win * pop, 8])."""
    n_win, pop = int(x.shape[0]), int(x.shape[1])
    if (tuple(x.shape) != (n_win, pop, 7) or tuple(lo.shape) != (n_win, 7) or tuple(hi.shape) != (n_win, 7)
            or tuple(u_idx.shape) != (n_win, pop, 3) or tuple(u_cross.shape) != (n_win, pop, 7)
            or tuple(u_j.shape) != (n_win, pop) or tuple(F.shape) != (n_win,)):
        raise ValueError("gb_de_trial: inconsistent shapes")
    if trial_x is None:
        trial_x = torch.empty_like(x)
    if trial_theta is None:
        trial_theta = torch.empty((n_win * pop, 8), dtype=torch.float64, device=x.device)
    if base is not None and tuple(base.shape) != (n_win,):
        raise ValueError("gb_de_trial: base must be [n_win]")
    f = lambda t, n: _dev(t, torch.float64, n)
    _check(lib().gb_de_trial(n_win, pop, f(lo, "lo"), f(hi, "hi"), f(x, "x"), f(u_idx, "u_idx"), f(u_cross, "u_cross"),
                             f(u_j, "u_j"), f(F, "F"), None if base is None else _dev(base, torch.int32, "base"),
                             float(cr), float(amp), f(trial_x, "trial_x"), f(trial_theta, "trial_theta"),
                             _stream(stream)), "gb_de_trial")
    return trial_x, trial_theta


def gb_de_select(comps: torch.Tensor, x: torch.Tensor, s: torch.Tensor, trial_x: torch.Tensor,
                 best: Optional[torch.Tensor] = None, best_idx: Optional[torch.Tensor] = None,
                 stream=None) -> torch.Tensor:
    """Greedy DE selection in place on x [n_win, pop, 7] and s [n_win, pop] from the trials'
    components comps [n_win * pop, 2]; returns best [n_win] (largest rho per window) and, if
    best_idx [n_win] int32 is given, writes the smallest index holding it there."""
    n_win, pop = int(x.shape[0]), int(x.shape[1])
    if (tuple(comps.shape) != (n_win * pop, 2) or tuple(s.shape) != (n_win, pop) or tuple(trial_x.shape) != (n_win, pop, 7)
            or tuple(x.shape) != (n_win, pop, 7)):
        raise ValueError("gb_de_select: inconsistent shapes")
    if best is None:
        best = torch.empty(n_win, dtype=torch.float64, device=x.device)
    f = lambda t, n: _dev(t, torch.float64, n)
    if best_idx is not None and tuple(best_idx.shape) != (n_win,):
        raise ValueError("gb_de_select: best_idx must be [n_win]")
    _check(lib().gb_de_select(n_win, pop, f(comps, "comps"), f(x, "x"), f(s, "s"), f(trial_x, "trial_x"),
                              f(best, "best"), None if best_idx is None else _dev(best_idx, torch.int32, "best_idx"),
                              _stream(stream)), "gb_de_select")
    return best


def gb_add_templates(ctx: int, table, theta: torch.Tensor, src_win, sign: float, d_in: torch.Tensor,
                     d_out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """d_out = d_in + sign * sum of the templates of theta [n, 8], source s placed in window
    src_win[s] of table.  Returns d_out (a new tensor unless given)."""
    wins = windows_array(table)
    sw = np.ascontiguousarray(np.asarray(src_win, dtype=np.int32))
    if d_out is None:
        d_out = torch.empty_like(d_in)
    n_src = int(len(sw))
    n = _data_len(wins)
    _check_len(d_in, n, "d_in")
    _check_len(d_out, n, "d_out")
    if n_src:
        _check_rows(theta, n_src, 8, "theta")
    th = theta if n_src else torch.zeros((1, 8), dtype=torch.float64, device=d_in.device)
    _check(lib().gb_add_templates(ctx, wins, len(wins), _dev(th, torch.float64, "theta"),
                                  sw.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), n_src, float(sign),
                                  _real_view(d_in).data_ptr(), _real_view(d_out).data_ptr(), _stream(stream)),
           "gb_add_templates")
    return d_out


def apply_tuning(ctx: int, report: str) -> int:
    """Re-apply the choices of a gb_autotune report (its 'kernel=k_batch<R,N,LPC,C,WPB,MODE,OCC>'
    entries); returns how many were set."""
    import re
    n = 0
    for m in re.finditer(r"kernel=k_batch<(double|float),(\d+),(\d+),(\d+),(\d+),(\d+),(\d+)>", report):
        r, N, lpc, C, wpb, mode, occ = m.groups()
        gb_select_variant(ctx, GB_FP64 if r == "double" else GB_MIXED, int(mode), int(N), int(C), int(lpc),
                          int(wpb), int(occ))
        n += 1
    return n


def tuning_key(ctx: "Context", device: Optional[str] = None) -> str:
    """Key of a tuning report: the library build (sha256 of libgbx.so), the device name and the
    context's settings (observation time, TDI generation) -- what the timings depend on."""
    import hashlib
    h = hashlib.sha256(open(LIB_PATH, "rb").read()).hexdigest()[:16]
    if device is None:
        device = torch.cuda.get_device_name(torch.cuda.current_device())
    return f"{h}|{device}|T={ctx.T!r}|tdi={ctx.tdi}"


def autotune_cached(ctx: "Context", path: str, reps: int = 3, tune=None, device: Optional[str] = None) -> tuple:
    """gb_autotune through a cache file (JSON, {key: report}): a report stored under this
    context's tuning_key is re-applied (apply_tuning) instead of timing again; otherwise the
    context is tuned (tune(ctx), by default gb_autotune with `reps`) and the report stored.
    Returns (report, True if it came from the cache).  Reports are plain text, so the file can
    be shared between processes that run the same build on the same device."""
    import json
    key = tuning_key(ctx, device)
    cache = {}
    if os.path.exists(path):
        with open(path) as fh:
            cache = json.load(fh)
    if key in cache:
        apply_tuning(ctx.handle, cache[key])
        return cache[key], True
    report = tune(ctx) if tune is not None else gb_autotune(ctx.handle, reps)
    cache[key] = report
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1)
    os.replace(tmp, path)
    return report, False


# ------------------------------------------------------------------------------------------
# Destruction during a HIP-graph capture.  gb_destroy and gb_plan_destroy free device memory,
# and a free while a stream is being captured invalidates the capture.  A capture may see such a
# destruction without asking for it: the cyclic garbage collector can collect an unreferenced
# Plan or Context at any allocation, including one inside the captured body.  So while a
# capture is open (capturing()), the destructors queue their frees; the outermost capture runs
# them when it closes.
_capture_depth = 0
_deferred = []


class capturing:
    """Context manager around a HIP-graph capture: Plan and Context destruction inside it is
    deferred to its end (nested captures count, the outermost one runs the queue)."""

    def __enter__(self):
        global _capture_depth
        _capture_depth += 1
        return self

    def __exit__(self, *exc):
        global _capture_depth
        _capture_depth -= 1
        if _capture_depth == 0:
            release_deferred()
        return False


def release_deferred():
    """Run the frees queued during captures (a no-op while a capture is still open)."""
    while _deferred and _capture_depth == 0:
        fn, handle = _deferred.pop(0)
        fn(handle)


def _release(fn, handle):
    if _capture_depth > 0:
        _deferred.append((fn, handle))
    else:
        fn(handle)


class Context:
    """Owns a gb_ctx for one (T, orbit, arm length, TDI generation) setting on the current device."""

    def __init__(self, T: float, orbit_period: float, arm_length: float, au: float, tdi: int = 1):
        self.T = float(T)
        self.tdi = int(tdi)
        self.handle = gb_create(T, orbit_period, arm_length, au, tdi)

    def set_orbit(self, pos=None, t0: float = 0.0, dt: float = 0.0):
        """Numerical orbits (gb_set_orbit); no arguments: back to the analytic orbits."""
        gb_set_orbit(self.handle, pos, t0, dt)

    def waveform(self, theta: torch.Tensor, N: int, C: int, precision: int = GB_FP64, stream=None):
        return gb_waveform(self.handle, theta, N, C, precision, stream)

    def close(self):
        if self.handle:
            _release(gb_destroy, self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Owns a gb_plan for a fixed set of windows; outputs are allocated per call."""

    def __init__(self, ctx: Context, table, precision: int):
        self.ctx = ctx
        t = np.asarray(table, dtype=np.int64).reshape(len(table), -1)
        self.table = t
        self.rows = int((t[:, 6] + t[:, 7]).max()) if len(t) else 0
        self.n_win = len(t)
        self.handle = gb_plan_create(ctx.handle, t, precision)
        self.d = self.w = None

    def prepare(self, d: torch.Tensor, w: torch.Tensor, stream=None):
        d = d.contiguous()
        w = w.contiguous()
        gb_window_prepare(self.handle, d, w, stream)
        self.d, self.w = d, w

    def loglik(self, theta: torch.Tensor, comps: bool = False, stream=None):
        logL = torch.empty(self.rows, dtype=torch.float64, device=theta.device)
        cp = torch.empty((self.rows, 2), dtype=torch.float64, device=theta.device) if comps else None
        gb_loglik(self.handle, self.d, self.w, theta, logL, cp, stream)
        return (logL, cp) if comps else logL

    def loglik_grad(self, theta: torch.Tensor, stream=None):
        logL = torch.empty(self.rows, dtype=torch.float64, device=theta.device)
        grad = torch.empty((self.rows, 8), dtype=torch.float64, device=theta.device)
        gb_loglik_grad(self.handle, self.d, self.w, theta, logL, grad, stream)
        return logL, grad

    def mh_step(self, theta, log_g, u, temperature: float, stream=None):
        logL = torch.empty(self.rows, dtype=torch.float64, device=theta.device)
        chain = torch.empty(self.rows, dtype=torch.int32, device=theta.device)
        nacc = torch.empty(self.n_win, dtype=torch.int64, device=theta.device)
        gb_mh_step(self.handle, self.d, self.w, theta, log_g, u, temperature, logL, chain, nacc, stream)
        return logL, chain, nacc

    def close(self):
        if self.handle:
            _release(gb_plan_destroy, self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class LogLikelihood(torch.autograd.Function):
    """logL of every candidate of a prepared plan as a differentiable torch function: the
    forward pass runs gb_loglik_grad (likelihood and the hand-written adjoint gradient in one
    launch) and keeps the gradient; the backward pass scales it by the incoming cotangent.
    The plan's windows need a gradient-capable precision (mixed; the FP64 gradient is off)."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, plan: "Plan") -> torch.Tensor:
        logL, grad = plan.loglik_grad(theta.detach().contiguous())
        ctx.save_for_backward(grad)
        return logL

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        (grad,) = ctx.saved_tensors
        return grad_out[:, None] * grad, None


def loglik(plan: "Plan", theta: torch.Tensor) -> torch.Tensor:
    """Differentiable logL of theta [rows, 8] on a prepared plan (see LogLikelihood)."""
    return LogLikelihood.apply(theta, plan)


def context_for(T: float, tdi: int = 1):
    """Context with the synthetic setting's constellation constants (TDI generation 1 or 2)."""
    from . import inputs as I
    return Context(T, I.YEAR, I.ARM_L, I.AU, tdi)


def template_fn(ctx: Context, precision: int = GB_FP64, device="cuda"):
    """Adapter for inputs.finalize_data: injections computed by the HIP path."""
    def fn(theta, N, C, T):
        th = torch.as_tensor(np.ascontiguousarray(theta), dtype=torch.float64, device=device)
        h, fb = ctx.waveform(th, N, C, precision)
        return h.cpu().numpy(), fb.cpu().numpy()
    return fn
