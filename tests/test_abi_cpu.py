"""The C-ABI library loads and exports every symbol include/gbx.h declares (no GPU needed)."""

import ctypes

import numpy as np
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gbx.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gb_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("gb_waveform", "gb_loglik", "gb_loglik_grad", "gb_mh_step", "gb_create",
              "gb_plan_create", "gb_window_prepare", "gb_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2307_03763_amd import api
    L = api.lib()
    for n in declared_functions():
        assert hasattr(L, n), n
    assert set(declared_functions()) == set(api.EXPORTS)


def test_argument_validation_without_device():
    """Calls that fail validation return an error code and a message before touching HIP."""
    from paper_2307_03763_amd import api
    L = api.lib()
    out = ctypes.c_void_p()
    assert L.gb_create(None, ctypes.byref(out)) == api.GB_EINVAL
    assert b"config" in L.gb_last_error()
    bad = api.gb_config(-1.0, 1.0, 1.0, 1.0)
    assert L.gb_create(ctypes.byref(bad), ctypes.byref(out)) == api.GB_EINVAL and out.value is None
    bad = api.gb_config(1.0, 1.0, 1.0, 1.0, 3, 0)
    assert L.gb_create(ctypes.byref(bad), ctypes.byref(out)) == api.GB_EINVAL and out.value is None
    assert b"tdi_generation" in L.gb_last_error()
    assert L.gb_plan_create(None, None, 0, 0, ctypes.byref(out)) == api.GB_EINVAL
    assert L.gb_waveform(None, None, 1, 128, 2, 0, None, None, None) == api.GB_EINVAL
    assert L.gb_loglik(None, None, None, None, None, None, None) == api.GB_EINVAL
    assert L.gb_loglik_grad(None, None, None, None, None, None, None) == api.GB_EINVAL
    assert L.gb_mh_step(None, None, None, None, None, None, 1.0, None, None, None, None) == api.GB_EINVAL
    assert L.gb_window_prepare(None, None, None, None) == api.GB_EINVAL
    assert L.gb_plan_info(None, None, None, None) == api.GB_EINVAL
    assert L.gb_autotune_windows(None, None, 0, None, None, None, 1, None, 0) == api.GB_EINVAL
    assert L.gb_set_orbit(None, None, 0, 0.0, 0.0) == api.GB_EINVAL
    assert b"null context" in L.gb_last_error()
    with pytest.raises(ValueError):
        api.gb_set_orbit(1, np.zeros((8, 3)), 0.0, 1.0)   # shape checked before any call


def test_merge_tuning_reports():
    """A window-tuned line replaces the generic line of its (precision, mode, N, C) family; other
    lines stay, families only the override holds are appended."""
    from paper_2307_03763_amd import api
    base = ("fp64  loglik N=512 C=3: lanes/template=128 min waves/SIMD=3 0.25 ms / 16384 (9 variants) "
            "kernel=k_batch<double,512,128,3,4,1,3>\n"
            "mixed grad   N=512 C=3: lanes/template=64 min waves/SIMD=2 0.31 ms / 16384 (6 variants) "
            "kernel=k_batch<float,512,64,3,4,2,2>\n")
    over = ("fp64  loglik N=512 C=3: lanes/template=128 min waves/SIMD=3 4.9 ms / 400000 (9 variants) "
            "kernel=k_batch<double,512,128,3,2,1,3>\n"
            "mixed loglik N=64 C=2: lanes/template=8 min waves/SIMD=2 0.26 ms / 450000 (4 variants) "
            "kernel=k_batch<float,64,8,2,4,1,2>\n")
    out = api.merge_tuning(base, over).splitlines()
    assert out == [over.splitlines()[0], base.splitlines()[1], over.splitlines()[1]]


def test_struct_layouts_match_header():
    from paper_2307_03763_amd import api
    assert ctypes.sizeof(api.gb_config) == 40 and api.gb_config.tdi_generation.offset == 32
    assert ctypes.sizeof(api.gb_window) == 48
    assert api.gb_window.data_off.offset == 24 and api.gb_window.n_cand.offset == 40


def test_noalloc_noise_estimate_validation_without_device():
    """The allocation-free noise estimate refuses more windows than its staging array holds, and
    bad windows, before touching HIP."""
    from paper_2307_03763_amd import api
    L = api.lib()
    wins = api.windows_array([[1000, 64, 64, 2, 0, 0, 0, 1]] * 16385)
    assert L.gb_noise_estimate_noalloc(wins, 16385, 1, 1.0, 1, None, None) == api.GB_EINVAL
    assert b"16384" in L.gb_last_error()
    bad = api.windows_array([[1000, 4097, 64, 2, 0, 0, 0, 1]])
    assert L.gb_noise_estimate_noalloc(bad, 1, 1, 1.0, 1, None, None) == api.GB_EINVAL
    assert L.gb_noise_estimate_noalloc(wins, 1, 1, -1.0, 1, None, None) == api.GB_EINVAL


class _NoLaunch:
    """Stands in for the library: any call other than the size query fails the test."""

    def __getattr__(self, name):
        def call(*args):
            raise AssertionError(f"{name} was called although an argument had the wrong size")
        return call


def test_binding_refuses_missized_tensors_before_any_call(monkeypatch):
    """The kernels index raw pointers, so the binding checks every tensor against the plan's
    rows, window count and data length before it calls the library (here with a stub library
    that fails the test when reached, and host tensors: the size checks come first)."""
    import torch
    from paper_2307_03763_amd import api
    rows, n_win, n = 10, 2, 100
    monkeypatch.setattr(api, "gb_plan_info", lambda plan: (rows, n_win, n))
    monkeypatch.setattr(api, "lib", lambda: _NoLaunch())
    f64 = torch.float64
    d = torch.zeros(n, dtype=torch.complex128)
    w = torch.zeros(n, dtype=f64)
    th = torch.zeros((rows, 8), dtype=f64)
    one = torch.zeros(rows, dtype=f64)
    cases = [
        lambda: api.gb_window_prepare(1, d[:n - 1], w),
        lambda: api.gb_window_prepare(1, d, w[:n - 1]),
        lambda: api.gb_loglik(1, d, w, th[:rows - 1], one),
        lambda: api.gb_loglik(1, d, w, th[:, :7].contiguous(), one),
        lambda: api.gb_loglik(1, d, w, th, one[:rows - 1]),
        lambda: api.gb_loglik(1, d, w, th, one, torch.zeros((rows, 3), dtype=f64)),
        lambda: api.gb_loglik_grad(1, d, w, th, one, torch.zeros((rows - 1, 8), dtype=f64)),
        lambda: api.gb_mh_step(1, d, w, th, one[:5], one, 1.0, one, one.to(torch.int32),
                               torch.zeros(n_win, dtype=torch.int64)),
        lambda: api.gb_mh_step(1, d, w, th, one, one, 1.0, one, one.to(torch.int32),
                               torch.zeros(n_win - 1, dtype=torch.int64)),
    ]
    for c in cases:
        with pytest.raises(ValueError):
            c()
    # correctly sized host tensors pass the size checks and are then refused as not on the device
    with pytest.raises(TypeError):
        api.gb_loglik(1, d, w, th, one, torch.zeros((rows, 2), dtype=f64))


def test_autotune_cache(tmp_path, monkeypatch):
    """autotune_cached tunes once per (library build, device, T, TDI generation) and re-applies
    the stored report afterwards; another key tunes again."""
    from paper_2307_03763_amd import api

    class Ctx:
        handle, T, tdi = 7, 6.3e7, 1
    applied, tuned = [], []
    monkeypatch.setattr(api, "apply_tuning", lambda h, rep: applied.append((h, rep)) or 1)
    path = str(tmp_path / "tune.json")

    def tune(c):
        tuned.append(c)
        return f"report {len(tuned)}"
    r1, hit1 = api.autotune_cached(Ctx(), path, tune=tune, device="gfx950 A")
    r2, hit2 = api.autotune_cached(Ctx(), path, tune=tune, device="gfx950 A")
    assert (r1, hit1, r2, hit2) == ("report 1", False, "report 1", True)
    assert applied == [(7, "report 1")] and len(tuned) == 1
    r3, hit3 = api.autotune_cached(Ctx(), path, tune=tune, device="gfx950 B")
    c2 = Ctx()
    c2.tdi = 2
    r4, hit4 = api.autotune_cached(c2, path, tune=tune, device="gfx950 A")
    assert (hit3, hit4) == (False, False) and len(tuned) == 3
    import json
    assert len(json.load(open(path))) == 3
