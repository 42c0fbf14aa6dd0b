"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/hf.h declares, derives the same constants as the oracle
bit for bit, and rejects bad arguments before touching a device."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

import oracle
from paper_2110_11408_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2110_11408_amd import build
        build.build()
    return _lib.load()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "hf.h")).read()
    return sorted(set(re.findall(r"\b(hf_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_function(lib):
    names = declared_functions()
    assert set(names) == set(_lib.EXPORTS)
    for name in names:
        assert hasattr(lib, name), name


def test_struct_layouts():
    assert ctypes.sizeof(_lib.HfParams) == 11 * 8 + 2 * 4
    assert ctypes.sizeof(_lib.HfHalo) == 40
    assert _lib.HALO_WORDS == 10


def test_defaults_match_paper_table(lib):
    p = _lib.default_params()
    for k, v in oracle.DEFAULTS.items():
        if k in ("box",):
            continue
        assert getattr(p, k) == v, k


@pytest.mark.parametrize("kw", [dict(box=64.0), dict(box=256.0), dict(box=31.7, mean_density=0.9),
                                dict(box=50.0, delta_l1=258.2, alpha_elig=0.7, c_roche=1.5,
                                     b_kernel=0.35, l_fof=0.3)])
@pytest.mark.parametrize("n", [1000, 262144, 16777216])
def test_derived_constants_bit_identical_to_oracle(lib, kw, n):
    p = _lib.default_params(**kw)
    mine = _lib.derived(p, n)
    ref = oracle.derive(n, **kw)
    for k in ref:
        assert mine[k] == ref[k], (k, mine[k], ref[k])


def test_invalid_arguments_rejected_without_device(lib):
    p = _lib.default_params(box=-1.0)
    out = (ctypes.c_double * 11)()
    assert lib.hf_derived(ctypes.byref(p), 10, out) == _lib.HF_ERR_INVALID
    p = _lib.default_params(box=10.0, delta_l1=float("nan"))
    assert lib.hf_derived(ctypes.byref(p), 10, out) == _lib.HF_ERR_INVALID
    # a NULL context is an argument error
    p = _lib.default_params(box=10.0)
    st = lib.hf_find(None, None, 0, ctypes.byref(p), None, None, None, None, 0, None, None)
    assert st == _lib.HF_ERR_INVALID


def test_create_without_gpu_is_unsupported(lib):
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("GPU present")
    except Exception:
        pass
    h = ctypes.c_void_p()
    assert lib.hf_create(ctypes.byref(h), 0, 0) == _lib.HF_ERR_UNSUPPORTED


def _c_layout():
    """sizeof / offsetof of the public structs as the C compiler lays them out."""
    import subprocess
    import tempfile
    fields = {"hf_params": [f for f, _ in _lib.HfParams._fields_],
              "hf_halo": [f for f, _ in _lib.HfHalo._fields_],
              "hf_stats": [f for f, _ in _lib.HfStats._fields_],
              "hf_request": [f for f, _ in _lib.HfRequest._fields_],
              "hf_halo_summary": [f for f, _ in _lib.HfHaloSummary._fields_],
              "hf_result": [f for f, _ in _lib.HfResult._fields_]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hf.h"', "int main(void) {"]
    for s, fs in fields.items():
        lines.append(f'printf("{s} size %zu\\n", sizeof({s}));')
        for f in fs:
            lines.append(f'printf("{s} {f} %zu\\n", offsetof({s}, {f}));')
    lines.append("return 0; }")
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "layout.c"), os.path.join(d, "layout")
        open(src, "w").write("\n".join(lines))
        subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), src, "-o", exe])
        out = subprocess.check_output([exe]).decode().split("\n")
    res = {}
    for ln in out:
        if ln:
            s, f, v = ln.split()
            res[(s, f)] = int(v)
    return res


def test_ctypes_structs_match_c_layout():
    c = _c_layout()
    for s, cls in (("hf_params", _lib.HfParams), ("hf_halo", _lib.HfHalo), ("hf_stats", _lib.HfStats),
                   ("hf_request", _lib.HfRequest), ("hf_result", _lib.HfResult),
                   ("hf_halo_summary", _lib.HfHaloSummary)):
        assert c[(s, "size")] == ctypes.sizeof(cls), s
        for f, _ in cls._fields_:
            assert c[(s, f)] == getattr(cls, f).offset, (s, f)


def test_batch_and_server_reject_bad_arguments(lib):
    p = _lib.default_params(box=10.0)
    offs = (ctypes.c_int64 * 2)(0, 0)
    st = lib.hf_find_batch(None, 1, offs, None, ctypes.byref(p), None, None, None, None, offs,
                           None, 0, None)
    assert st == _lib.HF_ERR_INVALID
    g = ctypes.c_int32(0)
    assert lib.hf_tune_batch(None, 1, offs, None, ctypes.byref(p), None, None, None, None, offs, None,
                             2, 1, None, ctypes.byref(g), None, None) == _lib.HF_ERR_INVALID
    assert lib.hf_load_tuning(None, b"/nonexistent", None) == _lib.HF_ERR_INVALID
    assert lib.hf_batch_groups(None, 1, 10, 0, ctypes.byref(g)) == _lib.HF_ERR_INVALID
    v = ctypes.c_int64(0)
    assert lib.hf_set_option(None, _lib.HF_OPT_RADIUS_SEARCH, _lib.HF_RADIUS_BINS) == _lib.HF_ERR_INVALID
    assert lib.hf_get_option(None, _lib.HF_OPT_RADIUS_SEARCH, ctypes.byref(v)) == _lib.HF_ERR_INVALID
    assert lib.hf_find_grouped(None, None, 0, ctypes.byref(p), None, None, None, None, 0, None, None, None,
                               None) == _lib.HF_ERR_INVALID
    h = ctypes.c_void_p()
    # slot count outside 1..16 and a zero budget are argument errors, checked first
    assert lib.hf_server_create(ctypes.byref(h), 0, 0, 1 << 30) == _lib.HF_ERR_INVALID
    assert lib.hf_server_create(ctypes.byref(h), 0, 17, 1 << 30) == _lib.HF_ERR_INVALID
    assert lib.hf_server_create(ctypes.byref(h), 0, 2, 0) == _lib.HF_ERR_INVALID
    assert lib.hf_server_submit(None, None, None) == _lib.HF_ERR_INVALID
    assert lib.hf_server_wait(None, 1, None) == _lib.HF_ERR_INVALID
    assert lib.hf_server_now(None) == 0.0


def test_server_without_gpu_is_unsupported(lib):
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("GPU present")
    except Exception:
        pass
    h = ctypes.c_void_p()
    assert lib.hf_server_create(ctypes.byref(h), 0, 2, 1 << 30) == _lib.HF_ERR_UNSUPPORTED


@pytest.mark.parametrize("om, z", [(0.315, 0.5), (1.0, 2.0), (0.3, 0.0), (0.25, 3.0)])
def test_params_at_redshift_matches_oracle(lib, om, z):
    """The library's redshift scaling (host code) against the oracle's own."""
    p = _lib.default_params(box=50.0)
    mine = _lib.params_at_redshift(p, om, z)
    ref = oracle.params_at_redshift(om, z, box=50.0)
    for k in ("delta_l1", "delta_l2", "delta_l0_min", "l_fof", "b_kernel", "alpha_elig"):
        assert getattr(mine, k) == pytest.approx(ref[k], rel=1e-14), k
    bad = _lib.HfParams()
    assert lib.hf_params_at_redshift(ctypes.byref(p), 0.0, 0.5, ctypes.byref(bad)) == _lib.HF_ERR_INVALID
