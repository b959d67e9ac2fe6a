"""The C-ABI library builds, loads and exports every symbol include/apcg.h
declares; the binding covers each of them.  CPU only: no compute calls."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "apcg.h")
LIB = os.path.join(ROOT, "paper_2306_17801_amd", "libapcg.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(apcg_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["apcg_ctx_create", "apcg_ctx_fork", "apcg_ctx_join", "apcg_ctx_wait_for", "apcg_ctx_query_idle",
                 "apcg_ctx_synchronize", "apcg_vec_dot_async", "apcg_vec_norm2_async", "apcg_vec_axpy_async",
                 "apcg_vec_aypx_async", "apcg_mat_mult_async", "apcg_ksp_solve", "apcg_scalar_get"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "run __graft_entry__.build() first"
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s+(apcg_[a-z0-9_]+)$", out, flags=re.M))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, f"not exported: {missing}"


def test_binding_covers_every_declared_symbol():
    from paper_2306_17801_amd import _capi
    import paper_2306_17801_amd as apcg

    for n in declared_functions():
        assert n in _capi.SIGNATURES, n
        assert hasattr(apcg, n), n


def test_library_loads_and_reports_version_without_gpu():
    import paper_2306_17801_amd as apcg
    import torch

    assert apcg.apcg_abi_version() == 1
    if torch.cuda.is_available():
        pytest.skip("GPU present: covered by the GPU tests")
    assert apcg.apcg_device_count() == 0
    with pytest.raises(apcg.ApcgError) as e:
        apcg.apcg_ctx_create(0)
    assert e.value.code == apcg.APCG_ERR_UNSUPPORTED
    assert "no HIP device" in apcg.apcg_last_error()


def test_struct_layouts_match_header():
    from paper_2306_17801_amd import _capi

    assert ctypes.sizeof(_capi.apcg_solve_opts) == 16 * 4
    assert ctypes.sizeof(_capi.apcg_solve_info) == 4 * 4 + 2 * 8
    assert ctypes.sizeof(_capi.apcg_spmv_config) == 16
    assert ctypes.sizeof(_capi.apcg_counters) == 16 * 8
