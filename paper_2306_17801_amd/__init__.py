"""apcg -- asynchronous, device-resident preconditioned CG for AMD MI355X.

Python binding of the C ABI declared in include/apcg.h.  Each ``apcg_*``
function below calls the C entry point of the same name: it marshals
arguments (handles are ints, vectors and matrices are float64/int32 torch
tensors on the GPU), returns what the C call writes through its out-pointers
and raises ApcgError on failure.  All computation happens in the HIP library;
there is no Python or CPU fallback, and using any function without the built
library raises.

PyTorch provides device memory only: the library never allocates the caller's
vectors, and tensors passed in must stay alive until the work using them has
finished (``apcg_ctx_synchronize`` or an accessor).  Tensors written by torch
kernels must be complete before the library reads them (for example
``torch.cuda.synchronize()`` after filling them).
"""
from __future__ import annotations

import ctypes
import os

from . import _capi
from ._capi import *  # noqa: F401,F403  -- constants and structures
from ._capi import ApcgError, check, load

__all__ = [n for n in dir(_capi) if n.startswith(("APCG_", "apcg_"))] + ["ApcgError", "load"]


def _L():
    return load()


def _h(x):
    """Handle -> c_void_p value (None for NULL)."""
    return None if x is None else ctypes.c_void_p(int(x))


def _tensor_ptr(t, dtype_name):
    import torch

    want = {"float64": torch.float64, "int32": torch.int32}[dtype_name]
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch.Tensor")
    if t.dtype != want:
        raise TypeError(f"expected dtype {dtype_name}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr(), t.device.index or 0


# ------------------------------------------------------------------ misc

def apcg_abi_version() -> int:
    return int(_L().apcg_abi_version())


def apcg_last_error() -> str:
    m = _L().apcg_last_error()
    return m.decode() if m else ""


def apcg_device_count() -> int:
    c = ctypes.c_int32()
    check("apcg_device_count", _L().apcg_device_count(ctypes.byref(c)))
    return c.value


def apcg_device_props_get(device: int = 0) -> dict:
    p = _capi.apcg_device_props()
    check("apcg_device_props_get", _L().apcg_device_props_get(device, ctypes.byref(p)))
    return {"name": p.name.decode(), "arch": p.arch.decode(), "compute_units": p.compute_units,
            "wavefront_size": p.wavefront_size, "global_mem_bytes": p.global_mem_bytes,
            "clock_khz": p.clock_khz, "l2_bytes": p.l2_bytes, "lds_bytes_per_block": p.lds_bytes_per_block}


def apcg_counters_get() -> dict:
    c = _capi.apcg_counters()
    check("apcg_counters_get", _L().apcg_counters_get(ctypes.byref(c)))
    return c.as_dict()


def apcg_counters_reset() -> None:
    check("apcg_counters_reset", _L().apcg_counters_reset())


# ------------------------------------------------------------------ contexts

def apcg_ctx_create(device: int = 0, stream_type: int = _capi.APCG_STREAM_DEFAULT) -> int:
    out = ctypes.c_void_p()
    check("apcg_ctx_create", _L().apcg_ctx_create(device, stream_type, ctypes.byref(out)))
    return out.value


def apcg_ctx_destroy(ctx) -> None:
    check("apcg_ctx_destroy", _L().apcg_ctx_destroy(_h(ctx)))


def apcg_ctx_wait_for(waiter, waitee) -> None:
    check("apcg_ctx_wait_for", _L().apcg_ctx_wait_for(_h(waiter), _h(waitee)))


def apcg_ctx_query_idle(ctx) -> bool:
    out = ctypes.c_int32()
    check("apcg_ctx_query_idle", _L().apcg_ctx_query_idle(_h(ctx), ctypes.byref(out)))
    return bool(out.value)


def apcg_ctx_synchronize(ctx) -> None:
    check("apcg_ctx_synchronize", _L().apcg_ctx_synchronize(_h(ctx)))


def apcg_ctx_fork(parent, n: int) -> list:
    arr = (ctypes.c_void_p * max(n, 1))()
    check("apcg_ctx_fork", _L().apcg_ctx_fork(_h(parent), n, arr))
    return [arr[i] for i in range(n)]


def apcg_ctx_join(parent, children, mode: int = _capi.APCG_JOIN_DESTROY) -> list:
    n = len(children)
    arr = (ctypes.c_void_p * max(n, 1))(*[int(c) for c in children])
    check("apcg_ctx_join", _L().apcg_ctx_join(_h(parent), n, mode, arr))
    return [arr[i] for i in range(n)]


def apcg_ctx_get_stream_type(ctx) -> int:
    out = ctypes.c_int32()
    check("apcg_ctx_get_stream_type", _L().apcg_ctx_get_stream_type(_h(ctx), ctypes.byref(out)))
    return out.value


def apcg_ctx_kernel_times(ctx, kind: int):
    mean = ctypes.c_double()
    cnt = ctypes.c_int32()
    check("apcg_ctx_kernel_times", _L().apcg_ctx_kernel_times(_h(ctx), kind, ctypes.byref(mean), ctypes.byref(cnt)))
    return mean.value, cnt.value


# ------------------------------------------------------------------ scalars

def apcg_scalar_create(ctx=None) -> int:
    out = ctypes.c_void_p()
    check("apcg_scalar_create", _L().apcg_scalar_create(_h(ctx), ctypes.byref(out)))
    return out.value


def apcg_scalar_destroy(s) -> None:
    check("apcg_scalar_destroy", _L().apcg_scalar_destroy(_h(s)))


def apcg_scalar_set(s, value: float, ctx=None) -> None:
    check("apcg_scalar_set", _L().apcg_scalar_set(_h(s), float(value), _h(ctx)))


def apcg_scalar_get(s) -> float:
    out = ctypes.c_double()
    check("apcg_scalar_get", _L().apcg_scalar_get(_h(s), ctypes.byref(out)))
    return out.value


def apcg_scalar_op(opcode: int, out, a, b=None, ctx=None) -> None:
    check("apcg_scalar_op", _L().apcg_scalar_op(opcode, _h(out), _h(a), _h(b), _h(ctx)))


# ------------------------------------------------------ dependency marking

def apcg_ctx_get_stream(ctx) -> int:
    out = ctypes.c_void_p()
    check("apcg_ctx_get_stream", _L().apcg_ctx_get_stream(_h(ctx), ctypes.byref(out)))
    return out.value


def apcg_memory_register(device: int, ptr: int, nbytes: int) -> int:
    out = ctypes.c_uint64()
    check("apcg_memory_register", _L().apcg_memory_register(device, ctypes.c_void_p(ptr), nbytes, ctypes.byref(out)))
    return out.value


def apcg_memory_lookup(device: int, ptr: int):
    """(id, start, bytes) of the registered region holding ptr."""
    i, st, nb = ctypes.c_uint64(), ctypes.c_void_p(), ctypes.c_int64()
    check("apcg_memory_lookup", _L().apcg_memory_lookup(device, ctypes.c_void_p(ptr), ctypes.byref(i),
                                                        ctypes.byref(st), ctypes.byref(nb)))
    return i.value, st.value, nb.value


def apcg_memory_unregister(mid: int) -> None:
    check("apcg_memory_unregister", _L().apcg_memory_unregister(mid))


def _get_id(fn, h) -> int:
    out = ctypes.c_uint64()
    check(fn, getattr(_L(), fn)(_h(h), ctypes.byref(out)))
    return out.value


def apcg_vec_get_id(v) -> int:
    return _get_id("apcg_vec_get_id", v)


def apcg_scalar_get_id(s) -> int:
    return _get_id("apcg_scalar_get_id", s)


def apcg_mat_get_id(A) -> int:
    return _get_id("apcg_mat_get_id", A)


def apcg_mark_intent_begin(ctx, mid: int, mode: int, description: str | None = None) -> None:
    d = description.encode() if description else None
    check("apcg_mark_intent_begin", _L().apcg_mark_intent_begin(_h(ctx), mid, mode, d))


def apcg_mark_intent_end(ctx, mid: int, mode: int, description: str | None = None) -> None:
    d = description.encode() if description else None
    check("apcg_mark_intent_end", _L().apcg_mark_intent_end(_h(ctx), mid, mode, d))


# ------------------------------------------------------ scalar expressions

def apcg_expr_compile(tokens, ninputs: int, noutputs: int) -> int:
    """tokens: sequence of (op, arg, value) postfix tokens."""
    arr = (_capi.apcg_expr_token * len(tokens))(*[_capi.apcg_expr_token(int(o), int(a), float(v))
                                                  for o, a, v in tokens])
    out = ctypes.c_void_p()
    check("apcg_expr_compile", _L().apcg_expr_compile(arr, len(tokens), ninputs, noutputs, ctypes.byref(out)))
    return out.value


def apcg_expr_stats(e) -> dict:
    n, f, sh = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    check("apcg_expr_stats", _L().apcg_expr_stats(_h(e), ctypes.byref(n), ctypes.byref(f), ctypes.byref(sh)))
    return {"instructions": n.value, "folded": f.value, "shared": sh.value}


def apcg_expr_execute(e, ctx, inputs, outputs) -> None:
    ins = (ctypes.c_void_p * max(len(inputs), 1))(*[_h(i) for i in inputs])
    outs = (ctypes.c_void_p * len(outputs))(*[_h(o) for o in outputs])
    check("apcg_expr_execute", _L().apcg_expr_execute(_h(e), _h(ctx), ins, outs))


def apcg_expr_destroy(e) -> None:
    check("apcg_expr_destroy", _L().apcg_expr_destroy(_h(e)))


# ------------------------------------------------------------------ vectors

def apcg_vec_wrap(tensor) -> int:
    """Wraps a contiguous float64 GPU tensor (borrowed; keep it alive)."""
    ptr, dev = _tensor_ptr(tensor, "float64")
    out = ctypes.c_void_p()
    check("apcg_vec_wrap", _L().apcg_vec_wrap(dev, ctypes.c_void_p(ptr), tensor.numel(), ctypes.byref(out)))
    return out.value


def apcg_vec_destroy(v) -> None:
    check("apcg_vec_destroy", _L().apcg_vec_destroy(_h(v)))


def apcg_vec_dot_async(x, y, out, ctx=None) -> None:
    check("apcg_vec_dot_async", _L().apcg_vec_dot_async(_h(x), _h(y), _h(out), _h(ctx)))


def apcg_vec_norm2_async(x, out, ctx=None) -> None:
    check("apcg_vec_norm2_async", _L().apcg_vec_norm2_async(_h(x), _h(out), _h(ctx)))


def apcg_vec_axpy_async(y, a, negate: bool, x, ctx=None) -> None:
    check("apcg_vec_axpy_async", _L().apcg_vec_axpy_async(_h(y), _h(a), int(bool(negate)), _h(x), _h(ctx)))


def apcg_vec_aypx_async(y, b, x, ctx=None) -> None:
    check("apcg_vec_aypx_async", _L().apcg_vec_aypx_async(_h(y), _h(b), _h(x), _h(ctx)))


def apcg_vec_scale_async(x, a, ctx=None) -> None:
    check("apcg_vec_scale_async", _L().apcg_vec_scale_async(_h(x), _h(a), _h(ctx)))


def apcg_vec_copy_async(dst, src, ctx=None) -> None:
    check("apcg_vec_copy_async", _L().apcg_vec_copy_async(_h(dst), _h(src), _h(ctx)))


def apcg_vec_set_async(x, value: float, ctx=None) -> None:
    check("apcg_vec_set_async", _L().apcg_vec_set_async(_h(x), float(value), _h(ctx)))


def apcg_vec_copy_to_host(v, n: int):
    import numpy as np

    out = np.empty(n, dtype=np.float64)
    check("apcg_vec_copy_to_host", _L().apcg_vec_copy_to_host(_h(v), out.ctypes.data_as(ctypes.c_void_p)))
    return out


def apcg_vec_copy_from_host(v, host, ctx=None) -> None:
    import numpy as np

    host = np.ascontiguousarray(host, dtype=np.float64)
    check("apcg_vec_copy_from_host",
          _L().apcg_vec_copy_from_host(_h(v), host.ctypes.data_as(ctypes.c_void_p), _h(ctx)))


# ------------------------------------------------------------------ matrices

def apcg_mat_wrap_csr(rowptr, col, val, host_rowptr=None) -> int:
    """Wraps device CSR tensors (int32 rowptr/col, float64 val; borrowed).
    host_rowptr: optional numpy int32 copy of rowptr for validation."""
    import numpy as np

    rp, dev = _tensor_ptr(rowptr, "int32")
    n = rowptr.numel() - 1
    nnz = val.numel()
    cp = _tensor_ptr(col, "int32")[0] if nnz else 0
    vp = _tensor_ptr(val, "float64")[0] if nnz else 0
    hp = None
    if host_rowptr is not None:
        host_rowptr = np.ascontiguousarray(host_rowptr, dtype=np.int32)
        hp = host_rowptr.ctypes.data_as(ctypes.c_void_p)
    out = ctypes.c_void_p()
    check("apcg_mat_wrap_csr", _L().apcg_mat_wrap_csr(dev, n, nnz, ctypes.c_void_p(rp), ctypes.c_void_p(cp or None),
                                                      ctypes.c_void_p(vp or None), hp, ctypes.byref(out)))
    return out.value


def apcg_mat_destroy(A) -> None:
    check("apcg_mat_destroy", _L().apcg_mat_destroy(_h(A)))


def apcg_mat_mult_async(A, x, y, ctx=None) -> None:
    check("apcg_mat_mult_async", _L().apcg_mat_mult_async(_h(A), _h(x), _h(y), _h(ctx)))


def apcg_mat_set_spmv_config(A, lanes_per_row: int, block_size: int = 256, blocks: int = 0,
                             schedule: int = _capi.APCG_SPMV_ROWGROUP) -> None:
    cfg = _capi.apcg_spmv_config(lanes_per_row, block_size, blocks, schedule)
    check("apcg_mat_set_spmv_config", _L().apcg_mat_set_spmv_config(_h(A), ctypes.byref(cfg)))


def apcg_mat_get_sdia_info(A) -> dict:
    """The sliced-diagonal analysis of A (see include/apcg.h); waits for the
    device to go idle."""
    out = (ctypes.c_int32 * 6)()
    check("apcg_mat_get_sdia_info", _L().apcg_mat_get_sdia_info(_h(A), out))
    return {"state": out[0], "value_slots": out[1], "offset_slots": out[2], "plane_stride": out[3],
            "structurally_symmetric": out[4], "values_symmetric": out[5]}


def apcg_mat_get_dia_info(A) -> dict:
    """The diagonal analysis of A (see include/apcg.h); waits for the device
    to go idle."""
    out = (ctypes.c_int32 * 4)()
    check("apcg_mat_get_dia_info", _L().apcg_mat_get_dia_info(_h(A), out))
    return {"state": out[0], "diagonals": out[1], "offsets_symmetric": out[2], "values_symmetric": out[3]}


def apcg_mat_get_spmv_config(A) -> dict:
    cfg = _capi.apcg_spmv_config()
    check("apcg_mat_get_spmv_config", _L().apcg_mat_get_spmv_config(_h(A), ctypes.byref(cfg)))
    return {"lanes_per_row": cfg.lanes_per_row, "block_size": cfg.block_size, "blocks": cfg.blocks,
            "schedule": cfg.schedule}


def apcg_mat_autotune(A, ctx, reps: int = 20):
    cfg = _capi.apcg_spmv_config()
    us = ctypes.c_double()
    check("apcg_mat_autotune", _L().apcg_mat_autotune(_h(A), _h(ctx), reps, ctypes.byref(cfg), ctypes.byref(us)))
    return {"lanes_per_row": cfg.lanes_per_row, "block_size": cfg.block_size, "blocks": cfg.blocks,
            "schedule": cfg.schedule}, us.value


def apcg_mat_autotune_cached(A, ctx, reps: int = 20):
    """apcg_mat_autotune through the tuning table: (config dict, microseconds,
    True when the configuration came from the table)."""
    cfg = _capi.apcg_spmv_config()
    us = ctypes.c_double()
    hit = ctypes.c_int32()
    check("apcg_mat_autotune_cached", _L().apcg_mat_autotune_cached(_h(A), _h(ctx), reps, ctypes.byref(cfg),
                                                                    ctypes.byref(us), ctypes.byref(hit)))
    return ({"lanes_per_row": cfg.lanes_per_row, "block_size": cfg.block_size, "blocks": cfg.blocks,
             "schedule": cfg.schedule}, us.value, bool(hit.value))


def apcg_batch_autotune(ctx, A_list, b_list, x_list, kind: int = 0, iters: int = 32):
    """Times the batched solve's launch configurations (see include/apcg.h);
    returns (config dict, milliseconds, True when it came from the table).
    x_list's vectors are overwritten."""
    n = len(A_list)
    if len(b_list) != n or len(x_list) != n:
        raise ValueError("A_list, b_list and x_list must have the same length")
    arr = lambda hs: (ctypes.c_void_p * max(n, 1))(*[int(h) for h in hs])  # noqa: E731
    cfg = _capi.apcg_batch_config()
    ms = ctypes.c_double()
    hit = ctypes.c_int32()
    check("apcg_batch_autotune", _L().apcg_batch_autotune(_h(ctx), n, arr(A_list), arr(b_list), arr(x_list),
                                                          int(kind), int(iters), ctypes.byref(cfg),
                                                          ctypes.byref(ms), ctypes.byref(hit)))
    return ({"schedule": cfg.schedule, "block_size": cfg.block_size, "tile_rows": cfg.tile_rows,
             "sdia": cfg.sdia}, ms.value, bool(hit.value))


def apcg_tune_key_pattern(arch: str, rowptr, col) -> str:
    """Tuning key of host CSR arrays (numpy int32) for architecture `arch`."""
    import numpy as np

    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    n = rp.size - 1
    out = ctypes.create_string_buffer(512)
    check("apcg_tune_key_pattern", _L().apcg_tune_key_pattern(arch.encode(), n, int(rp[-1]) if n >= 0 else 0,
                                                              rp.ctypes.data_as(ctypes.c_void_p),
                                                              cl.ctypes.data_as(ctypes.c_void_p), out, 512))
    return out.value.decode()


def apcg_mat_tune_key(A) -> str:
    out = ctypes.create_string_buffer(512)
    check("apcg_mat_tune_key", _L().apcg_mat_tune_key(_h(A), out, 512))
    return out.value.decode()


def apcg_tune_cache_insert(key: str, values, us: float) -> None:
    v = (ctypes.c_int32 * 4)(*[int(x) for x in values])
    check("apcg_tune_cache_insert", _L().apcg_tune_cache_insert(key.encode(), v, float(us)))


def apcg_tune_cache_lookup(key: str):
    """(values tuple, microseconds) or None."""
    v = (ctypes.c_int32 * 4)()
    us = ctypes.c_double()
    found = ctypes.c_int32()
    check("apcg_tune_cache_lookup", _L().apcg_tune_cache_lookup(key.encode(), v, ctypes.byref(us),
                                                                ctypes.byref(found)))
    return (tuple(v), us.value) if found.value else None


def apcg_tune_cache_clear() -> None:
    check("apcg_tune_cache_clear", _L().apcg_tune_cache_clear())


def apcg_tune_cache_size() -> int:
    n = ctypes.c_int32()
    check("apcg_tune_cache_size", _L().apcg_tune_cache_size(ctypes.byref(n)))
    return n.value


def apcg_tune_cache_load(path: str) -> int:
    n = ctypes.c_int32()
    check("apcg_tune_cache_load", _L().apcg_tune_cache_load(os.fsencode(path), ctypes.byref(n)))
    return n.value


def apcg_tune_cache_save(path: str) -> int:
    n = ctypes.c_int32()
    check("apcg_tune_cache_save", _L().apcg_tune_cache_save(os.fsencode(path), ctypes.byref(n)))
    return n.value


def apcg_mat_time_kernels(A, ctx, reps: int = 100):
    """Mean microseconds per launch of the product and update kernels at
    A's SpMV configuration (back-to-back launches, HIP events)."""
    pu, uu = ctypes.c_double(), ctypes.c_double()
    check("apcg_mat_time_kernels", _L().apcg_mat_time_kernels(_h(A), _h(ctx), reps, ctypes.byref(pu), ctypes.byref(uu)))
    return pu.value, uu.value


def apcg_latency_floors(device: int = 0, reps: int = 1000) -> dict:
    """Microseconds: empty kernel back to back, per captured graph node,
    per iteration of the one-workgroup loop's synchronisation, host round
    trip (see include/apcg.h)."""
    out = (ctypes.c_double * 4)()
    check("apcg_latency_floors", _L().apcg_latency_floors(int(device), int(reps), out))
    return {"empty_kernel_us": out[0], "graph_node_us": out[1], "workgroup_iteration_us": out[2],
            "host_round_trip_us": out[3]}


# ------------------------------------------------------------------ solve

def apcg_solve_opts_default(**overrides):
    o = _capi.apcg_solve_opts()
    check("apcg_solve_opts_default", _L().apcg_solve_opts_default(ctypes.byref(o)))
    for k, v in overrides.items():
        setattr(o, k, int(v))
    return o


def apcg_info_create(device: int = 0, count: int = 1) -> int:
    out = ctypes.c_void_p()
    check("apcg_info_create", _L().apcg_info_create(device, count, ctypes.byref(out)))
    return out.value


def apcg_info_destroy(info) -> None:
    check("apcg_info_destroy", _L().apcg_info_destroy(_h(info)))


def apcg_info_get(info, index: int = 0) -> dict:
    out = _capi.apcg_solve_info()
    check("apcg_info_get", _L().apcg_info_get(_h(info), index, ctypes.byref(out)))
    return out.as_dict()


def apcg_ksp_solve(ctx, A, b, x, rtol: float, maxit: int, opts=None, info=None, info_index: int = 0) -> None:
    po = ctypes.byref(opts) if opts is not None else None
    check("apcg_ksp_solve", _L().apcg_ksp_solve(_h(ctx), _h(A), _h(b), _h(x), float(rtol), int(maxit), po, _h(info),
                                                int(info_index)))


def apcg_ksp_solve_small_noalloc(ctx, n: int, rowptr: int, col: int, val: int, b: int, x: int, rtol: float,
                                 maxit: int, opts=None, info: int = 0) -> None:
    """rowptr, col, val, b, x, info: raw device addresses (e.g. tensor.data_ptr());
    info is one apcg_solve_info record (32 bytes) of device memory."""
    po = ctypes.byref(opts) if opts is not None else None
    check("apcg_ksp_solve_small_noalloc",
          _L().apcg_ksp_solve_small_noalloc(_h(ctx), int(n), ctypes.c_void_p(int(rowptr)), ctypes.c_void_p(int(col)),
                                            ctypes.c_void_p(int(val)), ctypes.c_void_p(int(b)),
                                            ctypes.c_void_p(int(x)), float(rtol), int(maxit), po,
                                            ctypes.c_void_p(int(info))))


def apcg_ksp_solve_tfqmr(ctx, A, b, x, rtol: float, maxit: int, opts=None, info=None, info_index: int = 0) -> None:
    po = ctypes.byref(opts) if opts is not None else None
    check("apcg_ksp_solve_tfqmr", _L().apcg_ksp_solve_tfqmr(_h(ctx), _h(A), _h(b), _h(x), float(rtol), int(maxit),
                                                            po, _h(info), int(info_index)))


def apcg_ksp_solve_batched(ctx, A_list, b_list, x_list, rtol: float, maxit: int, opts=None, info=None) -> None:
    """A_list, b_list, x_list: equal-length sequences of handles."""
    n = len(A_list)
    if len(b_list) != n or len(x_list) != n:
        raise ValueError("A_list, b_list and x_list must have the same length")
    arr = lambda hs: (ctypes.c_void_p * max(n, 1))(*[int(h) for h in hs])  # noqa: E731
    po = ctypes.byref(opts) if opts is not None else None
    check("apcg_ksp_solve_batched", _L().apcg_ksp_solve_batched(_h(ctx), n, arr(A_list), arr(b_list), arr(x_list),
                                                                float(rtol), int(maxit), po, _h(info)))


# ------------------------------------------------------------------ learned preconditioner

def _dptr(t, dtype):
    import torch

    want = {"float32": torch.float32, "float64": torch.float64}[dtype]
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == want and t.is_contiguous()):
        raise TypeError(f"expected a contiguous {dtype} GPU tensor")
    return ctypes.c_void_p(t.data_ptr())


def apcg_pc_features(ctx, A, b, feat, lmax) -> None:
    """feat: float32[16], lmax: float64[1] (GPU tensors, written on ctx)."""
    check("apcg_pc_features", _L().apcg_pc_features(_h(ctx), _h(A), _h(b), _dptr(feat, "float32"),
                                                    _dptr(lmax, "float64")))


def apcg_pc_label(ctx, A, b, rtol: float, maxit: int, G, h, label) -> None:
    """G: float32[81], h: float32[9], label: float64[3] = (lmin, a, lmax)."""
    check("apcg_pc_label", _L().apcg_pc_label(_h(ctx), _h(A), _h(b), float(rtol), int(maxit), _dptr(G, "float32"),
                                              _dptr(h, "float32"), _dptr(label, "float64")))


def apcg_mlp_standardize(ctx, X, mean, std, compute_stats: bool) -> None:
    check("apcg_mlp_standardize", _L().apcg_mlp_standardize(_h(ctx), _dptr(X, "float32"), X.shape[0],
                                                            _dptr(mean, "float32"), _dptr(std, "float32"),
                                                            int(bool(compute_stats))))


def apcg_mlp_forward(ctx, params, X, C) -> None:
    check("apcg_mlp_forward", _L().apcg_mlp_forward(_h(ctx), _dptr(params, "float32"), _dptr(X, "float32"),
                                                    X.shape[0], _dptr(C, "float32")))


def apcg_mlp_loss_grad(ctx, params, X, G, h, loss, grad, mu=1.0, eps=0.05) -> None:
    check("apcg_mlp_loss_grad", _L().apcg_mlp_loss_grad(_h(ctx), _dptr(params, "float32"), _dptr(X, "float32"),
                                                        _dptr(G, "float32"), _dptr(h, "float32"), X.shape[0],
                                                        float(mu), float(eps), _dptr(loss, "float32"),
                                                        _dptr(grad, "float32")))


def apcg_mlp_train_step(ctx, params, m, v, t: int, lr: float, X, G, h, loss, mu=1.0, eps=0.05) -> None:
    check("apcg_mlp_train_step", _L().apcg_mlp_train_step(_h(ctx), _dptr(params, "float32"), _dptr(m, "float32"),
                                                          _dptr(v, "float32"), int(t), float(lr),
                                                          _dptr(X, "float32"), _dptr(G, "float32"),
                                                          _dptr(h, "float32"), X.shape[0], float(mu), float(eps),
                                                          _dptr(loss, "float32")))


def apcg_fcg_opts_default(**overrides):
    o = _capi.apcg_fcg_opts()
    check("apcg_fcg_opts_default", _L().apcg_fcg_opts_default(ctypes.byref(o)))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def apcg_ksp_solve_fcg_poly(ctx, A, b, x, rtol: float, maxit: int, coeffs, lmax, opts=None, fopts=None,
                            info=None, info_index: int = 0) -> None:
    """coeffs: float32[9] GPU tensor, lmax: float64[1] GPU tensor."""
    po = ctypes.byref(opts) if opts is not None else None
    pf = ctypes.byref(fopts) if fopts is not None else None
    check("apcg_ksp_solve_fcg_poly", _L().apcg_ksp_solve_fcg_poly(_h(ctx), _h(A), _h(b), _h(x), float(rtol),
                                                                  int(maxit), _dptr(coeffs, "float32"),
                                                                  _dptr(lmax, "float64"), po, pf, _h(info),
                                                                  int(info_index)))


def apcg_ksp_solve_learned(ctx, A, b, x, rtol: float, maxit: int, params, mean, std, opts=None, fopts=None,
                           info=None, info_index: int = 0) -> None:
    """params: float32[5833], mean / std: float32[16] GPU tensors."""
    po = ctypes.byref(opts) if opts is not None else None
    pf = ctypes.byref(fopts) if fopts is not None else None
    check("apcg_ksp_solve_learned", _L().apcg_ksp_solve_learned(_h(ctx), _h(A), _h(b), _h(x), float(rtol),
                                                                int(maxit), _dptr(params, "float32"),
                                                                _dptr(mean, "float32"), _dptr(std, "float32"),
                                                                po, pf, _h(info), int(info_index)))


def apcg_ksp_solve_batched_fcg_poly(ctx, A_list, b_list, x_list, rtol: float, maxit: int, coeffs, lmax, opts=None,
                                    fopts=None, info=None) -> None:
    """coeffs: float32[nsys * 9], lmax: float64[nsys] GPU tensors."""
    n = len(A_list)
    if len(b_list) != n or len(x_list) != n:
        raise ValueError("A_list, b_list and x_list must have the same length")
    arr = lambda hs: (ctypes.c_void_p * max(n, 1))(*[int(h) for h in hs])  # noqa: E731
    po = ctypes.byref(opts) if opts is not None else None
    pf = ctypes.byref(fopts) if fopts is not None else None
    check("apcg_ksp_solve_batched_fcg_poly",
          _L().apcg_ksp_solve_batched_fcg_poly(_h(ctx), n, arr(A_list), arr(b_list), arr(x_list), float(rtol),
                                               int(maxit), _dptr(coeffs, "float32"), _dptr(lmax, "float64"), po, pf,
                                               _h(info)))


def apcg_pc_features_batched(ctx, A_list, b_list, feat, lmax) -> None:
    """feat: float32[nsys * 16], lmax: float64[nsys] GPU tensors (written on ctx)."""
    n = len(A_list)
    if len(b_list) != n:
        raise ValueError("A_list and b_list must have the same length")
    arr = lambda hs: (ctypes.c_void_p * max(n, 1))(*[int(h) for h in hs])  # noqa: E731
    check("apcg_pc_features_batched", _L().apcg_pc_features_batched(_h(ctx), n, arr(A_list), arr(b_list),
                                                                    _dptr(feat, "float32"), _dptr(lmax, "float64")))


def apcg_ksp_solve_batched_learned(ctx, A_list, b_list, x_list, rtol: float, maxit: int, params, mean, std,
                                   opts=None, fopts=None, info=None) -> None:
    """params: float32[5833], mean / std: float32[16] GPU tensors."""
    n = len(A_list)
    if len(b_list) != n or len(x_list) != n:
        raise ValueError("A_list, b_list and x_list must have the same length")
    arr = lambda hs: (ctypes.c_void_p * max(n, 1))(*[int(h) for h in hs])  # noqa: E731
    po = ctypes.byref(opts) if opts is not None else None
    pf = ctypes.byref(fopts) if fopts is not None else None
    check("apcg_ksp_solve_batched_learned",
          _L().apcg_ksp_solve_batched_learned(_h(ctx), n, arr(A_list), arr(b_list), arr(x_list), float(rtol),
                                              int(maxit), _dptr(params, "float32"), _dptr(mean, "float32"),
                                              _dptr(std, "float32"), po, pf, _h(info)))


# ------------------------------------------------------------------ timers

def apcg_timer_create() -> int:
    out = ctypes.c_void_p()
    check("apcg_timer_create", _L().apcg_timer_create(ctypes.byref(out)))
    return out.value


def apcg_timer_destroy(t) -> None:
    check("apcg_timer_destroy", _L().apcg_timer_destroy(_h(t)))


def apcg_timer_start(t, ctx) -> None:
    check("apcg_timer_start", _L().apcg_timer_start(_h(t), _h(ctx)))


def apcg_timer_stop(t, ctx) -> None:
    check("apcg_timer_stop", _L().apcg_timer_stop(_h(t), _h(ctx)))


def apcg_timer_elapsed_ms(t) -> float:
    out = ctypes.c_double()
    check("apcg_timer_elapsed_ms", _L().apcg_timer_elapsed_ms(_h(t), ctypes.byref(out)))
    return out.value
