"""ctypes declarations of the apcg C ABI (include/apcg.h).

Argument marshalling only: every function here has the name of the C entry
point it calls, takes Python values and handles instead of out-pointers,
returns the outputs, and raises ApcgError on a non-zero status.  No step of
the solver runs in Python.

PyTorch is imported before the library is loaded so that the HIP runtime
PyTorch ships is the one the library binds to (both carry the same soname);
loading the library first would put two HIP runtimes into the process.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libapcg.so")

c_i32, c_i64, c_f64, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
c_char_p = ctypes.c_char_p

# constants (mirror include/apcg.h)
APCG_SUCCESS = 0
APCG_ERR_INVALID_ARG = 1
APCG_ERR_INVALID_STATE = 2
APCG_ERR_HIP = 3
APCG_ERR_OUT_OF_MEMORY = 4
APCG_ERR_UNSUPPORTED = 5

APCG_SOLVE_RUNNING = 0
APCG_SOLVE_CONVERGED = 1
APCG_SOLVE_MAXIT = 2
APCG_SOLVE_BREAKDOWN_PAP = 4
APCG_SOLVE_BREAKDOWN_RZ = 8
APCG_SOLVE_NAN = 16
APCG_SOLVE_STALL = 32
APCG_SOLVE_FALLBACK = 64
APCG_SOLVE_SETUP_ERROR = 128

APCG_STREAM_DEFAULT = 0
APCG_STREAM_GLOBAL_BLOCKING = 1
APCG_JOIN_DESTROY = 0
APCG_JOIN_SYNC = 1
APCG_JOIN_NO_SYNC = 2

APCG_SCALAR_COPY = 0
APCG_SCALAR_NEG = 1
APCG_SCALAR_RECIP = 2
APCG_SCALAR_SQRT = 3
APCG_SCALAR_ADD = 4
APCG_SCALAR_SUB = 5
APCG_SCALAR_MUL = 6
APCG_SCALAR_DIV = 7

APCG_PC_NONE = 0
APCG_PC_JACOBI = 1
APCG_NORM_UNPRECONDITIONED = 0
APCG_NORM_PRECONDITIONED = 1
APCG_MODE_GRAPH = 0
APCG_MODE_STREAM = 1
APCG_MODE_HOST_CHECK = 2
APCG_MODE_PERSISTENT = 3
APCG_MODE_AUTO = 4
APCG_PERSISTENT_MAX_N = 4096
APCG_NOALLOC_MAX_N = 4096
APCG_SPMV_ROWGROUP = 0
APCG_SPMV_STREAM = 1
APCG_SPMV_SELL = 2
APCG_SPMV_SDIA = 3
APCG_SPMV_DIA = 4
APCG_BATCH_AUTO = 0
APCG_BATCH_PERSISTENT = 1
APCG_BATCH_SEGMENTED = 2


class apcg_spmv_config(ctypes.Structure):
    _fields_ = [("lanes_per_row", c_i32), ("block_size", c_i32), ("blocks", c_i32), ("schedule", c_i32)]


class apcg_batch_config(ctypes.Structure):
    _fields_ = [("schedule", c_i32), ("block_size", c_i32), ("tile_rows", c_i32), ("sdia", c_i32)]


class apcg_solve_opts(ctypes.Structure):
    _fields_ = [("pc", c_i32), ("norm_type", c_i32), ("mode", c_i32), ("iters_per_graph", c_i32),
                ("lookahead", c_i32), ("x0_is_zero", c_i32), ("kernel_timing", c_i32),
                ("batch_block_size", c_i32), ("batch_schedule", c_i32), ("batch_tile_rows", c_i32),
                ("batch_tail_tile_rows", c_i32), ("reserved", c_i32 * 5)]


class apcg_solve_info(ctypes.Structure):
    _fields_ = [("iterations", c_i32), ("status", c_i32), ("fcg_iterations", c_i32), ("half_steps", c_i32),
                ("res_norm", c_f64), ("ref_norm", c_f64)]

    def as_dict(self):
        return {"iterations": self.iterations, "status": self.status, "fcg_iterations": self.fcg_iterations,
                "half_steps": self.half_steps, "res_norm": self.res_norm, "ref_norm": self.ref_norm}


class apcg_fcg_opts(ctypes.Structure):
    _fields_ = [("stall_min", c_i32), ("fallback", c_i32), ("stall_frac", c_f64), ("reserved", c_i32 * 4)]


class apcg_counters(ctypes.Structure):
    _fields_ = [("kernel_launches", c_i64), ("graph_launches", c_i64), ("host_syncs", c_i64),
                ("host_polls", c_i64), ("d2h_copies", c_i64), ("h2d_copies", c_i64), ("stream_waits", c_i64),
                ("reserved", c_i64 * 9)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class apcg_device_props(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 64), ("arch", ctypes.c_char * 32), ("compute_units", c_i32),
                ("wavefront_size", c_i32), ("global_mem_bytes", c_i64), ("clock_khz", c_i32),
                ("l2_bytes", c_i32), ("lds_bytes_per_block", c_i32), ("reserved", c_i32 * 7)]


APCG_ACCESS_READ = 1
APCG_ACCESS_WRITE = 2
APCG_ACCESS_READ_WRITE = 3
APCG_EXPR_INPUT = 1
APCG_EXPR_CONST = 2
APCG_EXPR_NEG = 10
APCG_EXPR_RECIP = 11
APCG_EXPR_SQRT = 12
APCG_EXPR_ABS = 13
APCG_EXPR_EXP = 14
APCG_EXPR_LOG = 15
APCG_EXPR_SIN = 16
APCG_EXPR_COS = 17
APCG_EXPR_ADD = 20
APCG_EXPR_SUB = 21
APCG_EXPR_MUL = 22
APCG_EXPR_DIV = 23
APCG_EXPR_MIN = 24
APCG_EXPR_MAX = 25
APCG_EXPR_OUTPUT = 30


class apcg_expr_token(ctypes.Structure):
    _fields_ = [("op", c_i32), ("arg", c_i32), ("value", c_f64)]


P = ctypes.POINTER
# name -> argtypes (restype apcg_status unless listed in _RESTYPE)
SIGNATURES = {
    "apcg_abi_version": [],
    "apcg_ctx_get_stream": [c_vp, P(c_vp)],
    "apcg_memory_register": [c_i32, c_vp, c_i64, P(ctypes.c_uint64)],
    "apcg_memory_lookup": [c_i32, c_vp, P(ctypes.c_uint64), P(c_vp), P(c_i64)],
    "apcg_memory_unregister": [ctypes.c_uint64],
    "apcg_vec_get_id": [c_vp, P(ctypes.c_uint64)],
    "apcg_scalar_get_id": [c_vp, P(ctypes.c_uint64)],
    "apcg_mat_get_id": [c_vp, P(ctypes.c_uint64)],
    "apcg_mark_intent_begin": [c_vp, ctypes.c_uint64, c_i32, ctypes.c_char_p],
    "apcg_mark_intent_end": [c_vp, ctypes.c_uint64, c_i32, ctypes.c_char_p],
    "apcg_expr_compile": [P(apcg_expr_token), c_i32, c_i32, c_i32, P(c_vp)],
    "apcg_expr_stats": [c_vp, P(c_i32), P(c_i32), P(c_i32)],
    "apcg_expr_execute": [c_vp, c_vp, P(c_vp), P(c_vp)],
    "apcg_expr_destroy": [c_vp],
    "apcg_last_error": [],
    "apcg_device_count": [P(c_i32)],
    "apcg_device_props_get": [c_i32, P(apcg_device_props)],
    "apcg_ctx_create": [c_i32, c_i32, P(c_vp)],
    "apcg_ctx_destroy": [c_vp],
    "apcg_ctx_wait_for": [c_vp, c_vp],
    "apcg_ctx_query_idle": [c_vp, P(c_i32)],
    "apcg_ctx_synchronize": [c_vp],
    "apcg_ctx_fork": [c_vp, c_i32, P(c_vp)],
    "apcg_ctx_join": [c_vp, c_i32, c_i32, P(c_vp)],
    "apcg_ctx_get_stream_type": [c_vp, P(c_i32)],
    "apcg_scalar_create": [c_vp, P(c_vp)],
    "apcg_scalar_destroy": [c_vp],
    "apcg_scalar_set": [c_vp, c_f64, c_vp],
    "apcg_scalar_get": [c_vp, P(c_f64)],
    "apcg_scalar_op": [c_i32, c_vp, c_vp, c_vp, c_vp],
    "apcg_vec_wrap": [c_i32, c_vp, c_i64, P(c_vp)],
    "apcg_vec_destroy": [c_vp],
    "apcg_vec_dot_async": [c_vp, c_vp, c_vp, c_vp],
    "apcg_vec_norm2_async": [c_vp, c_vp, c_vp],
    "apcg_vec_axpy_async": [c_vp, c_vp, c_i32, c_vp, c_vp],
    "apcg_vec_aypx_async": [c_vp, c_vp, c_vp, c_vp],
    "apcg_vec_scale_async": [c_vp, c_vp, c_vp],
    "apcg_vec_copy_async": [c_vp, c_vp, c_vp],
    "apcg_vec_set_async": [c_vp, c_f64, c_vp],
    "apcg_vec_copy_to_host": [c_vp, c_vp],
    "apcg_vec_copy_from_host": [c_vp, c_vp, c_vp],
    "apcg_mat_wrap_csr": [c_i32, c_i32, c_i64, c_vp, c_vp, c_vp, c_vp, P(c_vp)],
    "apcg_mat_destroy": [c_vp],
    "apcg_mat_mult_async": [c_vp, c_vp, c_vp, c_vp],
    "apcg_mat_set_spmv_config": [c_vp, P(apcg_spmv_config)],
    "apcg_mat_get_spmv_config": [c_vp, P(apcg_spmv_config)],
    "apcg_mat_get_sdia_info": [c_vp, P(c_i32)],
    "apcg_mat_get_dia_info": [c_vp, P(c_i32)],
    "apcg_mat_autotune": [c_vp, c_vp, c_i32, P(apcg_spmv_config), P(c_f64)],
    "apcg_mat_time_kernels": [c_vp, c_vp, c_i32, P(c_f64), P(c_f64)],
    "apcg_latency_floors": [c_i32, c_i32, P(c_f64)],
    "apcg_tune_key_pattern": [c_char_p, c_i32, c_i64, c_vp, c_vp, c_char_p, c_i32],
    "apcg_mat_tune_key": [c_vp, c_char_p, c_i32],
    "apcg_tune_cache_insert": [c_char_p, P(c_i32), c_f64],
    "apcg_tune_cache_lookup": [c_char_p, P(c_i32), P(c_f64), P(c_i32)],
    "apcg_tune_cache_clear": [],
    "apcg_tune_cache_size": [P(c_i32)],
    "apcg_tune_cache_load": [c_char_p, P(c_i32)],
    "apcg_tune_cache_save": [c_char_p, P(c_i32)],
    "apcg_mat_autotune_cached": [c_vp, c_vp, c_i32, P(apcg_spmv_config), P(c_f64), P(c_i32)],
    "apcg_batch_autotune": [c_vp, c_i32, c_vp, c_vp, c_vp, c_i32, c_i32, P(apcg_batch_config), P(c_f64), P(c_i32)],
    "apcg_ksp_solve_small_noalloc": [c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_f64, c_i32, P(apcg_solve_opts),
                                     c_vp],
    "apcg_solve_opts_default": [P(apcg_solve_opts)],
    "apcg_info_create": [c_i32, c_i32, P(c_vp)],
    "apcg_info_destroy": [c_vp],
    "apcg_info_get": [c_vp, c_i32, P(apcg_solve_info)],
    "apcg_ksp_solve": [c_vp, c_vp, c_vp, c_vp, c_f64, c_i32, P(apcg_solve_opts), c_vp, c_i32],
    "apcg_ksp_solve_tfqmr": [c_vp, c_vp, c_vp, c_vp, c_f64, c_i32, P(apcg_solve_opts), c_vp, c_i32],
    "apcg_ksp_solve_batched": [c_vp, c_i32, P(c_vp), P(c_vp), P(c_vp), c_f64, c_i32, P(apcg_solve_opts), c_vp],
    "apcg_ctx_kernel_times": [c_vp, c_i32, P(c_f64), P(c_i32)],
    "apcg_pc_features": [c_vp, c_vp, c_vp, c_vp, c_vp],
    "apcg_pc_label": [c_vp, c_vp, c_vp, c_f64, c_i32, c_vp, c_vp, c_vp],
    "apcg_mlp_standardize": [c_vp, c_vp, c_i32, c_vp, c_vp, c_i32],
    "apcg_mlp_forward": [c_vp, c_vp, c_vp, c_i32, c_vp],
    "apcg_mlp_loss_grad": [c_vp, c_vp, c_vp, c_vp, c_vp, c_i32, ctypes.c_float, ctypes.c_float, c_vp, c_vp],
    "apcg_mlp_train_step": [c_vp, c_vp, c_vp, c_vp, c_i32, ctypes.c_float, c_vp, c_vp, c_vp, c_i32, ctypes.c_float,
                            ctypes.c_float, c_vp],
    "apcg_fcg_opts_default": [P(apcg_fcg_opts)],
    "apcg_ksp_solve_fcg_poly": [c_vp, c_vp, c_vp, c_vp, c_f64, c_i32, c_vp, c_vp, P(apcg_solve_opts),
                                P(apcg_fcg_opts), c_vp, c_i32],
    "apcg_ksp_solve_batched_fcg_poly": [c_vp, c_i32, c_vp, c_vp, c_vp, c_f64, c_i32, c_vp, c_vp, P(apcg_solve_opts),
                                        P(apcg_fcg_opts), c_vp],
    "apcg_pc_features_batched": [c_vp, c_i32, c_vp, c_vp, c_vp, c_vp],
    "apcg_ksp_solve_batched_learned": [c_vp, c_i32, c_vp, c_vp, c_vp, c_f64, c_i32, c_vp, c_vp, c_vp,
                                       P(apcg_solve_opts), P(apcg_fcg_opts), c_vp],
    "apcg_ksp_solve_learned": [c_vp, c_vp, c_vp, c_vp, c_f64, c_i32, c_vp, c_vp, c_vp, P(apcg_solve_opts),
                               P(apcg_fcg_opts), c_vp, c_i32],
    "apcg_timer_create": [P(c_vp)],
    "apcg_timer_destroy": [c_vp],
    "apcg_timer_start": [c_vp, c_vp],
    "apcg_timer_stop": [c_vp, c_vp],
    "apcg_timer_elapsed_ms": [c_vp, P(c_f64)],
    "apcg_counters_get": [P(apcg_counters)],
    "apcg_counters_reset": [],
}
_RESTYPE = {"apcg_abi_version": c_i32, "apcg_last_error": ctypes.c_char_p}


class ApcgError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} failed with status {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Loads libapcg.so (after torch); raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  -- binds the library to torch's HIP runtime

    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in SIGNATURES.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = _RESTYPE.get(name, c_i32)
    _lib = lib
    return lib


def check(fn: str, status: int):
    if status != APCG_SUCCESS:
        msg = load().apcg_last_error()
        raise ApcgError(fn, status, msg.decode() if msg else "")
