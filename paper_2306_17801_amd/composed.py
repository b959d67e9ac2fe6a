"""Jacobi-preconditioned CG composed from the library's asynchronous
primitives, the way Section 3.3 writes KSPSolve_CG with the stream-aware
calls: MatMult, VecDot, VecNorm, AXPY, AYPX and scalar arithmetic, every
scalar a device-resident value that is never read back until the end.

This is the programming-model demonstration, not the fast path (the fused
solve, apcg_ksp_solve, does the same iteration in two kernels).  With
``sync=True`` the result of every inner product is read to the host before
the next call is made: the synchronous shape of the paper's baseline
(Section 4, "main_gpu"), where each reduction blocks the host.

The preconditioner is applied as a copy plus a scaling by the device scalar
1 / diag, so the matrix must have a constant diagonal ``diag`` (the paper's
constant-coefficient Laplace benchmarks do): then z = D^-1 r exactly.
"""
from __future__ import annotations

from . import _capi
from . import (apcg_mat_mult_async, apcg_scalar_create, apcg_scalar_destroy, apcg_scalar_get, apcg_scalar_op,
               apcg_scalar_set, apcg_vec_axpy_async, apcg_vec_aypx_async, apcg_vec_copy_async, apcg_vec_dot_async,
               apcg_vec_norm2_async, apcg_vec_scale_async)


class ComposedCG:
    """Work vectors and device scalars for repeated solves of one size."""

    def __init__(self, ctx, n: int, device: int = 0):
        from .device import DeviceVec

        self.ctx = ctx
        self.n = n
        self.r, self.z, self.p, self.w = (DeviceVec.zeros(n, device) for _ in range(4))
        names = ("rho", "rho_new", "delta", "alpha", "beta", "res", "diag", "dinv")
        self.s = {k: apcg_scalar_create(ctx) for k in names}

    def close(self):
        for v in (self.r, self.z, self.p, self.w):
            v.close()
        for h in self.s.values():
            apcg_scalar_destroy(h)
        self.s = {}

    def solve(self, A, b, x, diag: float, iters: int, sync: bool = False) -> float:
        """iters iterations from x0 = 0 (x must hold zeros); returns the
        2-norm of the last residual (read on the host, the one blocking call
        of the asynchronous variant)."""
        c, s = self.ctx, self.s
        r, z, p, w = self.r.h, self.z.h, self.p.h, self.w.h
        apcg_scalar_set(s["diag"], diag, c)
        apcg_scalar_op(_capi.APCG_SCALAR_RECIP, s["dinv"], s["diag"], None, c)  # 1/diag on the device
        apcg_vec_copy_async(r, b, c)  # r = b - A x0 with x0 = 0
        apcg_vec_copy_async(z, r, c)
        apcg_vec_scale_async(z, s["dinv"], c)  # z = D^-1 r
        apcg_vec_copy_async(p, z, c)
        apcg_vec_dot_async(r, z, s["rho"], c)
        if sync:
            apcg_scalar_get(s["rho"])
        for _ in range(iters):
            apcg_mat_mult_async(A, p, w, c)
            apcg_vec_dot_async(p, w, s["delta"], c)
            if sync:
                apcg_scalar_get(s["delta"])
            apcg_scalar_op(_capi.APCG_SCALAR_DIV, s["alpha"], s["rho"], s["delta"], c)
            apcg_vec_axpy_async(x, s["alpha"], False, p, c)  # x += alpha p
            apcg_vec_axpy_async(r, s["alpha"], True, w, c)  # r -= alpha w
            apcg_vec_copy_async(z, r, c)
            apcg_vec_scale_async(z, s["dinv"], c)
            apcg_vec_dot_async(r, z, s["rho_new"], c)
            apcg_vec_norm2_async(r, s["res"], c)
            if sync:
                apcg_scalar_get(s["rho_new"])
                apcg_scalar_get(s["res"])
            apcg_scalar_op(_capi.APCG_SCALAR_DIV, s["beta"], s["rho_new"], s["rho"], c)
            apcg_scalar_op(_capi.APCG_SCALAR_COPY, s["rho"], s["rho_new"], None, c)
            apcg_vec_aypx_async(p, s["beta"], z, c)  # p = z + beta p
        return apcg_scalar_get(s["res"])
