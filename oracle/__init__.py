"""CPU oracle for the asynchronous PCG hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the package smoke check and the CPU-baseline leg of the
benchmark may import this package.  The product path (the HIP library and
its Python binding) never imports, loads or calls it, and this package never
imports the product package.

The numeric core is ``apcg_oracle.c`` (plain serial FP64 C, built with gcc
into ``liboracle.so`` by :func:`build`).  This module adds ctypes marshalling
and the small dense steps written in numpy: the CG-Lanczos tridiagonal and its
eigenvalues, Chebyshev helper polynomials and the FP64 MLP used to check the
learned-preconditioner kernels.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "apcg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_SRC_T = os.path.join(_HERE, "oracle_threads.c")
_LIB_T = os.path.join(_HERE, "liboracle_threads.so")

# status bits, as numbered inside apcg_oracle.c
CONVERGED = 1
MAXIT = 2
BREAKDOWN_PAP = 4
BREAKDOWN_RZ = 8
NAN = 16
STALL = 32
FALLBACK = 64
SETUP_ERROR = 128

PC_NONE = 0
PC_JACOBI = 1
NORM_UNPRECONDITIONED = 0
NORM_PRECONDITIONED = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
               "-Wall", "-Wno-jump-misses-init", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    if force or not os.path.exists(_LIB_T) or os.path.getmtime(_LIB_T) < os.path.getmtime(_SRC_T):
        tmp = _LIB_T + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-Wall", _SRC_T, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_T)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, f64 = ctypes.c_int32, ctypes.c_double
        L.or_spmv.argtypes = [i32, P, P, P, P, P]
        L.or_spmv.restype = None
        L.or_dot.argtypes = [ctypes.c_int64, P, P]
        L.or_dot.restype = f64
        L.or_norm2.argtypes = [ctypes.c_int64, P]
        L.or_norm2.restype = f64
        L.or_jacobi_inverse.argtypes = [i32, P, P, P, P]
        L.or_jacobi_inverse.restype = i32
        L.or_gershgorin.argtypes = [i32, P, P, P, P, P]
        L.or_gershgorin.restype = i32
        L.or_pcg.argtypes = [i32, P, P, P, P, P, f64, i32, i32, i32, P, P, P, P, P, P, P, i32]
        L.or_pcg.restype = i32
        L.or_poly_apply.argtypes = [i32, P, P, P, P, f64, i32, P, P, P]
        L.or_poly_apply.restype = i32
        L.or_tfqmr.argtypes = [i32, P, P, P, P, P, i32, f64, i32, i32, P, P, P, P, P]
        L.or_tfqmr.restype = i32
        L.or_fcg_poly.argtypes = [i32, P, P, P, P, P, f64, i32, i32, P, f64, i32, f64, i32, i32, P, P, P, P]
        L.or_fcg_poly.restype = i32
        _lib = L
    return _lib


_lib_t = None


def lib_threads():
    """The threaded timing copy of the Jacobi-PCG loop (oracle_threads.c)."""
    global _lib_t
    if _lib_t is None:
        if not os.path.exists(_LIB_T) or os.path.getmtime(_LIB_T) < os.path.getmtime(_SRC_T):
            build(force=True)
        L = ctypes.CDLL(_LIB_T)
        P = ctypes.c_void_p
        i32, f64 = ctypes.c_int32, ctypes.c_double
        L.or_pcg_threads.argtypes = [i32, P, P, P, P, P, f64, i32, i32, P, P, P]
        L.or_pcg_threads.restype = i32
        _lib_t = L
    return _lib_t


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _csr(A):
    rp = np.ascontiguousarray(A.rowptr, dtype=np.int32)
    c = np.ascontiguousarray(A.col, dtype=np.int32)
    v = np.ascontiguousarray(A.val, dtype=np.float64)
    return rp, c, v


def spmv(A, x):
    rp, c, v = _csr(A)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(A.n, dtype=np.float64)
    lib().or_spmv(A.n, _p(rp), _p(c), _p(v), _p(x), _p(y))
    return y


def dot(x, y):
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    return float(lib().or_dot(x.size, _p(x), _p(y)))


def norm2(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    return float(lib().or_norm2(x.size, _p(x)))


def jacobi_inverse(A):
    rp, c, v = _csr(A)
    d = np.empty(A.n, dtype=np.float64)
    if lib().or_jacobi_inverse(A.n, _p(rp), _p(c), _p(v), _p(d)) != 0:
        raise ValueError("missing or non-positive diagonal entry")
    return d


def gershgorin(A):
    rp, c, v = _csr(A)
    lo, hi = ctypes.c_double(), ctypes.c_double()
    if lib().or_gershgorin(A.n, _p(rp), _p(c), _p(v), ctypes.byref(lo), ctypes.byref(hi)) != 0:
        raise ValueError("zero diagonal entry")
    return lo.value, hi.value


class PCGResult:
    def __init__(self, **kw):
        self.__dict__.update(kw)

    def __repr__(self):
        return f"PCGResult(status={self.status}, its={self.its}, res={self.res:.3e}, ref={self.ref:.3e})"


def pcg(A, b, x0=None, rtol=1e-8, maxit=None, pc=PC_JACOBI, norm_type=NORM_UNPRECONDITIONED,
        history=False, ndir=0):
    """Jacobi-PCG / CG (see or_pcg in apcg_oracle.c).  Returns PCGResult with
    x, its, status, res, ref and, with ``history``, alpha/beta/res per
    iteration; ``ndir`` > 0 also returns the first search directions."""
    rp, c, v = _csr(A)
    n = A.n
    maxit = n if maxit is None else int(maxit)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    its = ctypes.c_int32()
    res, ref = ctypes.c_double(), ctypes.c_double()
    ah = np.zeros(max(maxit, 1)) if history else None
    bh = np.zeros(max(maxit, 1)) if history else None
    rh = np.zeros(max(maxit, 1)) if history else None
    dh = np.zeros((ndir, n)) if ndir > 0 else None
    st = lib().or_pcg(n, _p(rp), _p(c), _p(v), _p(b), _p(x), float(rtol), maxit, int(pc), int(norm_type),
                      ctypes.byref(its), ctypes.byref(res), ctypes.byref(ref), _p(ah), _p(bh), _p(rh),
                      _p(dh), int(ndir))
    out = PCGResult(x=x, its=its.value, status=st, res=res.value, ref=ref.value)
    if history:
        k = its.value
        out.alpha = ah[:k].copy()
        out.beta = bh[:k].copy()
        out.res_hist = rh[:k].copy()
    if ndir > 0:
        out.dirs = dh[: min(ndir, max(its.value, 0) + 1)].copy()
    return out


def pcg_threads(A, b, rtol=1e-8, maxit=None, threads=1):
    """Jacobi-PCG from x0 = 0 with its row loops on ``threads`` host threads
    (or_pcg_threads; for timing the host).  With one thread it equals
    :func:`pcg` bit for bit."""
    rp, c, v = _csr(A)
    n = A.n
    maxit = n if maxit is None else int(maxit)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(n)
    its = ctypes.c_int32()
    res, ref = ctypes.c_double(), ctypes.c_double()
    st = lib_threads().or_pcg_threads(n, _p(rp), _p(c), _p(v), _p(b), _p(x), float(rtol), maxit, int(threads),
                                      ctypes.byref(its), ctypes.byref(res), ctypes.byref(ref))
    return PCGResult(x=x, its=its.value, status=st, res=res.value, ref=ref.value)


def host_threads() -> int:
    """Host threads for CPU timing: the CPUs this process may run on, capped
    at 16 (the host share that goes with one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def tfqmr(A, b, x0=None, rtol=1e-8, maxit=None, pc=PC_JACOBI, history=False):
    """TFQMR, left-preconditioned by D^{-1} (see or_tfqmr in apcg_oracle.c).
    Returns PCGResult with x, its (iterations, two products each), half
    (half-steps), status, res (the quasi-residual bound tau sqrt(m + 1) of
    the last half-step) and ref (||D^{-1} (b - A x0)||); with ``history``
    also tau after every half-step."""
    rp, c, v = _csr(A)
    n = A.n
    maxit = n if maxit is None else int(maxit)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    its, half = ctypes.c_int32(), ctypes.c_int32()
    res, ref = ctypes.c_double(), ctypes.c_double()
    th = np.zeros(max(2 * maxit, 1)) if history else None
    st = lib().or_tfqmr(n, _p(rp), _p(c), _p(v), _p(b), _p(x), 1 if x0 is None else 0, float(rtol), maxit, int(pc),
                        ctypes.byref(its), ctypes.byref(half), ctypes.byref(res), ctypes.byref(ref), _p(th))
    out = PCGResult(x=x, its=its.value, half=half.value, status=st, res=res.value, ref=ref.value)
    if history:
        out.tau = th[: half.value].copy()
    return out


def poly_apply(A, dinv, lmax, coeffs, r):
    rp, c, v = _csr(A)
    coeffs = np.ascontiguousarray(coeffs, dtype=np.float64)
    dinv = np.ascontiguousarray(dinv, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    z = np.empty(A.n)
    if lib().or_poly_apply(A.n, _p(rp), _p(c), _p(v), _p(dinv), float(lmax), coeffs.size - 1, _p(coeffs),
                           _p(r), _p(z)) != 0:
        raise MemoryError
    return z


def fcg_poly(A, b, coeffs, lmax, x0=None, rtol=1e-8, maxit=None, stall_min=50, stall_frac=0.1,
             fallback=True, precheck=True):
    """FCG(1) with the Chebyshev polynomial preconditioner, the positivity
    pre-check and the Jacobi-PCG fallback (see or_fcg_poly)."""
    rp, c, v = _csr(A)
    n = A.n
    maxit = n if maxit is None else int(maxit)
    coeffs = np.ascontiguousarray(coeffs, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    its, fits = ctypes.c_int32(), ctypes.c_int32()
    res, ref = ctypes.c_double(), ctypes.c_double()
    st = lib().or_fcg_poly(n, _p(rp), _p(c), _p(v), _p(b), _p(x), float(rtol), maxit, coeffs.size - 1,
                           _p(coeffs), float(lmax), int(stall_min), float(stall_frac), int(bool(fallback)),
                           int(bool(precheck)), ctypes.byref(its), ctypes.byref(res), ctypes.byref(ref),
                           ctypes.byref(fits))
    return PCGResult(x=x, its=its.value, fcg_its=fits.value, status=st, res=res.value, ref=ref.value)


# ---------------------------------------------------------------------------
# Dense steps (numpy)
# ---------------------------------------------------------------------------

def lanczos_tridiagonal(alpha, beta):
    """Symmetric tridiagonal T_m of the Lanczos process that PCG runs
    implicitly (CG-Lanczos relation, Saad, Iterative Methods for Sparse
    Linear Systems, 2nd ed., Sec. 6.7.3):
        T[j, j]   = 1/alpha_j + beta_{j-1}/alpha_{j-1}   (beta_{-1} = 0)
        T[j, j+1] = sqrt(beta_j) / alpha_j
    built from the first m = len(alpha) coefficients."""
    alpha = np.asarray(alpha, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    m = alpha.size
    T = np.zeros((m, m))
    for j in range(m):
        T[j, j] = 1.0 / alpha[j] + (beta[j - 1] / alpha[j - 1] if j > 0 else 0.0)
        if j + 1 < m:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(beta[j]) / alpha[j]
    return T


def ritz_values(alpha, beta):
    """Eigenvalues (ascending) of the CG-Lanczos tridiagonal."""
    return np.linalg.eigvalsh(lanczos_tridiagonal(alpha, beta))


def gauss_nodes_weights(alpha, beta):
    """Gauss quadrature of the spectral measure of the starting residual:
    nodes = eigenvalues of T_m, weights = squared first eigenvector entries."""
    th, Q = np.linalg.eigh(lanczos_tridiagonal(alpha, beta))
    return th, Q[0, :] ** 2


def cheb_T(deg, y):
    """Matrix [T_0(y) .. T_deg(y)] by the defining recurrence."""
    y = np.asarray(y, dtype=np.float64)
    out = np.zeros(y.shape + (deg + 1,))
    out[..., 0] = 1.0
    if deg >= 1:
        out[..., 1] = y
    for j in range(2, deg + 1):
        out[..., j] = 2.0 * y * out[..., j - 1] - out[..., j - 2]
    return out


def poly_eval(coeffs, lam, lmax):
    """p(lam) = sum_j c_j T_j(2 lam / lmax - 1)."""
    coeffs = np.asarray(coeffs, dtype=np.float64)
    return cheb_T(coeffs.size - 1, 2.0 * np.asarray(lam, dtype=np.float64) / lmax - 1.0) @ coeffs
