"""GPU parity of TFQMR (the paper's second benchmark method) against the CPU
oracle, through the C ABI.

Bar: iteration count within +-1 of the oracle and ||x - x_ref|| / ||x_ref||
<= 1e-9 at rtol 1e-10; at a fixed iteration count (rtol 0, the benchmark's
20 iterations) the iterates agree to 1e-10.
"""
import numpy as np
import pytest

import oracle
from paper_2306_17801_amd import problems as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def apcg():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_17801_amd as m

    m.load()
    return m


@pytest.fixture(scope="module")
def ctx(apcg):
    c = apcg.apcg_ctx_create(0)
    yield c
    apcg.apcg_ctx_synchronize(c)
    apcg.apcg_ctx_destroy(c)


def tfqmr_gpu(apcg, ctx, A, b, rtol, maxit, x0=None, spmv=None, **opt):
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    dA, db = DeviceCSR(A), DeviceVec(b)
    if spmv is not None:
        apcg.apcg_mat_set_spmv_config(dA.h, *spmv)
    dx = DeviceVec(np.zeros(A.n) if x0 is None else x0)
    if x0 is None:
        opt.setdefault("x0_is_zero", 1)
    info = apcg.apcg_info_create(0, 1)
    apcg.apcg_ksp_solve_tfqmr(ctx, dA.h, db.h, dx.h, rtol, maxit, apcg.apcg_solve_opts_default(**opt), info, 0)
    res = apcg.apcg_info_get(info, 0)
    apcg.apcg_info_destroy(info)
    return res, dx.numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def system(which, seed):
    rng = np.random.default_rng(seed)
    if which == "convdiff2d":
        A = P.convection_diffusion((41, 37), (0.9, -0.4))
    elif which == "convdiff3d":
        A = P.convection_diffusion((13, 11, 9), (0.3, 0.7, -1.1))
    elif which == "laplace5":
        A = P.stencil_laplacian((64, 64), 5)
    elif which == "box27":
        A = P.stencil_laplacian((12, 12, 12), 27)
    else:
        A = P.diffusion_csr(np.exp(rng.standard_normal((9, 13, 17))), aniso=5.0)
    return A, rng.uniform(-1, 1, A.n)


@pytest.mark.parametrize("which", ["convdiff2d", "convdiff3d", "laplace5", "box27", "diffusion3d"])
@pytest.mark.parametrize("pc", [1, 0])
def test_tfqmr_parity(apcg, ctx, which, pc):
    A, b = system(which, 70)
    print(f"case tfqmr {which} pc={pc}", flush=True)
    ref = oracle.tfqmr(A, b, rtol=1e-10, maxit=5000, pc=pc)
    assert ref.status == oracle.CONVERGED
    res, x = tfqmr_gpu(apcg, ctx, A, b, 1e-10, 5000, pc=pc)
    assert res["status"] == apcg.APCG_SOLVE_CONVERGED
    assert abs(res["iterations"] - ref.its) <= 1
    assert rel(x, ref.x) <= 1e-9
    assert res["ref_norm"] == pytest.approx(ref.ref, rel=1e-13)
    assert res["res_norm"] <= 1e-10 * res["ref_norm"]


@pytest.mark.parametrize("which", ["convdiff2d", "laplace5", "box27"])
def test_tfqmr_twenty_iterations(apcg, ctx, which):
    """The benchmark's protocol: exactly 20 iterations (rtol 0)."""
    A, b = system(which, 71)
    print(f"case tfqmr-20 {which}", flush=True)
    ref = oracle.tfqmr(A, b, rtol=0.0, maxit=20)
    res, x = tfqmr_gpu(apcg, ctx, A, b, 0.0, 20)
    assert res["status"] == apcg.APCG_SOLVE_MAXIT and res["iterations"] == 20 and res["half_steps"] == 40
    assert rel(x, ref.x) <= 1e-10
    assert res["res_norm"] == pytest.approx(ref.res, rel=1e-8)


def test_tfqmr_modes_bitwise(apcg, ctx):
    """Graph, stream and host-check modes run the same kernels at the same
    launch shape: bit for bit the same iterate; a stop inside a graph period
    (converged at an odd half-step or at maxit) leaves the same state."""
    A, b = system("convdiff3d", 72)
    out = []
    for mode in (0, 1, 2):
        for rtol, maxit in ((1e-9, 5000), (0.0, 7)):
            print(f"case tfqmr-modes mode={mode} rtol={rtol} maxit={maxit}", flush=True)
            out.append((mode, rtol, maxit) + tfqmr_gpu(apcg, ctx, A, b, rtol, maxit, mode=mode))
    for rtol, maxit in ((1e-9, 5000), (0.0, 7)):
        runs = [o for o in out if o[1] == rtol and o[2] == maxit]
        for o in runs[1:]:
            assert o[3] == runs[0][3]
            assert np.array_equal(o[4], runs[0][4])


def test_tfqmr_status_cases(apcg, ctx):
    A, b = system("convdiff2d", 73)
    print("case tfqmr-status zero rhs", flush=True)
    res, x = tfqmr_gpu(apcg, ctx, A, np.zeros(A.n), 1e-8, 100)
    assert res["status"] == apcg.APCG_SOLVE_CONVERGED and res["iterations"] == 0 and np.all(x == 0.0)
    print("case tfqmr-status maxit 0", flush=True)
    res, x = tfqmr_gpu(apcg, ctx, A, b, 1e-8, 0)
    assert res["status"] == apcg.APCG_SOLVE_MAXIT and res["iterations"] == 0
    print("case tfqmr-status zero diagonal", flush=True)
    B = P.CSR(n=A.n, rowptr=A.rowptr, col=A.col, val=A.val.copy())
    q = B.rowptr[30] + int(np.nonzero(B.col[B.rowptr[30]:B.rowptr[31]] == 30)[0][0])
    B.val[q] = 0.0
    res, _ = tfqmr_gpu(apcg, ctx, B, b, 1e-8, 100)
    assert res["status"] == apcg.APCG_SOLVE_SETUP_ERROR
    res, _ = tfqmr_gpu(apcg, ctx, B, b, 1e-8, 100, pc=0)  # no preconditioner: fine
    assert res["status"] == apcg.APCG_SOLVE_CONVERGED
    print("case tfqmr-status initial guess", flush=True)
    x0 = np.random.default_rng(74).uniform(-1, 1, A.n)
    ref = oracle.tfqmr(A, b, x0=x0, rtol=1e-10, maxit=5000)
    res, x = tfqmr_gpu(apcg, ctx, A, b, 1e-10, 5000, x0=x0)
    assert res["status"] == apcg.APCG_SOLVE_CONVERGED and abs(res["iterations"] - ref.its) <= 1
    assert rel(x, ref.x) <= 1e-9
    assert res["ref_norm"] == pytest.approx(ref.ref, rel=1e-12)


def test_tfqmr_large_twenty_iterations(apcg, ctx):
    """A 7-point system of 10^6 rows (the sweep's 10^7-nonzero point):
    20 iterations against the oracle, in the graph mode the sweep times."""
    A = P.stencil_laplacian((100, 100, 100), 7)
    b = np.random.default_rng(75).uniform(-1, 1, A.n)
    print("case tfqmr-20 7-point 100^3", flush=True)
    ref = oracle.tfqmr(A, b, rtol=0.0, maxit=20)
    res, x = tfqmr_gpu(apcg, ctx, A, b, 0.0, 20)
    assert res["iterations"] == 20 and rel(x, ref.x) <= 1e-10


@pytest.mark.parametrize("which", ["convdiff2d", "convdiff3d", "box27", "diffusion3d"])
def test_tfqmr_sliced_diagonals_bitwise(apcg, ctx, which):
    """Patterns with a sliced-diagonal layout take it in the products (8, 16
    or 32 offset slots per slice).  Against the same matrix with one row's
    two first entries stored out of column order (no such layout: CSR
    products, that row summed in the other order) the solves agree to
    rounding, converged and at 20 iterations; both meet the oracle's bar."""
    A, b = system(which, 76)
    # an unsorted copy: identical matrix, CSR products only
    col, val = A.col.copy(), A.val.copy()
    s0 = A.rowptr[7]
    col[s0], col[s0 + 1] = col[s0 + 1], col[s0]
    val[s0], val[s0 + 1] = val[s0 + 1], val[s0]
    Au = P.CSR(n=A.n, rowptr=A.rowptr, col=col, val=val)
    for rtol, maxit in ((1e-10, 5000), (0.0, 20)):
        print(f"case tfqmr-sdia {which} rtol={rtol}", flush=True)
        r_sd, x_sd = tfqmr_gpu(apcg, ctx, A, b, rtol, maxit)
        r_csr, x_csr = tfqmr_gpu(apcg, ctx, Au, b, rtol, maxit)
        assert r_sd["iterations"] == r_csr["iterations"] and r_sd["status"] == r_csr["status"]
        assert rel(x_sd, x_csr) <= 1e-9
    ref = oracle.tfqmr(A, b, rtol=1e-10, maxit=5000)
    res, x = tfqmr_gpu(apcg, ctx, A, b, 1e-10, 5000, spmv=(1, 256, 0, apcg.APCG_SPMV_SDIA))
    assert res["status"] == apcg.APCG_SOLVE_CONVERGED and abs(res["iterations"] - ref.its) <= 1
    assert rel(x, ref.x) <= 1e-9
