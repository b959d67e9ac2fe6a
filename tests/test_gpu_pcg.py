"""GPU parity of the PCG hot path against the CPU oracle, through the C ABI.

Bar: iteration count within +-1 of the oracle and ||x - x_ref|| / ||x_ref||
<= 1e-9 at rtol 1e-10 (the two differ only in summation order and FMA use);
at matched iteration counts the iterates agree far more tightly.
"""
import math

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


def gpu_solve(apcg, ctx, A, b, rtol, maxit, x0=None, **opt):
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    dA = DeviceCSR(A)
    db = DeviceVec(b)
    dx = DeviceVec(np.zeros(A.n) if x0 is None else x0)
    if x0 is None and "x0_is_zero" not in opt:
        opt["x0_is_zero"] = 1
    info = apcg.apcg_info_create(0, 1)
    cfg = opt.pop("spmv", None)
    if cfg is not None:
        apcg.apcg_mat_set_spmv_config(dA.h, *cfg)
    opts = apcg.apcg_solve_opts_default(**opt)
    apcg.apcg_ksp_solve(ctx, dA.h, db.h, dx.h, rtol, maxit, opts, info, 0)
    res = apcg.apcg_info_get(info, 0)
    x = dx.numpy()
    apcg.apcg_info_destroy(info)
    return res, x


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("pc", [0, 1])
def test_poisson64_parity(apcg, ctx, mode, pc):
    """2D 5-point Poisson 64 x 64, x* ~ U[-1,1], x0 = 0, rtol 1e-10."""
    print(f"case poisson64 mode={mode} pc={pc}", flush=True)
    s = P.poisson2d_manufactured(64, 0)
    ref = oracle.pcg(s.A, s.b, rtol=1e-10, maxit=10000, pc=pc)
    res, x = gpu_solve(apcg, ctx, s.A, s.b, 1e-10, 10000, pc=pc, mode=mode)
    assert res["status"] == apcg.APCG_SOLVE_CONVERGED
    assert abs(res["iterations"] - ref.its) <= 1
    assert rel(x, ref.x) <= 1e-9
    assert rel(x, s.x_exact) <= 1711.7 * 1e-10
    assert res["ref_norm"] == pytest.approx(ref.ref, rel=1e-13)


@pytest.mark.parametrize("lpr", [-2, -1, 0, 1, 2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("tb", [256, 512])
def test_spmv_schedules_same_solve(apcg, ctx, lpr, tb):
    """Every SpMV schedule (lpr 0: the LDS-staged one, -1: the sliced one,
    -2: sliced diagonals) gives the oracle's iteration count on a ragged 3D
    variable-coefficient system (n = 21 * 17 * 13, not a multiple of 64)."""
    print(f"case schedule lpr={lpr} tb={tb}", flush=True)
    rng = np.random.default_rng(40)
    A = P.diffusion_csr(np.exp(rng.standard_normal((13, 17, 21))), aniso=7.0)
    b = rng.uniform(-1, 1, A.n)
    ref = oracle.pcg(A, b, rtol=1e-10, maxit=5000)
    spmv = {-2: (1, tb, 0, 3), -1: (1, tb, 0, 2), 0: (1, tb, 0, 1)}.get(lpr, (lpr, tb, 0, 0))
    res, x = gpu_solve(apcg, ctx, A, b, 1e-10, 5000, spmv=spmv)
    assert res["status"] == apcg.APCG_SOLVE_CONVERGED
    assert abs(res["iterations"] - ref.its) <= 1
    assert rel(x, ref.x) <= 1e-9


def test_matched_iterations_tight(apcg, ctx):
    """At a fixed iteration count (rtol = 0) the GPU and oracle iterates agree
    to rounding: the paper's fixed-20-iteration protocol (Section 4.1)."""
    rng = np.random.default_rng(41)
    A = P.diffusion_csr(np.exp(rng.standard_normal((40, 50))))
    b = rng.uniform(-1, 1, A.n)
    ref = oracle.pcg(A, b, rtol=0.0, maxit=20)
    res, x = gpu_solve(apcg, ctx, A, b, 0.0, 20)
    assert res["status"] == apcg.APCG_SOLVE_MAXIT and res["iterations"] == 20
    assert rel(x, ref.x) <= 1e-12
    assert res["res_norm"] == pytest.approx(ref.res, rel=1e-10)


def test_nonzero_initial_guess_and_preconditioned_norm(apcg, ctx):
    rng = np.random.default_rng(42)
    A = P.diffusion_csr(np.exp(1.5 * rng.standard_normal((30, 33))), aniso=20.0)
    b = rng.uniform(-1, 1, A.n)
    x0 = rng.uniform(-1, 1, A.n)
    ref = oracle.pcg(A, b, x0=x0, rtol=1e-10, maxit=5000, norm_type=oracle.NORM_PRECONDITIONED)
    res, x = gpu_solve(apcg, ctx, A, b, 1e-10, 5000, x0=x0, norm_type=1)
    assert res["status"] == apcg.APCG_SOLVE_CONVERGED
    assert abs(res["iterations"] - ref.its) <= 1
    assert rel(x, ref.x) <= 1e-9
    assert res["ref_norm"] == pytest.approx(ref.ref, rel=1e-13)


def test_edge_cases(apcg, ctx):
    A = P.laplace_2d(7)
    n = A.n
    # b = 0 with a nonzero x0: x = 0, converged in 0 iterations
    res, x = gpu_solve(apcg, ctx, A, np.zeros(n), 1e-8, 100, x0=np.ones(n))
    assert res["status"] == apcg.APCG_SOLVE_CONVERGED and res["iterations"] == 0 and np.all(x == 0)
    # maxit = 0 and 1
    res, _ = gpu_solve(apcg, ctx, A, np.ones(n), 1e-8, 0)
    assert res["status"] == apcg.APCG_SOLVE_MAXIT and res["iterations"] == 0
    res, x = gpu_solve(apcg, ctx, A, np.ones(n), 1e-14, 1)
    ref = oracle.pcg(A, np.ones(n), rtol=1e-14, maxit=1)
    assert res["status"] == apcg.APCG_SOLVE_MAXIT and res["iterations"] == 1 and rel(x, ref.x) <= 1e-14
    # x0 already the solution
    s = P.poisson2d_manufactured(7, 3)
    res, _ = gpu_solve(apcg, ctx, s.A, s.b, 1e-8, 100, x0=s.x_exact)
    assert res["status"] == apcg.APCG_SOLVE_CONVERGED and res["iterations"] == 0
    # one unknown
    one = P.CSR(n=1, rowptr=np.array([0, 1], np.int32), col=np.array([0], np.int32), val=np.array([4.0]))
    res, x = gpu_solve(apcg, ctx, one, np.array([2.0]), 1e-12, 10)
    assert res["status"] == apcg.APCG_SOLVE_CONVERGED and res["iterations"] == 1 and x[0] == 0.5


def test_failure_states(apcg, ctx):
    A = P.laplace_2d(6)
    n = A.n
    # non-positive diagonal: Jacobi setup error
    B = P.CSR(n=A.n, rowptr=A.rowptr, col=A.col, val=A.val.copy())
    diag_pos = np.array([k for i in range(n) for k in range(B.rowptr[i], B.rowptr[i + 1]) if B.col[k] == i])
    B.val[diag_pos[5]] = -4.0
    res, _ = gpu_solve(apcg, ctx, B, np.ones(n), 1e-8, 100)
    assert res["status"] == apcg.APCG_SOLVE_SETUP_ERROR
    # NaN in b
    b = np.ones(n)
    b[3] = np.nan
    res, _ = gpu_solve(apcg, ctx, A, b, 1e-8, 100)
    assert res["status"] == apcg.APCG_SOLVE_NAN
    # indefinite operator, no preconditioner: p.Ap = 0 at the first step
    D = P.CSR(n=2, rowptr=np.array([0, 1, 2], np.int32), col=np.array([0, 1], np.int32), val=np.array([1.0, -1.0]))
    res, _ = gpu_solve(apcg, ctx, D, np.array([1.0, 1.0]), 1e-10, 10, pc=0)
    ref = oracle.pcg(D, np.array([1.0, 1.0]), rtol=1e-10, maxit=10, pc=0)
    assert ref.status == oracle.BREAKDOWN_PAP
    assert res["status"] == apcg.APCG_SOLVE_BREAKDOWN_PAP and res["iterations"] == 0


def test_repeated_solves_bitwise_identical(apcg, ctx):
    """Fixed-order reductions: repeated solves agree bit for bit (the
    PostSolve residual check of Section 4.1 made exact)."""
    rng = np.random.default_rng(43)
    A = P.diffusion_csr(np.exp(rng.standard_normal((64, 70))))
    b = rng.uniform(-1, 1, A.n)
    r1, x1 = gpu_solve(apcg, ctx, A, b, 1e-8, 5000)
    r2, x2 = gpu_solve(apcg, ctx, A, b, 1e-8, 5000, mode=1)
    r3, x3 = gpu_solve(apcg, ctx, A, b, 1e-8, 5000, mode=2)
    assert r1 == r2 == r3
    assert np.array_equal(x1, x2) and np.array_equal(x1, x3)


@pytest.fixture(scope="module")
def diffusion128():
    return P.diffusion3d_smoothed(128, 2)


def test_full_size_diffusion128_parity(apcg, ctx, diffusion128):
    """The 128^3 variable-coefficient system at its full size, in the launch
    configuration the benchmark times (graph mode, autotuned schedule):
    iterations +-1 and ||x - x_ref|| / ||x_ref|| <= 1e-9 at rtol 1e-10."""
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    s = diffusion128
    print("case diffusion128 full size", flush=True)
    dA, db, dx = DeviceCSR(s.A), DeviceVec(s.b), DeviceVec.zeros(s.A.n)
    apcg.apcg_mat_autotune(dA.h, ctx, 3)
    info = apcg.apcg_info_create(0, 1)
    apcg.apcg_ksp_solve(ctx, dA.h, db.h, dx.h, 1e-10, 50000, apcg.apcg_solve_opts_default(x0_is_zero=1), info, 0)
    res = apcg.apcg_info_get(info, 0)
    x = dx.numpy()
    ref = oracle.pcg(s.A, s.b, rtol=1e-10, maxit=50000)
    print(f"gpu its={res['iterations']} oracle its={ref.its}", flush=True)
    assert res["status"] == apcg.APCG_SOLVE_CONVERGED
    assert abs(res["iterations"] - ref.its) <= 1
    assert rel(x, ref.x) <= 1e-9
    true = np.linalg.norm(s.b - s.A.to_scipy() @ x) / np.linalg.norm(s.b)
    assert true <= 1.5e-10
    apcg.apcg_info_destroy(info)


def test_graph_cache_after_matrix_destroy(apcg, ctx):
    """Matrices of different sizes, each destroyed before the next is
    wrapped, solved into the same x memory in graph mode: a new handle may
    land at a destroyed one's address, and the cached graph must not be
    replayed for it (its row count and arrays are baked into the capture)."""
    import torch
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    xbig = torch.zeros(2000, dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    info = apcg.apcg_info_create(0, 1)
    opts = apcg.apcg_solve_opts_default(x0_is_zero=1)
    for side in (40, 20, 40, 36, 8, 20):
        A = P.laplace_2d(side)
        b = np.random.default_rng(side).uniform(-1, 1, A.n)
        print(f"case graph-cache side={side}", flush=True)
        dA, db = DeviceCSR(A), DeviceVec(b)
        dx = DeviceVec(xbig[: A.n])
        assert dx.t.data_ptr() == xbig.data_ptr()
        apcg.apcg_ksp_solve(ctx, dA.h, db.h, dx.h, 1e-10, 10000, opts, info, 0)
        res = apcg.apcg_info_get(info, 0)
        ref = oracle.pcg(A, b, rtol=1e-10, maxit=10000)
        assert res["status"] == apcg.APCG_SOLVE_CONVERGED and abs(res["iterations"] - ref.its) <= 1
        assert rel(dx.numpy(), ref.x) <= 1e-9
        dx.close()
        db.close()
        dA.close()
    apcg.apcg_info_destroy(info)


def nine_point(m):
    """9-point operator 9 I - S (x) S, S = tridiag(1, 1, 1): SPD, interior rows
    of 9 entries (wider than the sliced kernel's unrolled path)."""
    import scipy.sparse as sp

    S = sp.diags([np.ones(m - 1), np.ones(m), np.ones(m - 1)], [-1, 0, 1])
    M = (9.0 * sp.identity(m * m) - sp.kron(S, S)).tocsr()
    M.sort_indices()
    return P.CSR(n=m * m, rowptr=M.indptr.astype(np.int32), col=M.indices.astype(np.int32), val=M.data.copy())


@pytest.mark.parametrize("which", ["diffusion3d_ragged", "ninepoint_45"])
def test_row_ordered_schedules_agree(apcg, ctx, which):
    """The sliced and sliced-diagonal schedules (both block sizes, the
    9-entry rows and 9 offsets per slice taking their looped paths) against
    the staged and one-lane-per-row ones: each meets the
    oracle's bar, and at a fixed iteration count the iterates agree to
    rounding (the reductions' trees follow the launch shape, so only the
    products themselves are bit for bit equal)."""
    rng = np.random.default_rng(43)
    if which == "ninepoint_45":
        A = nine_point(45)
    else:
        A = P.diffusion_csr(np.exp(rng.standard_normal((11, 19, 23))), aniso=3.0)
    b = rng.uniform(-1, 1, A.n)
    ref = oracle.pcg(A, b, rtol=1e-10, maxit=5000)
    ref20 = oracle.pcg(A, b, rtol=0.0, maxit=20)
    for spmv in [(1, 256, 0, 2), (1, 512, 40, 2), (1, 256, 0, 3), (1, 512, 40, 3), (1, 256, 0, 1), (1, 256, 0, 0)]:
        print(f"case {which} spmv={spmv}", flush=True)
        res, x = gpu_solve(apcg, ctx, A, b, 1e-10, 5000, spmv=spmv)
        assert res["status"] == apcg.APCG_SOLVE_CONVERGED and abs(res["iterations"] - ref.its) <= 1
        assert rel(x, ref.x) <= 1e-9
        res, x = gpu_solve(apcg, ctx, A, b, 0.0, 20, spmv=spmv)
        assert res["iterations"] == 20 and rel(x, ref20.x) <= 1e-12


def random_pattern(n, per_row, seed):
    """SPD, diagonally dominant, with per_row random off-diagonal columns
    per row (symmetrised): slices see many distinct column offsets."""
    import scipy.sparse as sp

    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(n), per_row)
    cols = rng.integers(0, n, n * per_row)
    M = sp.coo_matrix((-rng.uniform(0.1, 1.0, n * per_row), (rows, cols)), shape=(n, n)).tocsr()
    M = (M + M.T).tocsr()
    M.setdiag(0.0)
    M.eliminate_zeros()
    M = M + sp.diags(np.asarray(abs(M).sum(axis=1)).ravel() + 1.0)
    M = M.tocsr()
    M.sort_indices()
    return P.CSR(n=n, rowptr=M.indptr.astype(np.int32), col=M.indices.astype(np.int32), val=M.data.copy())


@pytest.mark.parametrize("which", ["diffusion3d_ragged", "ninepoint_45", "laplace1d_50"])
@pytest.mark.parametrize("tb,blocks", [(256, 0), (512, 24)])
def test_sliced_diagonals_bitwise_equal_sliced(apcg, ctx, which, tb, blocks):
    """Sliced diagonals and the sliced schedule at the same launch shape walk
    the same slices in the same order and add every row's entries in column
    order with the same fused multiply-adds, so whole solves (products,
    reductions, iterates) are bit for bit equal; both meet the oracle's bar.
    laplace1d_50: fewer rows than one slice."""
    rng = np.random.default_rng(44)
    if which == "ninepoint_45":
        A = nine_point(45)
    elif which == "laplace1d_50":
        import scipy.sparse as sp

        M = sp.diags([-np.ones(49), 2.5 * np.ones(50), -np.ones(49)], [-1, 0, 1]).tocsr()
        M.sort_indices()
        A = P.CSR(n=50, rowptr=M.indptr.astype(np.int32), col=M.indices.astype(np.int32), val=M.data.copy())
    else:
        A = P.diffusion_csr(np.exp(rng.standard_normal((11, 19, 23))), aniso=3.0)
    b = rng.uniform(-1, 1, A.n)
    ref = oracle.pcg(A, b, rtol=1e-10, maxit=5000)
    print(f"case sdia-vs-sell {which} tb={tb} blocks={blocks}", flush=True)
    r_sell, x_sell = gpu_solve(apcg, ctx, A, b, 1e-10, 5000, spmv=(1, tb, blocks, 2))
    r_sdia, x_sdia = gpu_solve(apcg, ctx, A, b, 1e-10, 5000, spmv=(1, tb, blocks, 3))
    assert r_sdia["status"] == apcg.APCG_SOLVE_CONVERGED and abs(r_sdia["iterations"] - ref.its) <= 1
    assert rel(x_sdia, ref.x) <= 1e-9
    assert r_sdia["iterations"] == r_sell["iterations"]
    assert r_sdia["res_norm"] == r_sell["res_norm"]
    assert np.array_equal(x_sdia, x_sell)


def test_sliced_diagonals_values_refilled(apcg, ctx):
    """The value copy is refilled at the start of every solve: scaling the
    CSR values in place between two solves of one wrapped matrix gives the
    oracle's solution of the scaled system."""
    import torch
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    rng = np.random.default_rng(45)
    A = P.diffusion_csr(np.exp(rng.standard_normal((9, 14, 17))))
    b = rng.uniform(-1, 1, A.n)
    dA, db = DeviceCSR(A), DeviceVec(b)
    apcg.apcg_mat_set_spmv_config(dA.h, 1, 256, 0, apcg.APCG_SPMV_SDIA)
    info = apcg.apcg_info_create(0, 1)
    opts = apcg.apcg_solve_opts_default(x0_is_zero=1)
    for scale in (1.0, 3.0):
        print(f"case sdia refill scale={scale}", flush=True)
        if scale != 1.0:
            dA.val.mul_(scale)
            torch.cuda.synchronize()
        dx = DeviceVec.zeros(A.n)
        apcg.apcg_ksp_solve(ctx, dA.h, db.h, dx.h, 1e-10, 5000, opts, info, 0)
        res = apcg.apcg_info_get(info, 0)
        As = P.CSR(n=A.n, rowptr=A.rowptr, col=A.col, val=A.val * scale)
        ref = oracle.pcg(As, b, rtol=1e-10, maxit=5000)
        assert res["status"] == apcg.APCG_SOLVE_CONVERGED and abs(res["iterations"] - ref.its) <= 1
        assert rel(dx.numpy(), ref.x) <= 1e-9
    apcg.apcg_info_destroy(info)


def test_sliced_diagonals_rejected(apcg, ctx):
    """The schedule is refused (APCG_ERR_UNSUPPORTED, the matrix keeps its
    configuration) for unsorted rows and for patterns with more than 32
    distinct column offsets in a slice; the autotuner then skips it."""
    from paper_2306_17801_amd.device import DeviceCSR

    A = random_pattern(700, 6, 46)
    dA = DeviceCSR(A)
    before = apcg.apcg_mat_get_spmv_config(dA.h)
    with pytest.raises(apcg.ApcgError) as e:
        apcg.apcg_mat_set_spmv_config(dA.h, 1, 256, 0, apcg.APCG_SPMV_SDIA)
    assert e.value.code == apcg.APCG_ERR_UNSUPPORTED
    assert apcg.apcg_mat_get_spmv_config(dA.h) == before
    best, _ = apcg.apcg_mat_autotune(dA.h, ctx, 2)
    assert best["schedule"] != apcg.APCG_SPMV_SDIA
    # a row with its columns out of order (same matrix, one row's two
    # entries swapped together with their values)
    B = nine_point(12)
    col, val = B.col.copy(), B.val.copy()
    s0 = B.rowptr[30]
    col[s0], col[s0 + 1] = col[s0 + 1], col[s0]
    val[s0], val[s0 + 1] = val[s0 + 1], val[s0]
    dB = DeviceCSR(P.CSR(n=B.n, rowptr=B.rowptr, col=col, val=val))
    with pytest.raises(apcg.ApcgError) as e:
        apcg.apcg_mat_set_spmv_config(dB.h, 1, 256, 0, apcg.APCG_SPMV_SDIA)
    assert e.value.code == apcg.APCG_ERR_UNSUPPORTED


@pytest.mark.parametrize("shape,points", [((40, 37), 9), ((12, 11, 9), 27), ((30, 20), 5), ((9, 10, 11), 7)])
def test_stencil_operators_all_schedules(apcg, ctx, shape, points):
    """The four stencils of the paper's CG benchmark (Section 4.1).  The
    27-point operator takes the wide paths: 27 offsets per slice (sliced
    diagonals, 32 offset slots) and 27-entry rows (sliced, row groups).
    Every schedule meets the oracle's bar; sliced diagonals equal the sliced
    schedule bit for bit at the same launch shape; at exactly 20 iterations
    (the benchmark's protocol) the iterates agree with the oracle to
    rounding."""
    A = P.stencil_laplacian(shape, points)
    b = np.random.default_rng(47).uniform(-1, 1, A.n)
    ref = oracle.pcg(A, b, rtol=1e-10, maxit=5000)
    ref20 = oracle.pcg(A, b, rtol=0.0, maxit=20)
    xs = {}
    for spmv in [(1, 256, 0, 3), (1, 256, 0, 2), (1, 512, 16, 3), (1, 512, 16, 2), (4, 256, 0, 0), (8, 512, 0, 0)]:
        print(f"case stencil {points}-pt {shape} spmv={spmv}", flush=True)
        res, x = gpu_solve(apcg, ctx, A, b, 1e-10, 5000, spmv=spmv)
        assert res["status"] == apcg.APCG_SOLVE_CONVERGED and abs(res["iterations"] - ref.its) <= 1
        assert rel(x, ref.x) <= 1e-9
        xs[spmv] = x
        res, x = gpu_solve(apcg, ctx, A, b, 0.0, 20, spmv=spmv)
        assert res["iterations"] == 20 and res["status"] == apcg.APCG_SOLVE_MAXIT
        assert rel(x, ref20.x) <= 1e-12
    assert np.array_equal(xs[(1, 256, 0, 3)], xs[(1, 256, 0, 2)])
    assert np.array_equal(xs[(1, 512, 16, 3)], xs[(1, 512, 16, 2)])


@pytest.mark.parametrize("sync", [False, True])
@pytest.mark.parametrize("shape,points,diag", [((33, 29), 9, 8.0), ((10, 9, 8), 27, 26.0), ((41, 23), 5, 4.0)])
def test_composed_cg_matches_oracle(apcg, ctx, shape, points, diag, sync):
    """CG written from the asynchronous primitives (MatMult, VecDot, VecNorm,
    AXPY, AYPX, scalar division; Section 3.3) with device scalars, with and
    without reading every reduction back to the host: 20 iterations agree
    with the oracle's Jacobi-PCG to rounding, and the returned residual norm
    with the oracle's."""
    from paper_2306_17801_amd.composed import ComposedCG
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    A = P.stencil_laplacian(shape, points)
    b = np.random.default_rng(48).uniform(-1, 1, A.n)
    ref = oracle.pcg(A, b, rtol=0.0, maxit=20)
    print(f"case composed {points}-pt {shape} sync={sync}", flush=True)
    dA, db, dx = DeviceCSR(A), DeviceVec(b), DeviceVec.zeros(A.n)
    cg = ComposedCG(ctx, A.n)
    res = cg.solve(dA.h, db.h, dx.h, diag, 20, sync=sync)
    cg.close()
    assert rel(dx.numpy(), ref.x) <= 1e-12
    assert res == pytest.approx(ref.res, rel=1e-10)


def banded(n, far):
    """SPD M-matrix with couplings to the neighbours at distance 1 and far."""
    import scipy.sparse as sp

    M = sp.diags([-np.ones(n - far), -np.ones(n - 1), 4.5 * np.ones(n), -np.ones(n - 1), -np.ones(n - far)],
                 [-far, -1, 0, 1, far]).tocsr()
    M.sort_indices()
    return P.CSR(n=n, rowptr=M.indptr.astype(np.int32), col=M.indices.astype(np.int32), val=M.data.copy())


@pytest.mark.parametrize("which", ["diffusion_10x16x16", "banded_1050_128", "box27_8x8x16"])
def test_sliced_diagonals_plane_marching(apcg, ctx, which):
    """Plane marching (lanes_per_row = planes per task > 1, any count): the +-plane
    windows are carried between the slices of a column instead of gathered.
    Patterns: a 3D grid whose planes are 4 slices, a banded matrix whose far
    band is 2 slices away with a partial last plane (17 slices), a 27-point
    grid (32 offset slots).  Each meets the oracle's bar, and at 20
    iterations agrees with the plain sliced-diagonal kernel to rounding (the
    products are the same sums; only the reduction's grouping differs)."""
    rng = np.random.default_rng(49)
    if which == "diffusion_10x16x16":
        A = P.diffusion_csr(np.exp(rng.standard_normal((10, 16, 16))), aniso=2.0)
    elif which == "banded_1050_128":
        A = banded(1050, 128)
    else:
        A = P.stencil_laplacian((8, 8, 16), 27)
    b = rng.uniform(-1, 1, A.n)
    ref = oracle.pcg(A, b, rtol=1e-10, maxit=5000)
    _, x_plain = gpu_solve(apcg, ctx, A, b, 0.0, 20, spmv=(1, 256, 0, 3))
    for spmv in [(2, 256, 0, 3), (3, 512, 0, 3), (4, 512, 0, 3), (6, 256, 0, 3), (8, 256, 0, 3), (64, 512, 0, 3)]:
        print(f"case march {which} spmv={spmv}", flush=True)
        res, x = gpu_solve(apcg, ctx, A, b, 1e-10, 5000, spmv=spmv)
        assert res["status"] == apcg.APCG_SOLVE_CONVERGED and abs(res["iterations"] - ref.its) <= 1
        assert rel(x, ref.x) <= 1e-9
        res, x = gpu_solve(apcg, ctx, A, b, 0.0, 20, spmv=spmv)
        assert res["iterations"] == 20 and rel(x, x_plain) <= 1e-13


def with_stored_zero(A):
    """A with one explicitly stored zero at (0, n-1) and none at (n-1, 0): the
    same operator, a structurally unsymmetric pattern."""
    rowptr = A.rowptr.copy()
    rowptr[1:] += 1
    e = int(A.rowptr[1])
    col = np.insert(A.col, e, A.n - 1).astype(np.int32)
    val = np.insert(A.val, e, 0.0)
    return P.CSR(n=A.n, rowptr=rowptr, col=col, val=val)


@pytest.mark.parametrize("which", ["diffusion_10x16x16", "banded_1050_128", "box27_8x8x16"])
def test_sliced_diagonals_symmetric_reads_bitwise(apcg, ctx, which):
    """With symmetric values the marching product reads each entry left of
    the diagonal as its transpose (for the -plane offset the previous
    slice's +plane slot, otherwise the same or an earlier slice's).  A twin with one stored zero that
    breaks the pattern's symmetry (same operator, every slot read directly)
    gives bit for bit the same solves at the same launch shape."""
    rng = np.random.default_rng(50)
    if which == "diffusion_10x16x16":
        A = P.diffusion_csr(np.exp(rng.standard_normal((10, 16, 16))), aniso=2.0)
    elif which == "banded_1050_128":
        A = banded(1050, 128)
    else:
        A = P.stencil_laplacian((8, 8, 16), 27)
    T = with_stored_zero(A)
    b = rng.uniform(-1, 1, A.n)
    ref = oracle.pcg(A, b, rtol=1e-10, maxit=5000)
    for spmv in [(2, 256, 0, 3), (8, 512, 0, 3)]:
        print(f"case symmetric reads {which} spmv={spmv}", flush=True)
        r_s, x_s = gpu_solve(apcg, ctx, A, b, 1e-10, 5000, spmv=spmv)
        r_t, x_t = gpu_solve(apcg, ctx, T, b, 1e-10, 5000, spmv=spmv)
        assert r_s["status"] == apcg.APCG_SOLVE_CONVERGED and abs(r_s["iterations"] - ref.its) <= 1
        assert rel(x_s, ref.x) <= 1e-9
        assert r_s["iterations"] == r_t["iterations"] and r_s["res_norm"] == r_t["res_norm"]
        assert np.array_equal(x_s, x_t)


def test_sliced_diagonals_symmetry_rechecked_each_solve(apcg, ctx):
    """The value-symmetry check runs with every refill: one entry left of the
    diagonal changed in place (values no longer symmetric) is read as
    stored, and after restoring it the matrix keeps reading every slot (the
    flag is only cleared); each solve meets the oracle's bar for the values
    it was given."""
    import torch
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    rng = np.random.default_rng(51)
    A = P.diffusion_csr(np.exp(rng.standard_normal((10, 16, 16))), aniso=2.0)
    b = rng.uniform(-1, 1, A.n)
    dA, db = DeviceCSR(A), DeviceVec(b)
    apcg.apcg_mat_set_spmv_config(dA.h, 4, 256, 0, apcg.APCG_SPMV_SDIA)
    row = A.n // 2 + 7
    k = int(A.rowptr[row])  # the row's first entry, left of the diagonal
    assert A.col[k] < row
    info = apcg.apcg_info_create(0, 1)
    opts = apcg.apcg_solve_opts_default(x0_is_zero=1)
    seen = []
    for factor in (1.0, 1.25, 1.0):
        print(f"case symmetry recheck factor={factor}", flush=True)
        val = A.val.copy()
        val[k] *= factor
        dA.val.copy_(torch.from_numpy(val))
        torch.cuda.synchronize()
        dx = DeviceVec.zeros(A.n)
        apcg.apcg_ksp_solve(ctx, dA.h, db.h, dx.h, 1e-10, 5000, opts, info, 0)
        res = apcg.apcg_info_get(info, 0)
        ref = oracle.pcg(P.CSR(n=A.n, rowptr=A.rowptr, col=A.col, val=val), b, rtol=1e-10, maxit=5000)
        assert res["status"] == apcg.APCG_SOLVE_CONVERGED and abs(res["iterations"] - ref.its) <= 1
        assert rel(dx.numpy(), ref.x) <= 1e-9
        seen.append(apcg.apcg_mat_get_sdia_info(dA.h)["values_symmetric"])
    # transposed reads while the values were symmetric, then never again
    assert seen == [1, 0, 0]
    apcg.apcg_info_destroy(info)


def test_sliced_diagonal_info(apcg, ctx):
    """The analysis as apcg_mat_get_sdia_info reports it: the 3D grid (planes
    of 4 slices) is structurally symmetric with symmetric values and a plane
    stride; the twin with one unmatched stored zero is not structurally
    symmetric; an unsorted pattern is rejected; a matrix never put on the
    schedule reads as not analysed."""
    from paper_2306_17801_amd.device import DeviceCSR

    rng = np.random.default_rng(52)
    A = P.diffusion_csr(np.exp(rng.standard_normal((10, 16, 16))), aniso=2.0)
    dA, dT = DeviceCSR(A), DeviceCSR(with_stored_zero(A))
    assert apcg.apcg_mat_get_sdia_info(dA.h)["state"] == 0
    for d in (dA, dT):
        apcg.apcg_mat_set_spmv_config(d.h, 4, 256, 0, apcg.APCG_SPMV_SDIA)
    ia, it = apcg.apcg_mat_get_sdia_info(dA.h), apcg.apcg_mat_get_sdia_info(dT.h)
    print("info", ia, it, flush=True)
    assert ia == {"state": 1, "value_slots": 7, "offset_slots": 8, "plane_stride": 4,
                  "structurally_symmetric": 1, "values_symmetric": 1}
    assert it["state"] == 1 and it["structurally_symmetric"] == 0 and it["values_symmetric"] == 0
    # slice 0 lies in the bottom plane (no -256), so the extra offset n - 1
    # keeps it at 7 distinct offsets
    assert it["value_slots"] == 7 and it["plane_stride"] == 4
    B = random_pattern(700, 6, 46)
    dB = DeviceCSR(B)
    with pytest.raises(apcg.ApcgError):
        apcg.apcg_mat_set_spmv_config(dB.h, 1, 256, 0, apcg.APCG_SPMV_SDIA)
    assert apcg.apcg_mat_get_sdia_info(dB.h)["state"] == -1


def test_overlapping_vectors_rejected(apcg, ctx):
    """A vector a call writes may share no memory with one it reads: the
    PCG, FCG and TFQMR solves (x against b) and MatMult (y against x) reject
    a view that overlaps the other in part, and the PCG solve runs to the
    oracle's bar once the two views of the buffer are adjacent."""
    import torch
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    A = P.laplace_2d(6)
    n = A.n
    rhs = np.random.default_rng(91).uniform(-1, 1, n)
    dA = DeviceCSR(A)
    big = torch.zeros(2 * n, dtype=torch.float64, device="cuda:0")
    big[:n] = torch.from_numpy(rhs).to("cuda:0")
    b = DeviceVec(big[0:n])
    half = DeviceVec(big[n // 2:n // 2 + n])
    info = apcg.apcg_info_create(0, 1)
    opts = apcg.apcg_solve_opts_default(x0_is_zero=1)
    coef = torch.zeros(9, dtype=torch.float32, device="cuda:0")
    lmax = torch.full((1,), 8.0, dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    calls = {
        "pcg": lambda: apcg.apcg_ksp_solve(ctx, dA.h, b.h, half.h, 1e-10, 100, opts, info, 0),
        "fcg": lambda: apcg.apcg_ksp_solve_fcg_poly(ctx, dA.h, b.h, half.h, 1e-10, 100, coef, lmax, opts,
                                                    apcg.apcg_fcg_opts_default(), info, 0),
        "tfqmr": lambda: apcg.apcg_ksp_solve_tfqmr(ctx, dA.h, b.h, half.h, 1e-10, 100, opts, info, 0),
        "matmult": lambda: apcg.apcg_mat_mult_async(dA.h, b.h, half.h, ctx),
    }
    for name, call in calls.items():
        print(f"case overlapping views rejected: {name}", flush=True)
        with pytest.raises(apcg.ApcgError):
            call()
    x = DeviceVec(big[n:2 * n])
    apcg.apcg_ksp_solve(ctx, dA.h, b.h, x.h, 1e-10, 1000, opts, info, 0)
    r = apcg.apcg_info_get(info, 0)
    ref = oracle.pcg(A, rhs, rtol=1e-10, maxit=1000)
    assert r["status"] == apcg.APCG_SOLVE_CONVERGED and abs(r["iterations"] - ref.its) <= 1
    assert rel(x.numpy(), ref.x) <= 1e-9
    assert np.array_equal(b.numpy(), rhs)
    apcg.apcg_info_destroy(info)
