"""GPU parity of the one-workgroup persistent solve (APCG_MODE_PERSISTENT /
APCG_MODE_AUTO) against the CPU oracle, through the C ABI, and the latency
floors it is measured against.

Bar: iterations +-1 and ||x - x_ref|| / ||x_ref|| <= 1e-9 at rtol 1e-10;
at a matched iteration count the iterates agree to 1e-12.  The sizes span
every rows-per-thread class (1, 2, 4 and 8 rows of each of the 512 threads)
and the three row paths (matrix entries of rows of at most 5 or 7 entries
held in registers, longer rows read every iteration), with sizes that are
not multiples of 64.
"""
import numpy as np
import pytest

import oracle
from paper_2306_17801_amd import problems as P

pytestmark = pytest.mark.gpu

PERSISTENT = 3
AUTO = 4


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
    opt.setdefault("mode", PERSISTENT)
    info = apcg.apcg_info_create(0, 1)
    opts = apcg.apcg_solve_opts_default(**opt)
    apcg.apcg_ksp_solve(ctx, dA.h, db.h, dx.h, rtol, maxit, opts, info, 0)
    res = apcg.apcg_info_get(info, 0)
    x = dx.numpy()
    apcg.apcg_info_destroy(info)
    for v in (dx, db):
        v.close()
    dA.close()
    return res, x


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def system(kind, n_target, seed):
    """kind 5: 2D 5-point (rows <= 5 entries), 7: 3D 7-point (<= 7), 9: 2D
    9-point box stencil (9 entries: rows read every iteration); variable
    coefficients for 5 and 7, sizes near n_target and not multiples of 64."""
    rng = np.random.default_rng(seed)
    if kind == 5:
        ny = max(1, int(round(n_target ** 0.5)))
        nx = max(1, n_target // ny)
        A = P.diffusion_csr(np.exp(rng.standard_normal((ny, nx))), aniso=3.0)
    elif kind == 7:
        s = max(1, int(round(n_target ** (1 / 3))))
        A = P.diffusion_csr(np.exp(rng.standard_normal((s, s + 1, max(1, n_target // (s * (s + 1)))))))
    else:
        ny = max(2, int(round(n_target ** 0.5)))
        A = P.stencil_laplacian((ny, max(2, n_target // ny)), 9)
    return A, rng.uniform(-1, 1, A.n)


CASES = [(5, 1, 1), (5, 300, 2), (7, 480, 3), (9, 500, 4), (5, 1000, 5), (7, 900, 6), (9, 1000, 7),
         (5, 1900, 8), (7, 2000, 9), (9, 2030, 10), (5, 3001, 11), (7, 4000, 12), (9, 4090, 13)]


@pytest.mark.parametrize("kind,n_target,seed", CASES)
def test_persistent_parity(apcg, ctx, kind, n_target, seed):
    A, b = system(kind, n_target, seed)
    assert A.n <= 4096
    print(f"case persistent kind={kind} n={A.n}", flush=True)
    ref = oracle.pcg(A, b, rtol=1e-10, maxit=20000)
    res, x = gpu_solve(apcg, ctx, A, b, 1e-10, 20000)
    assert res["status"] == ref.status == apcg.APCG_SOLVE_CONVERGED
    assert abs(res["iterations"] - ref.its) <= 1
    assert rel(x, ref.x) <= 1e-9
    assert res["ref_norm"] == pytest.approx(ref.ref, rel=1e-13)
    # matched iteration count: the same iterate up to rounding
    k = min(res["iterations"], 25)
    ref_k = oracle.pcg(A, b, rtol=0.0, maxit=k)
    res_k, x_k = gpu_solve(apcg, ctx, A, b, 0.0, k)
    assert res_k["iterations"] == ref_k.its == k
    assert rel(x_k, ref_k.x) <= 1e-12


@pytest.mark.parametrize("pc", [0, 1])
def test_poisson64_persistent(apcg, ctx, pc):
    """The 64 x 64 Poisson system at rtol 1e-10 (CG and Jacobi-PCG): the
    oracle's count +-1, the manufactured solution within kappa rtol."""
    s = P.poisson2d_manufactured(64, 0)
    ref = oracle.pcg(s.A, s.b, rtol=1e-10, maxit=10000, pc=pc)
    res, x = gpu_solve(apcg, ctx, s.A, s.b, 1e-10, 10000, pc=pc)
    assert res["status"] == apcg.APCG_SOLVE_CONVERGED
    assert abs(res["iterations"] - ref.its) <= 1
    assert rel(x, ref.x) <= 1e-9
    assert rel(x, s.x_exact) <= 1711.7 * 1e-10


def test_edge_cases(apcg, ctx):
    A, b = system(5, 700, 21)
    # b = 0: x = 0 in 0 iterations, whatever x0
    res, x = gpu_solve(apcg, ctx, A, np.zeros(A.n), 1e-10, 100, x0=np.ones(A.n), x0_is_zero=0)
    assert res["status"] == apcg.APCG_SOLVE_CONVERGED and res["iterations"] == 0 and not x.any()
    # maxit 0 and 1
    res, x = gpu_solve(apcg, ctx, A, b, 1e-10, 0)
    assert res["status"] == apcg.APCG_SOLVE_MAXIT and res["iterations"] == 0 and not x.any()
    ref = oracle.pcg(A, b, rtol=1e-10, maxit=1)
    res, x = gpu_solve(apcg, ctx, A, b, 1e-10, 1)
    assert res["status"] == ref.status == apcg.APCG_SOLVE_MAXIT and res["iterations"] == 1
    assert rel(x, ref.x) <= 1e-13
    # nonzero x0 and the preconditioned norm
    x0 = np.random.default_rng(3).uniform(-1, 1, A.n)
    ref = oracle.pcg(A, b, x0=x0, rtol=1e-10, maxit=5000, norm_type=oracle.NORM_PRECONDITIONED)
    res, x = gpu_solve(apcg, ctx, A, b, 1e-10, 5000, x0=x0, x0_is_zero=0, norm_type=1)
    assert res["status"] == apcg.APCG_SOLVE_CONVERGED and abs(res["iterations"] - ref.its) <= 1
    assert rel(x, ref.x) <= 1e-9
    # x0 = the solution: converged before the first iteration
    res, x = gpu_solve(apcg, ctx, A, b, 1e-6, 100, x0=ref.x, x0_is_zero=0)
    assert res["status"] == apcg.APCG_SOLVE_CONVERGED and res["iterations"] == 0
    assert np.array_equal(x, ref.x)
    # a diagonal entry that is not positive: setup error under Jacobi
    Ab = P.laplace_2d(9)
    k = int(np.nonzero(Ab.col[Ab.rowptr[4]:Ab.rowptr[5]] == 4)[0][0]) + Ab.rowptr[4]
    Ab.val[k] = -4.0
    res, _ = gpu_solve(apcg, ctx, Ab, np.ones(Ab.n), 1e-10, 100)
    assert res["status"] == apcg.APCG_SOLVE_SETUP_ERROR
    # an indefinite operator without preconditioning: p.Ap <= 0 breakdown
    Ai = P.laplace_2d(9)
    Ai.val = -Ai.val
    refi = oracle.pcg(Ai, np.ones(Ai.n), rtol=1e-10, maxit=100, pc=0)
    res, _ = gpu_solve(apcg, ctx, Ai, np.ones(Ai.n), 1e-10, 100, pc=0)
    assert res["status"] == refi.status == apcg.APCG_SOLVE_BREAKDOWN_PAP and res["iterations"] == refi.its


def test_auto_mode_and_limits(apcg, ctx):
    """AUTO takes the persistent solve at n <= 4096 (same bits as asking for
    it) and the graph solve above; PERSISTENT above the limit is an error.
    Repeated persistent solves are bit for bit equal."""
    A, b = system(7, 3500, 31)
    r1, x1 = gpu_solve(apcg, ctx, A, b, 1e-10, 5000, mode=PERSISTENT)
    r2, x2 = gpu_solve(apcg, ctx, A, b, 1e-10, 5000, mode=AUTO)
    r3, x3 = gpu_solve(apcg, ctx, A, b, 1e-10, 5000, mode=PERSISTENT)
    assert r1 == r2 == r3 and np.array_equal(x1, x2) and np.array_equal(x1, x3)
    B, bb = system(5, 5000, 32)
    assert B.n > 4096
    rg, xg = gpu_solve(apcg, ctx, B, bb, 1e-10, 5000, mode=0)
    ra, xa = gpu_solve(apcg, ctx, B, bb, 1e-10, 5000, mode=AUTO)
    assert rg == ra and np.array_equal(xg, xa)
    with pytest.raises(apcg.ApcgError):
        gpu_solve(apcg, ctx, B, bb, 1e-10, 5000, mode=PERSISTENT)


def test_latency_floors(apcg):
    f = apcg.apcg_latency_floors(0, 2000)
    print(f"latency floors: {f}", flush=True)
    for k, v in f.items():
        assert 0.0 < v < 1000.0, (k, v)
    # a kernel's queueing floor is below a host round trip
    assert f["graph_node_us"] < f["host_round_trip_us"]
