"""GPU tests of the asynchronous Vec/Mat/scalar calls against the oracle.

Reductions are compared with the exactly rounded sum (math.fsum) within the
worst-case bound of a length-n dot product, n u sum|x_i y_i| (u = 2^-53)
for any summation order; elementwise updates are compared bit for bit with
numpy where the kernel computes the same single rounding (fma vs a*b+c is
allowed to differ by one rounding, so those use a 1-ulp-scale bound)."""
import math

import numpy as np
import pytest

import oracle
from paper_2306_17801_amd import problems as P

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
SIZES = [0, 1, 63, 64, 65, 1000, 100003, 1 << 20]


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


def dvec(v):
    from paper_2306_17801_amd.device import DeviceVec

    return DeviceVec(np.asarray(v, dtype=np.float64))


@pytest.mark.parametrize("n", SIZES)
def test_dot_and_norm(apcg, ctx, n):
    print(f"case dot n={n}", flush=True)
    rng = np.random.default_rng(n + 1)
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    dx, dy = dvec(x), dvec(y)
    s = apcg.apcg_scalar_create(ctx)
    apcg.apcg_vec_dot_async(dx.h, dy.h, s, ctx)
    got = apcg.apcg_scalar_get(s)
    exact = math.fsum(x * y) if n else 0.0
    bound = n * U * float(np.sum(np.abs(x * y))) * 1.01 + 1e-300
    assert abs(got - exact) <= bound
    apcg.apcg_vec_norm2_async(dx.h, s, ctx)
    got = apcg.apcg_scalar_get(s)
    assert got == pytest.approx(math.sqrt(math.fsum(x * x)) if n else 0.0, rel=4 * (n + 1) * U, abs=1e-300)
    # deterministic: the same call gives the same bits
    apcg.apcg_vec_dot_async(dx.h, dy.h, s, ctx)
    a = apcg.apcg_scalar_get(s)
    apcg.apcg_vec_dot_async(dx.h, dy.h, s, ctx)
    assert apcg.apcg_scalar_get(s) == a
    apcg.apcg_scalar_destroy(s)


@pytest.mark.parametrize("n", [1, 65, 100003])
def test_axpy_aypx_scale_copy_set(apcg, ctx, n):
    rng = np.random.default_rng(n + 7)
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    a = apcg.apcg_scalar_create(ctx)
    apcg.apcg_scalar_set(a, 0.375, ctx)  # exactly representable: products are exact-ish
    dx, dy = dvec(x), dvec(y)
    apcg.apcg_vec_axpy_async(dy.h, a, False, dx.h, ctx)
    assert np.allclose(dy.numpy(), y + 0.375 * x, rtol=2 * U, atol=4 * U)
    apcg.apcg_vec_axpy_async(dy.h, a, True, dx.h, ctx)  # y - a x
    assert np.allclose(dy.numpy(), (y + 0.375 * x) - 0.375 * x, rtol=4 * U, atol=8 * U)
    dy2 = dvec(y)
    apcg.apcg_vec_aypx_async(dy2.h, a, dx.h, ctx)  # y = x + a y
    assert np.allclose(dy2.numpy(), x + 0.375 * y, rtol=2 * U, atol=4 * U)
    apcg.apcg_vec_scale_async(dx.h, a, ctx)
    assert np.array_equal(dx.numpy(), 0.375 * x)
    dz = dvec(np.zeros(n))
    apcg.apcg_vec_copy_async(dz.h, dx.h, ctx)
    assert np.array_equal(dz.numpy(), 0.375 * x)
    apcg.apcg_vec_set_async(dz.h, -2.5, ctx)
    assert np.all(dz.numpy() == -2.5)
    apcg.apcg_vec_copy_from_host(dz.h, x, ctx)
    assert np.array_equal(dz.numpy(), x)
    apcg.apcg_scalar_destroy(a)


def test_scalar_ops(apcg, ctx):
    a, b, o = (apcg.apcg_scalar_create(ctx) for _ in range(3))
    apcg.apcg_scalar_set(a, 6.0, ctx)
    apcg.apcg_scalar_set(b, 4.0, ctx)
    cases = [(apcg.APCG_SCALAR_COPY, None, 6.0), (apcg.APCG_SCALAR_NEG, None, -6.0),
             (apcg.APCG_SCALAR_RECIP, None, 1 / 6.0), (apcg.APCG_SCALAR_SQRT, None, math.sqrt(6.0)),
             (apcg.APCG_SCALAR_ADD, b, 10.0), (apcg.APCG_SCALAR_SUB, b, 2.0),
             (apcg.APCG_SCALAR_MUL, b, 24.0), (apcg.APCG_SCALAR_DIV, b, 1.5)]
    for op, bb, want in cases:
        apcg.apcg_scalar_op(op, o, a, bb, ctx)
        assert apcg.apcg_scalar_get(o) == want
    # in place: a = a / b
    apcg.apcg_scalar_op(apcg.APCG_SCALAR_DIV, a, a, b, ctx)
    assert apcg.apcg_scalar_get(a) == 1.5
    with pytest.raises(apcg.ApcgError):
        apcg.apcg_scalar_op(apcg.APCG_SCALAR_DIV, o, a, None, ctx)
    with pytest.raises(apcg.ApcgError):
        apcg.apcg_scalar_op(99, o, a, None, ctx)
    for s in (a, b, o):
        apcg.apcg_scalar_destroy(s)


def test_async_normalize_without_host_sync(apcg, ctx):
    """The normalisation example of Section 3.3: norm, reciprocal on the
    device, scale -- no host synchronisation until the accessor."""
    v = np.random.default_rng(5).uniform(-1, 1, 1 << 16)
    dv = dvec(v)
    al = apcg.apcg_scalar_create(ctx)
    apcg.apcg_counters_reset()
    apcg.apcg_vec_norm2_async(dv.h, al, ctx)
    apcg.apcg_scalar_op(apcg.APCG_SCALAR_RECIP, al, al, None, ctx)
    apcg.apcg_vec_scale_async(dv.h, al, ctx)
    c = apcg.apcg_counters_get()
    assert c["host_syncs"] == 0 and c["d2h_copies"] == 0
    out = dv.numpy()
    assert abs(oracle.norm2(out) - 1.0) <= 4 * U * math.sqrt(out.size)
    apcg.apcg_scalar_destroy(al)


def _spmv_bound(A, x):
    """Per-row bound 2 gamma_k sum |a_ij x_j| for two summation orders."""
    absA = P.CSR(n=A.n, rowptr=A.rowptr, col=A.col, val=np.abs(A.val))
    k = np.maximum(np.diff(A.rowptr), 1)
    return 2.0 * k * U / (1 - k * U) * oracle.spmv(absA, np.abs(x)) + 1e-300


@pytest.mark.parametrize("schedule,lpr,tb", [(0, 1, 256), (0, 2, 256), (0, 4, 512), (0, 8, 256), (0, 32, 512),
                                             (1, 1, 256), (1, 1, 512), (2, 1, 256)])
@pytest.mark.parametrize("which", ["random_empty_rows", "stencil3d", "ragged2d"])
def test_spmv_against_oracle(apcg, ctx, schedule, lpr, tb, which):
    from paper_2306_17801_amd.device import DeviceCSR

    print(f"case spmv {which} schedule={schedule} lpr={lpr} tb={tb}", flush=True)
    if which == "random_empty_rows":
        A = P.random_csr(3001, 9, seed=3, empty_rows=True)
    elif which == "stencil3d":
        A = P.diffusion_csr(np.exp(np.random.default_rng(2).standard_normal((19, 23, 29))), aniso=3.0)
    else:
        A = P.diffusion_csr(np.exp(np.random.default_rng(3).standard_normal((37, 41))))
    x = np.random.default_rng(9).uniform(-1, 1, A.n)
    dA = DeviceCSR(A)
    apcg.apcg_mat_set_spmv_config(dA.h, lpr, tb, 0, schedule)
    dx, dy = dvec(x), dvec(np.zeros(A.n))
    apcg.apcg_mat_mult_async(dA.h, dx.h, dy.h, ctx)
    y = dy.numpy()
    ref = oracle.spmv(A, x)
    assert np.all(np.abs(y - ref) <= _spmv_bound(A, x))


def test_staged_schedule_rejects_long_rows(apcg):
    """A 6000-entry row puts 6255 nonzeros in the first 256-row block (6511
    in the first 512-row block): more than the 5376 the LDS stage holds, so
    the staged schedule is refused and not chosen by default."""
    from paper_2306_17801_amd.device import DeviceCSR

    big = 6000
    rp = np.zeros(big + 1, np.int64)
    cnt = np.ones(big, np.int64)
    cnt[0] = big
    rp[1:] = np.cumsum(cnt)
    cl = np.concatenate([np.arange(big)] + [np.array([i]) for i in range(1, big)]).astype(np.int32)
    B = P.CSR(n=big, rowptr=rp.astype(np.int32), col=cl, val=np.ones(int(rp[-1])))
    dB = DeviceCSR(B)
    assert apcg.apcg_mat_get_spmv_config(dB.h)["schedule"] == 0
    for tb in (256, 512):
        with pytest.raises(apcg.ApcgError) as e:
            apcg.apcg_mat_set_spmv_config(dB.h, 1, tb, 0, 1)
        assert e.value.code == apcg.APCG_ERR_UNSUPPORTED


def test_autotune_picks_a_valid_schedule(apcg, ctx):
    from paper_2306_17801_amd.device import DeviceCSR

    A = P.laplace_3d(40)
    dA = DeviceCSR(A)
    cfg, us = apcg.apcg_mat_autotune(dA.h, ctx, 3)
    assert us > 0 and cfg["block_size"] in (256, 512) and cfg["schedule"] in (0, 1, 2, 3)
    assert apcg.apcg_mat_get_spmv_config(dA.h) == cfg


@pytest.mark.parametrize("spmv", [(1, 256, 0, 0), (1, 512, 64, 2), (4, 512, 0, 3), (1, 256, 0, 3)])
def test_time_kernels(apcg, ctx, spmv):
    """Back-to-back timing of the product and update kernels at the matrix's
    configuration: positive means, the configuration unchanged, and the
    matrix still solves to the oracle's bar afterwards (the timing runs on
    scratch vectors)."""
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    A = P.laplace_3d(24)
    dA = DeviceCSR(A)
    apcg.apcg_mat_set_spmv_config(dA.h, *spmv)
    before = apcg.apcg_mat_get_spmv_config(dA.h)
    print(f"case time_kernels spmv={spmv}", flush=True)
    pu, uu = apcg.apcg_mat_time_kernels(dA.h, ctx, 5)
    assert pu > 0 and uu > 0 and pu < 1e5 and uu < 1e5
    assert apcg.apcg_mat_get_spmv_config(dA.h) == before
    b = np.random.default_rng(53).uniform(-1, 1, A.n)
    db, dx = DeviceVec(b), DeviceVec.zeros(A.n)
    info = apcg.apcg_info_create(0, 1)
    apcg.apcg_ksp_solve(ctx, dA.h, db.h, dx.h, 1e-10, 5000, apcg.apcg_solve_opts_default(x0_is_zero=1), info, 0)
    res = apcg.apcg_info_get(info, 0)
    apcg.apcg_info_destroy(info)
    ref = oracle.pcg(A, b, rtol=1e-10, maxit=5000)
    assert res["status"] == apcg.APCG_SOLVE_CONVERGED and abs(res["iterations"] - ref.its) <= 1
    assert np.linalg.norm(dx.numpy() - ref.x) <= 1e-9 * np.linalg.norm(ref.x)
