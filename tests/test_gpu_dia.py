"""GPU parity of the diagonal (DIA) product schedule, through the C ABI.

The diagonal product adds every row's entries in offset (= column) order
with one fused multiply-add each, the absent entries adding exact zeros, and
walks the rows of the row-per-thread schedule (lanes_per_row 1) in the same
order, so at the same launch shape a whole solve is bit for bit that of the
row-per-thread schedule; every solve meets the oracle's bar (iterations +-1,
||x - x_ref|| / ||x_ref|| <= 1e-9 at rtol 1e-10).
"""
import numpy as np
import pytest

import oracle
from paper_2306_17801_amd import problems as P

pytestmark = pytest.mark.gpu

DIA = 4


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


def gpu_solve(apcg, ctx, A, b, rtol, maxit, spmv=None, info_out=None, **opt):
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    dA, db, dx = DeviceCSR(A), DeviceVec(b), DeviceVec.zeros(A.n)
    opt.setdefault("x0_is_zero", 1)
    if spmv is not None:
        apcg.apcg_mat_set_spmv_config(dA.h, *spmv)
    info = apcg.apcg_info_create(0, 1)
    apcg.apcg_ksp_solve(ctx, dA.h, db.h, dx.h, rtol, maxit, apcg.apcg_solve_opts_default(**opt), info, 0)
    res = apcg.apcg_info_get(info, 0)
    x = dx.numpy()
    if info_out is not None:
        info_out.append(apcg.apcg_mat_get_dia_info(dA.h))
    apcg.apcg_info_destroy(info)
    for v in (dx, db):
        v.close()
    dA.close()
    return res, x


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def with_lower_value_changed(A, factor):
    """A copy of A whose first entry left of the diagonal in a middle row is
    scaled: the pattern stays symmetric, the values do not."""
    row = A.n // 2 + 3
    k = int(A.rowptr[row])
    assert A.col[k] < row
    val = A.val.copy()
    val[k] *= factor
    return P.CSR(n=A.n, rowptr=A.rowptr, col=A.col, val=val)


def laplace1d(n):
    import scipy.sparse as sp

    M = sp.diags([-np.ones(n - 1), 2.5 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    M.sort_indices()
    return P.CSR(n=n, rowptr=M.indptr.astype(np.int32), col=M.indices.astype(np.int32), val=M.data.copy())


def matrix(which):
    rng = np.random.default_rng(60 + len(which))
    if which == "diffusion3d_32":
        return P.diffusion_csr(np.exp(rng.standard_normal((32, 32, 32))), aniso=3.0)
    if which == "diffusion3d_ragged":
        return P.diffusion_csr(np.exp(rng.standard_normal((13, 17, 21))), aniso=7.0)
    if which == "diffusion2d_ragged":
        return P.diffusion_csr(np.exp(1.5 * rng.standard_normal((45, 71))))
    if which == "ninepoint_40x37":
        return P.stencil_laplacian((40, 37), 9)
    if which == "laplace1d_50":
        return laplace1d(50)
    raise KeyError(which)


WHICH = ["diffusion3d_32", "diffusion3d_ragged", "diffusion2d_ragged", "ninepoint_40x37", "laplace1d_50"]


@pytest.mark.parametrize("which", WHICH)
@pytest.mark.parametrize("tb", [256, 512])
def test_dia_matches_oracle_and_row_schedule(apcg, ctx, which, tb):
    A = matrix(which)
    b = np.random.default_rng(7).uniform(-1, 1, A.n)
    ref = oracle.pcg(A, b, rtol=1e-10, maxit=20000)
    print(f"case dia {which} n={A.n} tb={tb}", flush=True)
    inf = []
    r_d, x_d = gpu_solve(apcg, ctx, A, b, 1e-10, 20000, spmv=(1, tb, 0, DIA), info_out=inf)
    assert r_d["status"] == apcg.APCG_SOLVE_CONVERGED and abs(r_d["iterations"] - ref.its) <= 1
    assert rel(x_d, ref.x) <= 1e-9
    assert inf[0]["state"] == 1 and inf[0]["offsets_symmetric"] == 1 and inf[0]["values_symmetric"] == 1
    # matched iteration count against the oracle
    ref20 = oracle.pcg(A, b, rtol=0.0, maxit=20)
    r20, x20 = gpu_solve(apcg, ctx, A, b, 0.0, 20, spmv=(1, tb, 0, DIA))
    assert r20["iterations"] == 20 and rel(x20, ref20.x) <= 1e-12


@pytest.mark.parametrize("tb,blocks", [(256, 64), (512, 32)])
def test_dia_bitwise_equal_row_schedule(apcg, ctx, tb, blocks):
    """32^3 rows at a grid whose row-per-thread chunks are whole multiples of
    64 rows: the diagonal and row-per-thread schedules walk the same rows in
    the same order, so whole solves are bit for bit equal."""
    A = matrix("diffusion3d_32")
    b = np.random.default_rng(8).uniform(-1, 1, A.n)
    assert (A.n // blocks) % 64 == 0
    r_d, x_d = gpu_solve(apcg, ctx, A, b, 1e-10, 20000, spmv=(1, tb, blocks, DIA))
    r_r, x_r = gpu_solve(apcg, ctx, A, b, 1e-10, 20000, spmv=(1, tb, blocks, 0))
    assert r_d == r_r
    assert np.array_equal(x_d, x_r)


@pytest.mark.parametrize("which", ["diffusion3d_ragged", "ninepoint_40x37"])
def test_dia_unsymmetric_values_read_as_stored(apcg, ctx, which):
    """One entry left of the diagonal scaled (pattern symmetric, values not):
    the check run with the refill clears the value-symmetry flag, the product
    reads every diagonal as stored, and the solve meets the oracle's bar for
    those values."""
    A = matrix(which)
    B = with_lower_value_changed(A, 1.5)
    b = np.random.default_rng(9).uniform(-1, 1, A.n)
    ref = oracle.pcg(B, b, rtol=1e-10, maxit=20000)
    inf = []
    r_d, x_d = gpu_solve(apcg, ctx, B, b, 1e-10, 20000, spmv=(1, 256, 0, DIA), info_out=inf)
    assert inf[0]["offsets_symmetric"] == 1 and inf[0]["values_symmetric"] == 0
    assert r_d["status"] == apcg.APCG_SOLVE_CONVERGED and abs(r_d["iterations"] - ref.its) <= 1
    assert rel(x_d, ref.x) <= 1e-9


def test_dia_symmetry_rechecked_each_solve(apcg, ctx):
    """The value-symmetry check runs with every refill: values changed in
    place between solves (symmetric, then not, then symmetric again) give
    each solve the oracle's answer for its values, and once found
    unsymmetric the matrix keeps reading every diagonal."""
    import torch
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    A = matrix("diffusion3d_ragged")
    b = np.random.default_rng(10).uniform(-1, 1, A.n)
    dA, db = DeviceCSR(A), DeviceVec(b)
    apcg.apcg_mat_set_spmv_config(dA.h, 1, 256, 0, DIA)
    info = apcg.apcg_info_create(0, 1)
    opts = apcg.apcg_solve_opts_default(x0_is_zero=1)
    seen = []
    for factor in (1.0, 1.25, 1.0):
        B = with_lower_value_changed(A, factor)
        dA.val.copy_(torch.from_numpy(B.val))
        torch.cuda.synchronize()
        dx = DeviceVec.zeros(A.n)
        apcg.apcg_ksp_solve(ctx, dA.h, db.h, dx.h, 1e-10, 5000, opts, info, 0)
        res = apcg.apcg_info_get(info, 0)
        ref = oracle.pcg(B, b, rtol=1e-10, maxit=5000)
        assert res["status"] == apcg.APCG_SOLVE_CONVERGED and abs(res["iterations"] - ref.its) <= 1
        assert rel(dx.numpy(), ref.x) <= 1e-9
        seen.append(apcg.apcg_mat_get_dia_info(dA.h)["values_symmetric"])
        dx.close()
    assert seen == [1, 0, 0]
    apcg.apcg_info_destroy(info)


def test_dia_rejected_and_info(apcg, ctx):
    """More than 9 distinct offsets (the 27-point box stencil) and a row with
    unsorted columns are rejected; an unsymmetric offset set (one stored
    zero at (0, n-1)) is accepted with the transposed reads off; a matrix
    never put on the schedule reads as not analysed."""
    from paper_2306_17801_amd.device import DeviceCSR

    A27 = P.stencil_laplacian((6, 6, 6), 27)
    d27 = DeviceCSR(A27)
    assert apcg.apcg_mat_get_dia_info(d27.h)["state"] == 0
    with pytest.raises(apcg.ApcgError):
        apcg.apcg_mat_set_spmv_config(d27.h, 1, 256, 0, DIA)
    assert apcg.apcg_mat_get_dia_info(d27.h)["state"] == -1
    A = laplace1d(40)
    col = A.col.copy()
    col[[1, 2]] = col[[2, 1]]  # row 1's first two columns swapped
    dU = DeviceCSR(P.CSR(n=A.n, rowptr=A.rowptr, col=col, val=A.val))
    with pytest.raises(apcg.ApcgError):
        apcg.apcg_mat_set_spmv_config(dU.h, 1, 256, 0, DIA)
    # one stored zero at (0, n-1): offsets {-1, 0, 1, n-1}
    rowptr = A.rowptr.copy()
    rowptr[1:] += 1
    e = int(A.rowptr[1])
    Z = P.CSR(n=A.n, rowptr=rowptr, col=np.insert(A.col, e, A.n - 1).astype(np.int32), val=np.insert(A.val, e, 0.0))
    b = np.random.default_rng(11).uniform(-1, 1, A.n)
    inf = []
    r, x = gpu_solve(apcg, ctx, Z, b, 1e-10, 1000, spmv=(1, 256, 0, DIA), info_out=inf)
    assert inf[0] == {"state": 1, "diagonals": 4, "offsets_symmetric": 0, "values_symmetric": 0}
    ref = oracle.pcg(A, b, rtol=1e-10, maxit=1000)
    assert r["status"] == apcg.APCG_SOLVE_CONVERGED and abs(r["iterations"] - ref.its) <= 1
    assert rel(x, ref.x) <= 1e-9


def test_autotuner_offers_dia(apcg, ctx):
    """The autotuner times the diagonal schedule among the others; whichever
    it picks, the solve meets the oracle's bar."""
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    A = matrix("diffusion3d_32")
    b = np.random.default_rng(12).uniform(-1, 1, A.n)
    dA, db, dx = DeviceCSR(A), DeviceVec(b), DeviceVec.zeros(A.n)
    cfg, us = apcg.apcg_mat_autotune(dA.h, ctx, 3)
    print("autotune", cfg, us, flush=True)
    assert apcg.apcg_mat_get_dia_info(dA.h)["state"] == 1  # analysed while tuning
    info = apcg.apcg_info_create(0, 1)
    apcg.apcg_ksp_solve(ctx, dA.h, db.h, dx.h, 1e-10, 5000, apcg.apcg_solve_opts_default(x0_is_zero=1), info, 0)
    res = apcg.apcg_info_get(info, 0)
    ref = oracle.pcg(A, b, rtol=1e-10, maxit=5000)
    assert res["status"] == apcg.APCG_SOLVE_CONVERGED and abs(res["iterations"] - ref.its) <= 1
    assert rel(dx.numpy(), ref.x) <= 1e-9
    apcg.apcg_info_destroy(info)


def banded(n, off=128):
    """A symmetric positive definite band matrix with offsets -off, -1, 0,
    1, off (diagonally dominant, seeded values): n need not fill whole
    planes of `off` rows or whole 64-row slices."""
    import scipy.sparse as sp

    rng = np.random.default_rng(70 + n)
    e1 = -rng.uniform(0.5, 1.5, n - 1)
    eo = -rng.uniform(0.5, 1.5, n - off)
    d = np.zeros(n)
    d[:-1] += -e1
    d[1:] += -e1
    d[:-off] += -eo
    d[off:] += -eo
    M = sp.diags([eo, e1, d + 0.1, e1, eo], [-off, -1, 0, 1, off]).tocsr()
    M.sort_indices()
    return P.CSR(n=n, rowptr=M.indptr.astype(np.int32), col=M.indices.astype(np.int32), val=M.data.copy())


def march_matrix(which):
    rng = np.random.default_rng(80 + len(which))
    if which == "diffusion3d_32":
        return matrix("diffusion3d_32")  # plane 1024 rows = 16 slices
    if which == "diffusion2d_128x40":
        return P.diffusion_csr(np.exp(rng.standard_normal((40, 128))), aniso=2.0)  # rows of 128 = 2 slices
    if which == "banded_950":
        return banded(950)  # 15 slices, the last ragged; planes of 2 slices, the last partial
    raise KeyError(which)


@pytest.mark.parametrize("which", ["diffusion3d_32", "diffusion2d_128x40", "banded_950"])
@pytest.mark.parametrize("seg,tb", [(4, 256), (8, 512), (3, 256)])
@pytest.mark.parametrize("symmetric", [True, False])
def test_dia_march_bitwise_equal_sdia_march(apcg, ctx, which, seg, tb, symmetric):
    """Diagonals with plane marching against sliced diagonals with plane
    marching at the same planes per task and workgroup size: both walk the
    same tasks (the plane stride is the same) and add each row's entries in
    column order with one FMA each (absent entries adding exact zeros), so
    whole solves are bit for bit equal -- with symmetric values (the -plane
    value carried from the previous slice, the other lower entries read as
    their transposes) and with one lower value changed (every diagonal read
    as stored).  Each solve meets the oracle's bar."""
    A = march_matrix(which)
    if not symmetric:
        A = with_lower_value_changed(A, 1.5)
    b = np.random.default_rng(13).uniform(-1, 1, A.n)
    print(f"case dia-march {which} n={A.n} seg={seg} tb={tb} symmetric={symmetric}", flush=True)
    inf = []
    r_d, x_d = gpu_solve(apcg, ctx, A, b, 1e-10, 20000, spmv=(seg, tb, 0, DIA), info_out=inf)
    assert inf[0]["values_symmetric"] == (1 if symmetric else 0)
    r_s, x_s = gpu_solve(apcg, ctx, A, b, 1e-10, 20000, spmv=(seg, tb, 0, 3))
    assert r_d == r_s
    assert np.array_equal(x_d, x_s)
    ref = oracle.pcg(A, b, rtol=1e-10, maxit=20000)
    assert r_d["status"] == apcg.APCG_SOLVE_CONVERGED and abs(r_d["iterations"] - ref.its) <= 1
    assert rel(x_d, ref.x) <= 1e-9
