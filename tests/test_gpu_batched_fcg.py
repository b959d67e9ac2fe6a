"""GPU parity of the batched FCG(1) solve (each system with its own
polynomial and its own device-side fallback to Jacobi-PCG) against the
oracle's FCG, system by system, through the C ABI.

Bar (as for the single solves): status equal, iterations +-1, flexible
iterations +-1 and ||x - x_ref|| / ||x_ref|| <= 1e-9 at rtol 1e-10; the
fallback restarts from the recursive residual where the oracle recomputes
b - A x, which only changes rounding.
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


def cheb_coeffs(lmax, a):
    from numpy.polynomial import chebyshev as Ch

    T9 = [0] * 9 + [1]
    s0 = (lmax + a) / (lmax - a)

    def f(y):
        t = (y + 1) * lmax / 2
        return (1 - Ch.chebval((lmax + a - 2 * t) / (lmax - a), T9) / Ch.chebval(s0, T9)) / t

    return Ch.chebinterpolate(f, 8)


def one_row(d, bval):
    A = P.CSR(n=1, rowptr=np.array([0, 1], np.int32), col=np.array([0], np.int32), val=np.array([d]))
    return A, np.array([bval])


def mixed_cases():
    """(A, b, c (float32[9]), lmax, label) covering the paths."""
    rng = np.random.default_rng(61)
    out = []
    for k, (dim, side, sigma, aniso) in enumerate([(2, 30, 1.0, 1.0), (3, 11, 1.5, 20.0), (2, 47, 2.0, 5.0),
                                                   (3, 9, 0.7, 1.0), (2, 5, 1.0, 1.0)]):
        s = P._lognormal_system(rng, dim, side, sigma, aniso)
        lm = oracle.gershgorin(s.A)[1]
        out.append((s.A, s.b, cheb_coeffs(lm, lm / (20 + 10 * k)).astype(np.float32), lm, f"cheb{dim}d_{side}"))
    s = P._lognormal_system(rng, 2, 20, 1.0, 1.0)
    lm = oracle.gershgorin(s.A)[1]
    e0 = np.zeros(9, np.float32)
    e0[0] = 1
    out.append((s.A, s.b, e0, lm, "identity_poly"))
    bad = np.zeros(9, np.float32)
    bad[0], bad[1] = 0.2, -0.5
    s = P._lognormal_system(rng, 2, 24, 1.0, 1.0)
    out.append((s.A, s.b, bad, oracle.gershgorin(s.A)[1], "rejected_poly"))
    A1, b1 = one_row(4.0, 2.0)
    out.append((A1, b1, e0, 1.0, "one_row"))
    s = P._lognormal_system(rng, 2, 12, 1.0, 1.0)
    out.append((s.A, np.zeros(s.A.n), cheb_coeffs(2.0, 0.04).astype(np.float32), 2.0, "zero_rhs"))
    Ab = P.laplace_2d(6)
    k = Ab.rowptr[0] + int(np.nonzero(Ab.col[Ab.rowptr[0]:Ab.rowptr[1]] == 0)[0][0])
    Ab.val[k] = -1.0  # row 0's diagonal: Jacobi is undefined
    out.append((Ab, np.ones(Ab.n), e0, 2.0, "bad_diagonal"))
    return out


def run_batch(apcg, ctx, cases, rtol, maxit, x0=None, fopts=None, sdia=False, **opt):
    import torch
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    As = [DeviceCSR(c[0]) for c in cases]
    run_batch.mats = As
    run_batch.switched = []
    if sdia:  # every matrix whose pattern allows it on the sliced-diagonal schedule
        for i, a in enumerate(As):
            try:
                apcg.apcg_mat_set_spmv_config(a.h, 1, 256, 0, apcg.APCG_SPMV_SDIA)
                run_batch.switched.append(i)
            except apcg.ApcgError:
                pass
    bs = [DeviceVec(c[1]) for c in cases]
    xs = [DeviceVec(np.zeros(c[0].n) if x0 is None else x0[i]) for i, c in enumerate(cases)]
    coef = torch.from_numpy(np.concatenate([c[2] for c in cases]).astype(np.float32)).to("cuda:0")
    lm = torch.from_numpy(np.array([c[3] for c in cases], np.float64)).to("cuda:0")
    torch.cuda.synchronize()
    info = apcg.apcg_info_create(0, len(cases))
    if x0 is None and "x0_is_zero" not in opt:
        opt["x0_is_zero"] = 1
    opts = apcg.apcg_solve_opts_default(**opt)
    fo = apcg.apcg_fcg_opts_default(**(fopts or {}))
    apcg.apcg_ksp_solve_batched_fcg_poly(ctx, [a.h for a in As], [b.h for b in bs], [x.h for x in xs], rtol, maxit,
                                         coef, lm, opts, fo, info)
    res = [apcg.apcg_info_get(info, i) for i in range(len(cases))]
    xo = [x.numpy() for x in xs]
    apcg.apcg_info_destroy(info)
    return res, xo


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def check_against_oracle(apcg, cases, res, xs, rtol, maxit, x0=None, **fo):
    for i, (A, b, c, lm, name) in enumerate(cases):
        ref = oracle.fcg_poly(A, b, c.astype(np.float64), lm, x0=None if x0 is None else x0[i], rtol=rtol,
                              maxit=maxit, **fo)
        r = res[i]
        print(f"  {name}: gpu its {r['iterations']} fcg {r['fcg_iterations']} st {r['status']} | "
              f"oracle its {ref.its} fcg {ref.fcg_its} st {ref.status}", flush=True)
        assert r["status"] == ref.status, name
        assert abs(r["iterations"] - ref.its) <= 1, name
        assert abs(r["fcg_iterations"] - ref.fcg_its) <= 1, name
        if ref.status & oracle.CONVERGED:
            assert rel(xs[i], ref.x) <= 1e-9, name


@pytest.mark.parametrize("mode", [0, 1])
def test_mixed_batch_parity(apcg, ctx, mode):
    print(f"case batched-fcg mixed mode={mode}", flush=True)
    cases = mixed_cases()
    res, xs = run_batch(apcg, ctx, cases, 1e-10, 20000, mode=mode)
    check_against_oracle(apcg, cases, res, xs, 1e-10, 20000)
    names = [c[4] for c in cases]
    rj = res[names.index("rejected_poly")]
    assert rj["fcg_iterations"] == 0 and rj["status"] & apcg.APCG_SOLVE_FALLBACK
    assert res[names.index("bad_diagonal")]["status"] == apcg.APCG_SOLVE_SETUP_ERROR
    z = names.index("zero_rhs")
    assert res[z]["iterations"] == 0 and np.all(xs[z] == 0)


def test_graph_and_stream_bitwise_and_repeatable(apcg, ctx):
    cases = mixed_cases()
    runs = [run_batch(apcg, ctx, cases, 1e-9, 20000, mode=m) for m in (0, 0, 1)]
    for res, xs in runs[1:]:
        assert res == runs[0][0]
        assert all(np.array_equal(a, b) for a, b in zip(xs, runs[0][1]))


def test_without_fallback_and_with_x0(apcg, ctx):
    cases = mixed_cases()
    res, xs = run_batch(apcg, ctx, cases, 1e-10, 20000, fopts={"fallback": 0})
    check_against_oracle(apcg, cases, res, xs, 1e-10, 20000, fallback=False)
    names = [c[4] for c in cases]
    rj = names.index("rejected_poly")
    assert res[rj]["status"] == apcg.APCG_SOLVE_BREAKDOWN_RZ and np.all(xs[rj] == 0)
    # nonzero initial guesses (the zero right-hand side still returns x = 0)
    rng = np.random.default_rng(5)
    x0 = [rng.uniform(-1, 1, c[0].n) for c in cases]
    res, xs = run_batch(apcg, ctx, cases, 1e-10, 20000, x0=x0, x0_is_zero=0)
    check_against_oracle(apcg, cases, res, xs, 1e-10, 20000, x0=x0)
    assert np.all(xs[names.index("zero_rhs")] == 0)


def test_iteration_cap_and_stall_window(apcg, ctx):
    cases = [c for c in mixed_cases() if c[4] not in ("bad_diagonal",)]
    res, xs = run_batch(apcg, ctx, cases, 1e-12, 5)
    for i, (A, b, c, lm, name) in enumerate(cases):
        ref = oracle.fcg_poly(A, b, c.astype(np.float64), lm, rtol=1e-12, maxit=5)
        assert res[i]["status"] == ref.status and res[i]["iterations"] == ref.its, name
        assert rel(xs[i], ref.x) <= 1e-11, name
    # a window of one iteration: the first iteration without a new minimum of
    # ||r|| hands the system to Jacobi-PCG
    e0 = np.zeros(9, np.float32)
    e0[0] = 1
    rng = np.random.default_rng(77)
    sts = [P._lognormal_system(rng, 2, side, 2.0, 1.0) for side in (30, 40, 25)]
    cases = [(s.A, s.b, e0, oracle.gershgorin(s.A)[1], f"stall{i}") for i, s in enumerate(sts)]
    fo = {"stall_min": 1, "stall_frac": 0.0}
    res, xs = run_batch(apcg, ctx, cases, 1e-10, 20000, fopts=fo)
    check_against_oracle(apcg, cases, res, xs, 1e-10, 20000, **fo)
    assert all(r["status"] & apcg.APCG_SOLVE_STALL for r in res)


def feature_systems():
    rng = np.random.default_rng(91)
    out = [P._lognormal_system(rng, 2, 40, 2.0, 1.0), P._lognormal_system(rng, 3, 12, 1.5, 20.0),
           P._lognormal_system(rng, 3, 7, 0.5, 3.0)]
    sys_ = [(s.A, s.b) for s in out]
    lap = P.laplace_2d(20)
    sys_.append((lap, rng.uniform(-1, 1, lap.n)))
    sys_.append(one_row(2.0, 3.0))
    z = P.laplace_2d(5)
    sys_.append((z, np.zeros(z.n)))
    return sys_


def test_batched_features_parity(apcg, ctx):
    """Features of a mixed batch in one call against the oracle, system by
    system (incl. n = 1 and b = 0)."""
    import torch
    from oracle import learned as OL
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    sys_ = feature_systems()
    As = [DeviceCSR(A) for A, _ in sys_]
    bs = [DeviceVec(b) for _, b in sys_]
    feat = torch.zeros(16 * len(sys_), dtype=torch.float32, device="cuda:0")
    lm = torch.zeros(len(sys_), dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    apcg.apcg_pc_features_batched(ctx, [a.h for a in As], [b.h for b in bs], feat, lm)
    apcg.apcg_ctx_synchronize(ctx)
    F = feat.cpu().numpy().astype(np.float64).reshape(len(sys_), 16)
    L = lm.cpu().numpy()
    for i, (A, b) in enumerate(sys_):
        ref = OL.features(A, b)
        print(f"  system {i} n={A.n}: max |diff| {np.max(np.abs(F[i] - ref)):.2e}", flush=True)
        assert np.all(np.abs(F[i] - ref) <= 2e-6 * np.maximum(1.0, np.abs(ref))), (i, F[i], ref)
        assert L[i] == pytest.approx(oracle.gershgorin(A)[1], rel=1e-15)


def test_batched_learned_solve_equals_its_steps(apcg, ctx):
    """apcg_ksp_solve_batched_learned = batched features -> standardise ->
    network -> apcg_ksp_solve_batched_fcg_poly, bit for bit; every system
    converges (through its fallback where the polynomial is rejected)."""
    import torch
    from oracle import learned as OL
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    sys_ = [s for s in feature_systems()]
    As = [DeviceCSR(A) for A, _ in sys_]
    bs = [DeviceVec(b) for _, b in sys_]
    nsys = len(sys_)
    params = P.mlp_initial_params(3)
    params["b3"] = np.array([1.2, -0.5, 0.2, -0.05, 0, 0, 0, 0, 0])
    pv = np.concatenate([params[k].reshape(-1) for k, _ in OL.SHAPES]).astype(np.float32)
    dev = lambda a, dt=torch.float32: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0", dt)
    dP, dM, dS = dev(pv), dev(np.linspace(-1, 1, 16).astype(np.float32)), dev(np.linspace(0.5, 3, 16).astype(np.float32))
    feat = torch.zeros((nsys, 16), dtype=torch.float32, device="cuda:0")
    lm = torch.zeros(nsys, dtype=torch.float64, device="cuda:0")
    C = torch.zeros((nsys, 9), dtype=torch.float32, device="cuda:0")
    torch.cuda.synchronize()
    opts = apcg.apcg_solve_opts_default(x0_is_zero=1)
    info = apcg.apcg_info_create(0, 2 * nsys)
    x1 = [DeviceVec.zeros(A.n) for A, _ in sys_]
    x2 = [DeviceVec.zeros(A.n) for A, _ in sys_]
    apcg.apcg_pc_features_batched(ctx, [a.h for a in As], [b.h for b in bs], feat.view(-1), lm)
    apcg.apcg_mlp_standardize(ctx, feat, dM, dS, False)
    apcg.apcg_mlp_forward(ctx, dP, feat, C)
    info1 = apcg.apcg_info_create(0, nsys)
    info2 = apcg.apcg_info_create(0, nsys)
    apcg.apcg_ksp_solve_batched_fcg_poly(ctx, [a.h for a in As], [b.h for b in bs], [x.h for x in x1], 1e-9, 20000,
                                         C.view(-1), lm, opts, None, info1)
    apcg.apcg_ksp_solve_batched_learned(ctx, [a.h for a in As], [b.h for b in bs], [x.h for x in x2], 1e-9, 20000,
                                        dP, dM, dS, opts, None, info2)
    r1 = [apcg.apcg_info_get(info1, i) for i in range(nsys)]
    r2 = [apcg.apcg_info_get(info2, i) for i in range(nsys)]
    assert r1 == r2
    for i in range(nsys):
        assert r1[i]["status"] & apcg.APCG_SOLVE_CONVERGED, (i, r1[i])
        assert np.array_equal(x1[i].numpy(), x2[i].numpy())
    for inf in (info, info1, info2):
        apcg.apcg_info_destroy(inf)


@pytest.mark.parametrize("mode", [0, 1])
def test_sliced_diagonal_systems_bitwise(apcg, ctx, mode):
    """Systems whose matrices are on the sliced-diagonal schedule have the
    tile products and Clenshaw steps read that copy; each row's sum is the
    CSR one, so the batch is bit for bit the all-CSR batch, and the oracle's
    bar holds."""
    cases = mixed_cases()
    print(f"case batched fcg sdia mode={mode}", flush=True)
    r_csr, x_csr = run_batch(apcg, ctx, cases, 1e-10, 20000, mode=mode)
    r_sd, x_sd = run_batch(apcg, ctx, cases, 1e-10, 20000, sdia=True, mode=mode)
    print("switched", run_batch.switched, flush=True)
    assert len(run_batch.switched) >= 3
    for a, b2, xa, xb in zip(r_csr, r_sd, x_csr, x_sd):
        assert a == b2
        assert np.array_equal(xa, xb)
    check_against_oracle(apcg, cases, r_sd, x_sd, 1e-10, 20000)


@pytest.mark.parametrize("sdia", [False, True])
def test_tail_plan_bitwise(apcg, ctx, sdia):
    """Once the rows still running fill fewer than two large tiles per
    compute unit, the iteration continues on a plan of smaller tiles (the
    tiles only group slices, so the sums do not change).  These batches are
    below that size from the start, so the switch comes at the first poll:
    4096-row tiles with the tail plan at 256 or 512 rows are bit for bit the
    run that keeps its tiles, and the oracle's bar holds."""
    cases = mixed_cases()
    rng = np.random.default_rng(65)
    s = P._lognormal_system(rng, 2, 120, 1.0, 1.0)
    lm = oracle.gershgorin(s.A)[1]
    cases.append((s.A, s.b, cheb_coeffs(lm, lm / 30).astype(np.float32), lm, "long2d_120"))
    print(f"case batched fcg tail plan sdia={sdia}", flush=True)
    runs = [run_batch(apcg, ctx, cases, 1e-10, 20000, sdia=sdia, batch_tile_rows=4096, batch_tail_tile_rows=tt)
            for tt in (-1, 256, 0)]
    for res, xs in runs[1:]:
        assert res == runs[0][0]
        assert all(np.array_equal(a, b) for a, b in zip(xs, runs[0][1]))
    check_against_oracle(apcg, cases, *runs[0], 1e-10, 20000)


def test_tail_rows_rejected(apcg, ctx):
    cases = mixed_cases()[:2]
    for bad in (-2, 100, 9000):
        with pytest.raises(apcg.ApcgError):
            run_batch(apcg, ctx, cases, 1e-10, 100, batch_tail_tile_rows=bad)


def unsymmetric_twin(A, frac=0.3):
    """A copy of A with the same (symmetric) pattern whose values are no
    longer symmetric: one entry left of the diagonal changed in its last
    bits."""
    T = P.CSR(n=A.n, rowptr=A.rowptr.copy(), col=A.col.copy(), val=A.val.copy())
    for i in range(int(frac * A.n), A.n):
        lo = [e for e in range(A.rowptr[i], A.rowptr[i + 1]) if A.col[e] < i]
        if lo:
            T.val[lo[0]] *= 1.0 + 2.0 ** -40
            return T
    raise AssertionError("no entry left of the diagonal")


def test_sliced_diagonals_multi_tile_bitwise(apcg, ctx):
    """The tile product and every Clenshaw step walk the sliced-diagonal copy
    (scalar loads of offsets and masks, gathers clamped into the system):
    bit for bit the all-CSR batch on 2D and 3D systems over several tiles,
    symmetric or with unsymmetric values, at two tile sizes; the oracle's
    bar holds."""
    rng = np.random.default_rng(64)
    cases = []
    for dim, side, sigma, aniso in [(2, 75, 1.0, 3.0), (3, 17, 1.0, 1.0), (2, 110, 1.5, 1.0), (3, 21, 0.7, 5.0)]:
        s = P._lognormal_system(rng, dim, side, sigma, aniso)
        lm = oracle.gershgorin(s.A)[1]
        cases.append((s.A, s.b, cheb_coeffs(lm, lm / 40).astype(np.float32), lm, f"sym{dim}d_{side}"))
    for A, b, c, lm, name in cases[:2]:
        cases.append((unsymmetric_twin(A), b, c, lm, name + "_twin"))
    flags = [1, 1, 1, 1, 0, 0]
    print("case batched fcg sliced diagonals multi-tile", flush=True)
    r_csr, x_csr = run_batch(apcg, ctx, cases, 1e-10, 20000)
    for tr in (256, 2048):
        r_sd, x_sd = run_batch(apcg, ctx, cases, 1e-10, 20000, sdia=True, batch_tile_rows=tr)
        assert run_batch.switched == list(range(len(cases)))
        assert [apcg.apcg_mat_get_sdia_info(a.h)["values_symmetric"] for a in run_batch.mats] == flags
        for a, b2, xa, xb in zip(r_csr, r_sd, x_csr, x_sd):
            assert a == b2
            assert np.array_equal(xa, xb)
    check_against_oracle(apcg, cases[:4], r_csr[:4], x_csr[:4], 1e-10, 20000)


@pytest.mark.parametrize("sdia", [False, True])
def test_tile_rows_bitwise(apcg, ctx, sdia):
    """The batched FCG at 256, 1024 and 4096 rows per tile: tiles only group
    64-row slices for a workgroup, every slice's partials are its own
    wavefront's sums and each system adds its slices in index order, so the
    whole run (flexible phases, rejected polynomials and fallbacks included)
    is bit for bit the same at every tile size; the first run meets the
    oracle's bar."""
    cases = mixed_cases()
    print(f"case batched fcg tile rows sdia={sdia}", flush=True)
    runs = [run_batch(apcg, ctx, cases, 1e-10, 20000, sdia=sdia, batch_tile_rows=tr) for tr in (256, 1024, 4096)]
    for res, xs in runs[1:]:
        assert res == runs[0][0]
        assert all(np.array_equal(a, b) for a, b in zip(xs, runs[0][1]))
    check_against_oracle(apcg, cases, *runs[0], 1e-10, 20000)
