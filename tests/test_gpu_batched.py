"""GPU parity of the batched persistent PCG (one launch, one system per
workgroup) against the CPU oracle, system by system, through the C ABI."""
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


def run_batch(apcg, ctx, systems, rtol, maxit, x0s=None, sdia=(), **opt):
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    As = [DeviceCSR(s.A) for s in systems]
    run_batch.switched = []
    for i in sdia:  # these systems' matrices on the sliced-diagonal schedule, where the pattern allows it
        try:
            apcg.apcg_mat_set_spmv_config(As[i].h, 1, 256, 0, apcg.APCG_SPMV_SDIA)
            run_batch.switched.append(i)
        except apcg.ApcgError:
            pass
    run_batch.mats = As
    bs = [DeviceVec(s.b) for s in systems]
    xs = [DeviceVec(np.zeros(s.A.n) if x0s is None else x0s[i]) for i, s in enumerate(systems)]
    if x0s is None:
        opt.setdefault("x0_is_zero", 1)
    info = apcg.apcg_info_create(0, len(systems))
    opts = apcg.apcg_solve_opts_default(**opt)
    apcg.apcg_ksp_solve_batched(ctx, [a.h for a in As], [b.h for b in bs], [x.h for x in xs], rtol, maxit, opts, info)
    res = [apcg.apcg_info_get(info, i) for i in range(len(systems))]
    out = [x.numpy() for x in xs]
    apcg.apcg_info_destroy(info)
    return res, out


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def mixed_small_batch():
    rng = np.random.default_rng(60)
    out = []
    for i in range(24):
        dim = 2 + (i % 2)
        side = int(rng.integers(2, 40 if dim == 2 else 14))
        out.append(P._lognormal_system(rng, dim, side, float(rng.uniform(0.5, 2.0)),
                                       float(np.exp(rng.uniform(0, np.log(50))))))
    # edge cases: one unknown, b = 0, a non-positive diagonal
    one = P.CSR(n=1, rowptr=np.array([0, 1], np.int32), col=np.array([0], np.int32), val=np.array([4.0]))
    out.append(P.System(A=one, b=np.array([2.0])))
    z = P.laplace_2d(5)
    out.append(P.System(A=z, b=np.zeros(z.n)))
    bad = P.laplace_2d(4)
    bad.val = bad.val.copy()
    bad.val[0] = -1.0  # row 0's diagonal is its first entry
    out.append(P.System(A=bad, b=np.ones(bad.n)))
    return out


@pytest.mark.parametrize("sched,tb", [(1, 256), (1, 512), (1, 1024), (2, 0)])
@pytest.mark.parametrize("mode", [0, 1])
def test_mixed_batch_matches_oracle(apcg, ctx, sched, tb, mode):
    """Persistent (one workgroup per system, three block sizes) and segmented
    schedules, graph and direct launches."""
    print(f"case batched mixed sched={sched} tb={tb} mode={mode}", flush=True)
    systems = mixed_small_batch()
    res, xs = run_batch(apcg, ctx, systems, 1e-10, 5000, batch_block_size=tb, mode=mode, batch_schedule=sched)
    for i, (s, r, x) in enumerate(zip(systems, res, xs)):
        ref = oracle.pcg(s.A, s.b, rtol=1e-10, maxit=5000)
        assert r["status"] == ref.status, (i, r, ref)
        if ref.status == oracle.CONVERGED:
            assert abs(r["iterations"] - ref.its) <= 1, (i, r, ref)
            assert rel(x, ref.x) <= 1e-9, i
    assert np.all(xs[-2] == 0)  # b = 0 -> x = 0


@pytest.mark.parametrize("sched", [1, 2])
def test_batched_initial_guess_and_maxit(apcg, ctx, sched):
    rng = np.random.default_rng(61)
    systems = [P._lognormal_system(rng, 2, int(rng.integers(8, 30)), 1.0, 1.0) for _ in range(6)]
    x0s = [rng.uniform(-1, 1, s.A.n) for s in systems]
    res, xs = run_batch(apcg, ctx, systems, 0.0, 7, x0s=x0s, batch_schedule=sched)
    for s, r, x, x0 in zip(systems, res, xs, x0s):
        ref = oracle.pcg(s.A, s.b, x0=x0, rtol=0.0, maxit=7)
        assert r["status"] == oracle.MAXIT and r["iterations"] == 7
        assert rel(x, ref.x) <= 1e-12


@pytest.mark.parametrize("sched", [1, 2])
def test_batched_deterministic_and_graph_equals_direct(apcg, ctx, sched):
    systems = mixed_small_batch()[:20]
    r1, x1 = run_batch(apcg, ctx, systems, 1e-8, 5000, mode=0, batch_schedule=sched)
    r2, x2 = run_batch(apcg, ctx, systems, 1e-8, 5000, mode=1, batch_schedule=sched)
    r3, x3 = run_batch(apcg, ctx, systems, 1e-8, 5000, mode=0, batch_schedule=sched)
    assert r1 == r2 == r3
    assert all(np.array_equal(a, b) and np.array_equal(a, c) for a, b, c in zip(x1, x2, x3))


@pytest.fixture(scope="module")
def batch256():
    return P.batch2d_lognormal(256, seed=3)


@pytest.mark.parametrize("sched", [1, 2])
def test_batch2d_first_sixteen_full_size(apcg, ctx, batch256, sched):
    """The first 16 systems of the 256-system 2D batch, at full size,
    rtol 1e-10: iterations +-1 and rel <= 1e-9 per system."""
    systems = batch256[:16]
    res, xs = run_batch(apcg, ctx, systems, 1e-10, 20000, batch_schedule=sched)
    for s, r, x in zip(systems, res, xs):
        ref = oracle.pcg(s.A, s.b, rtol=1e-10, maxit=20000)
        assert r["status"] == apcg.APCG_SOLVE_CONVERGED
        assert abs(r["iterations"] - ref.its) <= 1
        assert rel(x, ref.x) <= 1e-9


@pytest.mark.parametrize("sched", [0, 1, 2])
def test_batch2d_all_256_in_bench_configuration(apcg, ctx, batch256, sched):
    """All 256 systems at rtol 1e-8 in the launch configurations the
    benchmark times: every system converges with a true residual within
    1.5 rtol; eight sampled systems match the oracle's iteration count +-1."""
    res, xs = run_batch(apcg, ctx, batch256, 1e-8, 20000, batch_schedule=sched)
    for s, r, x in zip(batch256, res, xs):
        assert r["status"] == apcg.APCG_SOLVE_CONVERGED
        tr = np.linalg.norm(s.b - oracle.spmv(s.A, x)) / np.linalg.norm(s.b)
        assert tr <= 1.5e-8
    for i in (0, 37, 64, 101, 150, 199, 230, 255):
        ref = oracle.pcg(batch256[i].A, batch256[i].b, rtol=1e-8, maxit=20000)
        assert abs(res[i]["iterations"] - ref.its) <= 1


@pytest.mark.parametrize("mode", [0, 1])
def test_segmented_sliced_diagonal_systems_bitwise(apcg, ctx, mode):
    """Systems whose matrices are on the sliced-diagonal schedule have their
    tile products read the sliced-diagonal copy in the segmented schedule;
    each row's sum is the CSR one (column order, one FMA per entry), so the
    batch is bit for bit the all-CSR batch (every system whose pattern allows
    it switched, the others left on CSR; sizes not multiples of 64 included)."""
    systems = mixed_small_batch()[:24]
    print(f"case batched seg sdia mode={mode}", flush=True)
    r_csr, x_csr = run_batch(apcg, ctx, systems, 1e-10, 5000, batch_schedule=2, mode=mode)
    r_sd, x_sd = run_batch(apcg, ctx, systems, 1e-10, 5000, sdia=range(24), batch_schedule=2, mode=mode)
    print("switched", run_batch.switched, flush=True)
    assert len(run_batch.switched) >= 4 and len(run_batch.switched) < 24
    for a, b2, xa, xb in zip(r_csr, r_sd, x_csr, x_sd):
        assert a == b2
        assert np.array_equal(xa, xb)
    for s, r, x in zip(systems, r_sd, x_sd):
        ref = oracle.pcg(s.A, s.b, rtol=1e-10, maxit=5000)
        assert abs(r["iterations"] - ref.its) <= 1 and rel(x, ref.x) <= 1e-9


def unsymmetric_twin(A, frac=0.3):
    """A copy of A with the same (symmetric) pattern whose values are no
    longer symmetric: one entry left of the diagonal, about frac of the way
    down the rows, changed in its last bits."""
    T = P.CSR(n=A.n, rowptr=A.rowptr.copy(), col=A.col.copy(), val=A.val.copy())
    for i in range(int(frac * A.n), A.n):
        lo = [e for e in range(A.rowptr[i], A.rowptr[i + 1]) if A.col[e] < i]
        if lo:
            T.val[lo[0]] *= 1.0 + 2.0 ** -40
            return T
    raise AssertionError("no entry left of the diagonal")


def sliced_diagonal_batch():
    """Symmetric 2D and 3D systems spanning several tiles (offsets of one, a
    grid row and a plane, whose columns lie in the same tile or an earlier
    one), and twins whose values are not symmetric."""
    rng = np.random.default_rng(63)
    sym = [P._lognormal_system(rng, 2, 75, 1.0, 3.0), P._lognormal_system(rng, 3, 17, 1.0, 1.0),
           P._lognormal_system(rng, 2, 130, 1.5, 1.0), P._lognormal_system(rng, 3, 22, 0.7, 5.0)]
    twins = [P.System(A=unsymmetric_twin(s.A), b=s.b) for s in sym[:2]]
    return sym + twins, [1] * len(sym) + [0] * len(twins)


@pytest.mark.parametrize("mode", [0, 1])
def test_segmented_sliced_diagonals_multi_tile_bitwise(apcg, ctx, mode):
    """The tile product walks each slice of the sliced-diagonal copy with
    scalar loads of its offsets and masks and gathers at row + offset clamped
    into the system (an absent entry's product is dropped by the mask): bit
    for bit the all-CSR batch on 2D and 3D systems over several tiles, at two
    tile sizes, with symmetric values or not.  The copy's value-symmetry flag
    is as the refill's check finds it: set for the symmetric matrices,
    cleared for the twins."""
    systems, flags = sliced_diagonal_batch()
    print(f"case batched seg sliced diagonals multi-tile mode={mode}", flush=True)
    r_csr, x_csr = run_batch(apcg, ctx, systems, 1e-10, 20000, batch_schedule=2, mode=mode)
    for tr in (256, 2048):
        r_sd, x_sd = run_batch(apcg, ctx, systems, 1e-10, 20000, sdia=range(len(systems)), batch_schedule=2,
                               mode=mode, batch_tile_rows=tr)
        assert run_batch.switched == list(range(len(systems)))
        got = [apcg.apcg_mat_get_sdia_info(a.h)["values_symmetric"] for a in run_batch.mats]
        assert got == flags
        for a, b2, xa, xb in zip(r_csr, r_sd, x_csr, x_sd):
            assert a == b2
            assert np.array_equal(xa, xb)
    for s, r, x in zip(systems[:4], r_csr, x_csr):
        ref = oracle.pcg(s.A, s.b, rtol=1e-10, maxit=20000)
        assert abs(r["iterations"] - ref.its) <= 1 and rel(x, ref.x) <= 1e-9


@pytest.mark.parametrize("sdia", [False, True])
def test_segmented_tile_rows_bitwise(apcg, ctx, sdia):
    """The segmented schedule at 256, 1024 and 4096 rows per tile: a tile
    only groups 64-row slices for one workgroup, each slice's partial is its
    own wavefront's sum and every system adds its slices in index order, so
    the tile size changes the launch shape and nothing else -- whole batched
    solves are bit for bit equal (CSR reads and sliced-diagonal reads; sizes
    from 4 to 12,000 rows, so some systems span many tiles and some less than
    one slice).  The first one matches the oracle system by system."""
    rng = np.random.default_rng(62)
    systems = mixed_small_batch()[:12]
    systems += [P._lognormal_system(rng, 2, side, 1.0, 3.0) for side in (70, 100, 110)]
    print(f"case batched tile rows sdia={sdia}", flush=True)
    sd = range(len(systems)) if sdia else ()
    runs = [run_batch(apcg, ctx, systems, 1e-10, 20000, sdia=sd, batch_schedule=2, batch_tile_rows=tr)
            for tr in (256, 1024, 4096)]
    for res, xs in runs[1:]:
        assert res == runs[0][0]
        assert all(np.array_equal(a, b) for a, b in zip(xs, runs[0][1]))
    for s, r, x in zip(systems, *runs[0]):
        ref = oracle.pcg(s.A, s.b, rtol=1e-10, maxit=20000)
        assert r["status"] == ref.status
        if ref.status == oracle.CONVERGED:
            assert abs(r["iterations"] - ref.its) <= 1 and rel(x, ref.x) <= 1e-9


@pytest.mark.parametrize("sdia", [False, True])
def test_segmented_tail_plan_bitwise(apcg, ctx, sdia):
    """Once the rows still running fill fewer than two large tiles per
    compute unit, the iteration continues on a plan of smaller tiles (the
    tiles only group slices: the same sums).  This batch is below that size
    from the start, so the switch comes at the first poll: 4096-row tiles
    with the tail plan at 256 or 512 rows are bit for bit the run that keeps
    its tiles; the oracle's bar holds."""
    rng = np.random.default_rng(66)
    systems = mixed_small_batch()[:12]
    systems += [P._lognormal_system(rng, 2, side, 1.0, 3.0) for side in (90, 140)]
    print(f"case batched tail plan sdia={sdia}", flush=True)
    sd = range(len(systems)) if sdia else ()
    runs = [run_batch(apcg, ctx, systems, 1e-10, 20000, sdia=sd, batch_schedule=2, batch_tile_rows=4096,
                      batch_tail_tile_rows=tt) for tt in (-1, 256, 0)]
    for res, xs in runs[1:]:
        assert res == runs[0][0]
        assert all(np.array_equal(a, b) for a, b in zip(xs, runs[0][1]))
    for s, r, x in zip(systems, *runs[0]):
        ref = oracle.pcg(s.A, s.b, rtol=1e-10, maxit=20000)
        assert r["status"] == ref.status
        if ref.status == oracle.CONVERGED:
            assert abs(r["iterations"] - ref.its) <= 1 and rel(x, ref.x) <= 1e-9


def test_segmented_tile_rows_rejected(apcg, ctx):
    systems = mixed_small_batch()[:2]
    for tr in (100, 128, 8448, -256):
        with pytest.raises(apcg.ApcgError):
            run_batch(apcg, ctx, systems, 1e-8, 100, batch_schedule=2, batch_tile_rows=tr)


def test_segmented_tail_rows_rejected(apcg, ctx):
    systems = mixed_small_batch()[:3]
    for bad in (-2, 100, 9000):
        with pytest.raises(apcg.ApcgError):
            run_batch(apcg, ctx, systems, 1e-10, 100, batch_schedule=2, batch_tail_tile_rows=bad)


def test_batch_autotune_and_table(apcg, ctx):
    """The batched autotuner times the schedules on the device, keeps the
    best under the batch's key (a second call takes it from the table
    without timing), and the solve in the tuned configuration meets the
    oracle's bar system by system.  The members start on the sliced-diagonal
    schedule; afterwards they are on it exactly when the pick reads the
    sliced-diagonal copies (a CSR pick moves them to the row schedule, so
    that the batch reads what was timed)."""
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    rng = np.random.default_rng(63)
    systems = mixed_small_batch()[:20] + [P._lognormal_system(rng, 2, 90, 1.0, 2.0)]
    As = [DeviceCSR(s.A) for s in systems]
    bs = [DeviceVec(s.b) for s in systems]
    xs = [DeviceVec.zeros(s.A.n) for s in systems]
    on_sdia = []
    for i, a in enumerate(As):
        try:
            apcg.apcg_mat_set_spmv_config(a.h, 1, 256, 0, apcg.APCG_SPMV_SDIA)
            on_sdia.append(i)
        except apcg.ApcgError:
            pass
    assert len(on_sdia) >= 10

    def members_on_sdia():
        return [i for i, a in enumerate(As)
                if apcg.apcg_mat_get_spmv_config(a.h)["schedule"] == apcg.APCG_SPMV_SDIA]

    apcg.apcg_tune_cache_clear()
    cfg, ms, hit = apcg.apcg_batch_autotune(ctx, [a.h for a in As], [b.h for b in bs], [x.h for x in xs], 0, 16)
    print(f"case batch autotune: {cfg} {ms:.3f} ms", flush=True)
    assert not hit and ms > 0
    assert cfg["schedule"] in (apcg.APCG_BATCH_PERSISTENT, apcg.APCG_BATCH_SEGMENTED)
    assert members_on_sdia() == (on_sdia if cfg["sdia"] else [])
    cfg2, ms2, hit2 = apcg.apcg_batch_autotune(ctx, [a.h for a in As], [b.h for b in bs], [x.h for x in xs], 0, 16)
    assert hit2 and cfg2 == cfg and ms2 == ms
    assert members_on_sdia() == (on_sdia if cfg["sdia"] else [])
    assert apcg.apcg_tune_cache_size() == 1
    info = apcg.apcg_info_create(0, len(systems))
    opts = apcg.apcg_solve_opts_default(x0_is_zero=1, batch_schedule=cfg["schedule"],
                                        batch_block_size=cfg["block_size"], batch_tile_rows=cfg["tile_rows"])
    apcg.apcg_ksp_solve_batched(ctx, [a.h for a in As], [b.h for b in bs], [x.h for x in xs], 1e-10, 20000, opts,
                                info)
    for i, s in enumerate(systems):
        r = apcg.apcg_info_get(info, i)
        ref = oracle.pcg(s.A, s.b, rtol=1e-10, maxit=20000)
        assert r["status"] == ref.status, i
        if ref.status == oracle.CONVERGED:
            assert abs(r["iterations"] - ref.its) <= 1 and rel(xs[i].numpy(), ref.x) <= 1e-9, i
    apcg.apcg_info_destroy(info)
    apcg.apcg_tune_cache_clear()


def test_batched_vector_overlaps_rejected(apcg, ctx):
    """A solution vector may share no memory with another system's solution
    or with any right-hand side: the batched PCG and the batched FCG reject
    such a batch on the host (the same handle twice, two overlapping views of
    one buffer, one system's x on another's b) and solve the systems once
    the views are disjoint (adjacent views of one buffer)."""
    import torch
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    A = P.laplace_2d(6)
    n = A.n
    rng = np.random.default_rng(90)
    rhs = [rng.uniform(-1, 1, n) for _ in range(2)]
    As = [DeviceCSR(A), DeviceCSR(A)]
    bs = [DeviceVec(r) for r in rhs]
    big = torch.zeros(2 * n, dtype=torch.float64, device="cuda:0")
    x0 = DeviceVec.zeros(n)
    overlapping = [DeviceVec(big[0:n]), DeviceVec(big[n // 2:n // 2 + n])]
    on_b0 = DeviceVec(bs[0].t)
    hA, hb = [a.h for a in As], [b.h for b in bs]
    info = apcg.apcg_info_create(0, 2)
    opts = apcg.apcg_solve_opts_default(x0_is_zero=1)
    coef = torch.zeros(18, dtype=torch.float32, device="cuda:0")
    lmax = torch.full((2,), 8.0, dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    bad = {"same handle": [x0.h, x0.h], "overlapping views": [v.h for v in overlapping],
           "x on another system's b": [x0.h, on_b0.h]}
    for name, hx in bad.items():
        print(f"case overlap rejected: {name}", flush=True)
        with pytest.raises(apcg.ApcgError):
            apcg.apcg_ksp_solve_batched(ctx, hA, hb, hx, 1e-10, 100, opts, info)
        with pytest.raises(apcg.ApcgError):
            apcg.apcg_ksp_solve_batched_fcg_poly(ctx, hA, hb, hx, 1e-10, 100, coef, lmax, opts,
                                                 apcg.apcg_fcg_opts_default(), info)
    adjacent = [DeviceVec(big[0:n]), DeviceVec(big[n:2 * n])]
    apcg.apcg_ksp_solve_batched(ctx, hA, hb, [v.h for v in adjacent], 1e-10, 1000, opts, info)
    for i in range(2):
        r = apcg.apcg_info_get(info, i)
        ref = oracle.pcg(A, rhs[i], rtol=1e-10, maxit=1000)
        assert r["status"] == apcg.APCG_SOLVE_CONVERGED and abs(r["iterations"] - ref.its) <= 1
        assert rel(adjacent[i].numpy(), ref.x) <= 1e-9
    apcg.apcg_info_destroy(info)
