"""GPU parity at the workloads' full sizes, through the C ABI.

1. The mixed 2D/3D batch: a batch of members of the 1024-system mixed batch
   (seed 5) with more than 4.2 M rows in total, run on 256-row tiles so that
   the batched kernels' workgroups each own several tiles, including a 525,625-row 2D
   system with anisotropy 592 and members of up to 0.8 M rows.  The
   coefficients come from a network trained on the GPU (features ->
   standardisation -> network, read back from the device); one member gets a
   polynomial that fails the positivity check (its fallback runs inside the
   batch) and one the constant polynomial (FCG = Jacobi-PCG).  Every matrix is
   on the sliced-diagonal schedule, as in the benchmark.  Sampled members
   (the large 2D one among them) are compared with the oracle's FCG: status
   equal, iterations +-1, flexible iterations +-1 and ||x - x_ref|| / ||x_ref||
   <= 1e-9 at rtol 1e-10; every member's true residual is checked on the host;
   the one-call learned batched solve gives the same bits for every member
   whose polynomial was not replaced.
2. The learned single solve on a 3D system of side 80 from the learned
   workload's distribution (512,000 rows): the one-call learned solve equals
   features -> network -> FCG from the feature run's 12-step iterate bit for
   bit, and that FCG solve matches the oracle's FCG from the oracle's own
   12-step iterate at the same bar.
"""
import numpy as np
import pytest

import oracle
from paper_2306_17801_amd import problems as P

pytestmark = pytest.mark.gpu

# members of the mixed batch (seed 5): index -> role
BIG_2D = 282          # 2D, 725^2 = 525,625 rows, anisotropy 592, sigma 0.51
FILL = [253, 437, 979, 268, 686, 759]  # 3D 512k-636k rows and 2D 628k-789k rows (anisotropy 308-657)
SMALL = [1, 2, 4, 7, 9, 12, 16, 19, 30]
REJECT = 27           # gets a polynomial that is negative on [0, lmax]: fallback from the start
IDENT = 28            # gets p = 1: FCG(1) with p = 1 is Jacobi-PCG
RTOL = 1e-10
MAXIT = 50000


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


@pytest.fixture(scope="module")
def network(apcg, ctx):
    """A network trained on the GPU on 48 systems of the mixed distribution
    (seed 6, at most 1e5 rows)."""
    from paper_2306_17801_amd import learned as L

    print("case fullsize: training the network", flush=True)
    train = [P.mixed_system((6, i, 1e3, 1e5)) for i in range(48)]
    data = L.collect(ctx, train, rtol=1e-8, maxit=50000)
    pc, losses = L.train(ctx, data, epochs=150, batch=32, lr=3e-3)
    print(f"  loss {losses[0]:.3g} -> {losses[-1]:.3g}", flush=True)
    return pc


def coefficients(apcg, ctx, pc, As, bs):
    """Batched features -> standardisation -> network: the coefficients and
    lmax the learned batched solve uses (device tensors, row per system)."""
    import torch

    nsys = len(As)
    feat = torch.zeros((nsys, 16), dtype=torch.float32, device="cuda:0")
    lm = torch.zeros(nsys, dtype=torch.float64, device="cuda:0")
    C = torch.zeros((nsys, 9), dtype=torch.float32, device="cuda:0")
    torch.cuda.synchronize()
    apcg.apcg_pc_features_batched(ctx, [a.h for a in As], [b.h for b in bs], feat.view(-1), lm)
    apcg.apcg_mlp_standardize(ctx, feat, pc.mean, pc.std, False)
    apcg.apcg_mlp_forward(ctx, pc.params, feat, C)
    apcg.apcg_ctx_synchronize(ctx)
    return C, lm


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def oracle_many(jobs):
    """Oracle FCG solves on host threads (the C oracle runs without the GIL)."""
    from concurrent.futures import ThreadPoolExecutor

    def one(j):
        A, b, c, lm = j
        return oracle.fcg_poly(A, b, c, lm, rtol=RTOL, maxit=MAXIT)

    with ThreadPoolExecutor(min(len(jobs), oracle.host_threads())) as ex:
        return list(ex.map(one, jobs))


@pytest.mark.timeout(900)
def test_mixed_batch_full_size_parity(apcg, ctx, network):
    import torch
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    members = [BIG_2D] + FILL + SMALL + [REJECT, IDENT]
    print(f"case fullsize mixed batch: members {members}", flush=True)
    systems = [P.mixed_system((5, i, 1e3, 1e6)) for i in members]
    rows = sum(s.A.n for s in systems)
    tiles = sum((s.A.n + 255) // 256 for s in systems)
    print(f"  rows {rows}, 256-row tiles {tiles}", flush=True)
    assert rows > 4_200_000 and tiles > 2 * 8192  # several tiles per workgroup (at most 8192 workgroups)
    big = systems[0]
    assert big.A.n >= 500_000 and big.meta["dim"] == 2 and big.meta["aniso"] >= 300
    As = [DeviceCSR(s.A) for s in systems]
    for a in As:
        apcg.apcg_mat_set_spmv_config(a.h, 1, 256, 0, apcg.APCG_SPMV_SDIA)
    bs = [DeviceVec(s.b) for s in systems]
    C, lm = coefficients(apcg, ctx, network, As, bs)
    coef = C.cpu().numpy().copy()
    lmax = lm.cpu().numpy()
    bad = np.zeros(9, np.float32)
    bad[0], bad[1] = 0.2, -0.5
    e0 = np.zeros(9, np.float32)
    e0[0] = 1.0
    coef[members.index(REJECT)] = bad
    coef[members.index(IDENT)] = e0
    dcoef = torch.from_numpy(coef.reshape(-1)).to("cuda:0")
    torch.cuda.synchronize()
    # 256-row tiles: more tiles than the grid's 8192 workgroups, so each
    # workgroup screens and runs several tiles
    opts = apcg.apcg_solve_opts_default(x0_is_zero=1, batch_tile_rows=256)
    nsys = len(systems)
    info = apcg.apcg_info_create(0, nsys)
    xs = [DeviceVec.zeros(s.A.n) for s in systems]
    apcg.apcg_ksp_solve_batched_fcg_poly(ctx, [a.h for a in As], [b.h for b in bs], [x.h for x in xs], RTOL, MAXIT,
                                         dcoef, lm, opts, None, info)
    res = [apcg.apcg_info_get(info, i) for i in range(nsys)]
    xo = [x.numpy() for x in xs]
    # the one-call learned batched solve: same features, network and kernels
    info2 = apcg.apcg_info_create(0, nsys)
    x2 = [DeviceVec.zeros(s.A.n) for s in systems]
    apcg.apcg_ksp_solve_batched_learned(ctx, [a.h for a in As], [b.h for b in bs], [x.h for x in x2], RTOL, MAXIT,
                                        network.params, network.mean, network.std, opts, None, info2)
    res2 = [apcg.apcg_info_get(info2, i) for i in range(nsys)]
    for i, m in enumerate(members):
        if m in (REJECT, IDENT):
            continue
        assert res2[i] == res[i], (m, res2[i], res[i])
        assert np.array_equal(x2[i].numpy(), xo[i]), m
    # every member: converged, true residual close to the recursive one
    for i, (m, s) in enumerate(zip(members, systems)):
        r = res[i]
        tr = np.linalg.norm(s.b - s.A.to_scipy() @ xo[i]) / np.linalg.norm(s.b)
        print(f"  member {m} n={s.A.n}: its {r['iterations']} fcg {r['fcg_iterations']} st {r['status']} "
              f"true relres {tr:.2e}", flush=True)
        assert r["status"] & apcg.APCG_SOLVE_CONVERGED, (m, r)
        assert tr <= 3 * RTOL, (m, tr)
    rj = res[members.index(REJECT)]
    assert rj["fcg_iterations"] == 0 and rj["status"] & apcg.APCG_SOLVE_FALLBACK
    # the oracle on the sampled members, with the coefficients the device used
    sample = [BIG_2D] + SMALL + [REJECT, IDENT]
    jobs = [(systems[members.index(m)].A, systems[members.index(m)].b, coef[members.index(m)].astype(np.float64),
             float(lmax[members.index(m)])) for m in sample]
    print(f"  oracle FCG on {len(sample)} members ...", flush=True)
    refs = oracle_many(jobs)
    for m, ref in zip(sample, refs):
        i = members.index(m)
        r = res[i]
        e = rel(xo[i], ref.x)
        print(f"  member {m}: gpu its {r['iterations']} fcg {r['fcg_iterations']} st {r['status']} | oracle its "
              f"{ref.its} fcg {ref.fcg_its} st {ref.status} | rel {e:.2e}", flush=True)
        assert r["status"] == ref.status, m
        assert abs(r["iterations"] - ref.its) <= 1, m
        assert abs(r["fcg_iterations"] - ref.fcg_its) <= 1, m
        assert e <= 1e-9, m
    for inf in (info, info2):
        apcg.apcg_info_destroy(inf)
    for v in xs + x2 + bs:
        v.close()
    for a in As:
        a.close()


@pytest.mark.timeout(600)
def test_learned_single_solve_side_80(apcg, ctx, network):
    import torch
    from paper_2306_17801_amd import learned as L
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    # the first member of the learned workload's held-out set (seed 40) drawn
    # at side 80: sigma and anisotropy from the workload's distribution
    s = P.learned_pc_fields((40, 0, 200, 80, 80)).system()
    print(f"case fullsize learned single solve: n={s.A.n} {s.meta}", flush=True)
    assert s.A.n == 512_000
    A, b = DeviceCSR(s.A), DeviceVec(s.b)
    feat = torch.zeros((1, 16), dtype=torch.float32, device="cuda:0")
    lm = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    C = torch.zeros((1, 9), dtype=torch.float32, device="cuda:0")
    torch.cuda.synchronize()
    apcg.apcg_pc_features(ctx, A.h, b.h, feat.view(-1), lm)
    apcg.apcg_mlp_standardize(ctx, feat, network.mean, network.std, False)
    apcg.apcg_mlp_forward(ctx, network.params, feat, C)
    opts = apcg.apcg_solve_opts_default(x0_is_zero=1)
    info = apcg.apcg_info_create(0, 2)
    x1, x2 = DeviceVec.zeros(s.A.n), DeviceVec.zeros(s.A.n)
    # the learned solve starts from the feature run's 12 Jacobi-PCG steps
    apcg.apcg_ksp_solve(ctx, A.h, b.h, x1.h, 0.0, 12, opts, info, 0)
    warm = apcg.apcg_solve_opts_default(x0_is_zero=0)
    apcg.apcg_ksp_solve_fcg_poly(ctx, A.h, b.h, x1.h, RTOL, MAXIT, C.view(-1), lm, warm, None, info, 0)
    L.solve(ctx, network, A.h, b.h, x2.h, RTOL, MAXIT, opts, None, info, 1)
    r1, r2 = apcg.apcg_info_get(info, 0), apcg.apcg_info_get(info, 1)
    assert r1 == r2
    xa = x1.numpy()
    assert np.array_equal(xa, x2.numpy())
    c = C.cpu().numpy().reshape(-1).astype(np.float64)
    x12 = oracle.pcg(s.A, s.b, rtol=0.0, maxit=12).x
    ref = oracle.fcg_poly(s.A, s.b, c, float(lm.cpu()[0]), x0=x12, rtol=RTOL, maxit=MAXIT)
    e = rel(xa, ref.x)
    print(f"  gpu its {r1['iterations']} fcg {r1['fcg_iterations']} st {r1['status']} | oracle its {ref.its} "
          f"fcg {ref.fcg_its} st {ref.status} | rel {e:.2e}", flush=True)
    assert r1["status"] == ref.status and r1["status"] & apcg.APCG_SOLVE_CONVERGED
    assert abs(r1["iterations"] - ref.its) <= 1 and abs(r1["fcg_iterations"] - ref.fcg_its) <= 1
    assert e <= 1e-9
    apcg.apcg_info_destroy(info)
    for v in (x1, x2, b):
        v.close()
    A.close()
