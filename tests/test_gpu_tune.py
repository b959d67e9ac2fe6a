"""GPU tests of the tuning table: the single-matrix autotuner through the
table (a second matrix of the same pattern class and size bucket takes the
first one's configuration without timing) and the batched autotuner of the
flexible (FCG) solve; the solves in the tuned configurations meet the
oracle's bar."""
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


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def test_mat_autotune_cached_reuses_the_pattern_class(apcg, ctx):
    """Two 24^3 diffusion matrices with different coefficients share the
    table key (device, pattern class, size bucket, nonzeros per row): the
    first call times the schedules and stores the best, the second applies
    it without timing; the second matrix then solves to the oracle's bar in
    that configuration."""
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    rng = np.random.default_rng(70)
    A1 = P.diffusion_csr(np.exp(rng.standard_normal((24, 24, 24))), aniso=1.0)
    A2 = P.diffusion_csr(np.exp(0.5 * rng.standard_normal((24, 24, 24))), aniso=3.0)
    d1, d2 = DeviceCSR(A1), DeviceCSR(A2)
    key = apcg.apcg_mat_tune_key(d1.h)
    assert key == apcg.apcg_mat_tune_key(d2.h)
    apcg.apcg_tune_cache_clear()
    print(f"case cached autotune {key}", flush=True)
    cfg1, us1, hit1 = apcg.apcg_mat_autotune_cached(d1.h, ctx, 3)
    assert not hit1 and us1 > 0
    look = apcg.apcg_tune_cache_lookup(key)
    assert look is not None
    assert look[0] == (cfg1["lanes_per_row"], cfg1["block_size"], cfg1["blocks"], cfg1["schedule"])
    cfg2, us2, hit2 = apcg.apcg_mat_autotune_cached(d2.h, ctx, 3)
    assert hit2 and cfg2 == cfg1 and us2 == us1
    assert apcg.apcg_mat_get_spmv_config(d2.h) == cfg1
    assert apcg.apcg_tune_cache_size() == 1
    b = rng.uniform(-1, 1, A2.n)
    db, dx = DeviceVec(b), DeviceVec.zeros(A2.n)
    info = apcg.apcg_info_create(0, 1)
    apcg.apcg_ksp_solve(ctx, d2.h, db.h, dx.h, 1e-10, 5000, apcg.apcg_solve_opts_default(x0_is_zero=1), info, 0)
    r = apcg.apcg_info_get(info, 0)
    ref = oracle.pcg(A2, b, rtol=1e-10, maxit=5000)
    assert r["status"] == apcg.APCG_SOLVE_CONVERGED and abs(r["iterations"] - ref.its) <= 1
    assert rel(dx.numpy(), ref.x) <= 1e-9
    apcg.apcg_info_destroy(info)
    apcg.apcg_tune_cache_clear()


def test_batch_autotune_fcg_and_table(apcg, ctx):
    """The batched autotuner of the flexible solve (kind 1: the constant
    polynomial, every Clenshaw step run) times segmented configurations,
    keeps the best under the batch's key and leaves the members on the
    layout it read (sliced-diagonal copies exactly when the pick does); the
    batched FCG in that configuration meets the oracle's bar."""
    from numpy.polynomial import chebyshev as Ch

    import torch
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    rng = np.random.default_rng(71)
    sides = [int(rng.integers(20, 70)) if k % 2 == 0 else int(rng.integers(8, 18)) for k in range(12)]
    systems = [P._lognormal_system(rng, 2 + (k % 2), sides[k], 1.0, 3.0) for k in range(12)]
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
    assert len(on_sdia) == len(As)

    def members_on_sdia():
        return [i for i, a in enumerate(As)
                if apcg.apcg_mat_get_spmv_config(a.h)["schedule"] == apcg.APCG_SPMV_SDIA]

    hA, hb, hx = [a.h for a in As], [b.h for b in bs], [x.h for x in xs]
    apcg.apcg_tune_cache_clear()
    cfg, ms, hit = apcg.apcg_batch_autotune(ctx, hA, hb, hx, 1, 4)
    print(f"case batch autotune fcg: {cfg} {ms:.3f} ms", flush=True)
    assert not hit and ms > 0 and cfg["schedule"] == apcg.APCG_BATCH_SEGMENTED
    assert members_on_sdia() == (on_sdia if cfg["sdia"] else [])
    cfg2, ms2, hit2 = apcg.apcg_batch_autotune(ctx, hA, hb, hx, 1, 4)
    assert hit2 and cfg2 == cfg and ms2 == ms
    assert members_on_sdia() == (on_sdia if cfg["sdia"] else [])

    # a Chebyshev polynomial on [lmax / 30, lmax] per system
    def cheb_coeffs(lmax, a):
        T9 = [0] * 9 + [1]
        s0 = (lmax + a) / (lmax - a)

        def f(y):
            t = (y + 1) * lmax / 2
            return (1 - Ch.chebval((lmax + a - 2 * t) / (lmax - a), T9) / Ch.chebval(s0, T9)) / t

        return Ch.chebinterpolate(f, 8)

    lms = [oracle.gershgorin(s.A)[1] for s in systems]
    cs = [cheb_coeffs(lm, lm / 30).astype(np.float32) for lm in lms]
    coef = torch.from_numpy(np.concatenate(cs)).to("cuda:0")
    lm = torch.from_numpy(np.array(lms, np.float64)).to("cuda:0")
    torch.cuda.synchronize()
    info = apcg.apcg_info_create(0, len(systems))
    opts = apcg.apcg_solve_opts_default(x0_is_zero=1, batch_tile_rows=cfg["tile_rows"])
    apcg.apcg_ksp_solve_batched_fcg_poly(ctx, hA, hb, hx, 1e-10, 20000, coef, lm, opts,
                                         apcg.apcg_fcg_opts_default(), info)
    for i, s in enumerate(systems):
        r = apcg.apcg_info_get(info, i)
        ref = oracle.fcg_poly(s.A, s.b, cs[i].astype(np.float64), lms[i], rtol=1e-10, maxit=20000)
        assert r["status"] == ref.status, i
        assert abs(r["iterations"] - ref.its) <= 1, i
        assert rel(xs[i].numpy(), ref.x) <= 1e-9, i
    apcg.apcg_info_destroy(info)
    apcg.apcg_tune_cache_clear()
