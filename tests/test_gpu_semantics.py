"""GPU tests of the context model (Section 3.1): program order on one
context, write-write / write-read / read-write ordering across contexts by
call order, no read-read ordering, fork/join, globally blocking contexts,
host accessors that wait for the last writer, safe destruction before idle,
and a solve that never blocks the host per iteration.

A long chain of large vector updates on one context makes a missing
cross-context wait visible: the other context would read partial data."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N = 1 << 25  # 256 MiB per vector: each update takes tens of microseconds
CHAIN = 40


@pytest.fixture(scope="module")
def apcg():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_17801_amd as m

    m.load()
    return m


@pytest.fixture(scope="module")
def vecs(apcg):
    from paper_2306_17801_amd.device import DeviceVec

    x = DeviceVec.zeros(N)
    ones = DeviceVec.zeros(N)
    yield x, ones


def _chain(apcg, ctx, x, ones, a):
    """x = CHAIN after CHAIN additions of ones (a = 1)."""
    apcg.apcg_vec_set_async(x.h, 0.0, ctx)
    for _ in range(CHAIN):
        apcg.apcg_vec_axpy_async(x.h, a, False, ones.h, ctx)


def test_write_then_read_on_another_context(apcg, vecs):
    x, ones = vecs
    A, B = apcg.apcg_ctx_create(0), apcg.apcg_ctx_create(0)
    a = apcg.apcg_scalar_create(A)
    apcg.apcg_scalar_set(a, 1.0, A)
    apcg.apcg_vec_set_async(ones.h, 1.0, A)
    s = apcg.apcg_scalar_create(B)
    _chain(apcg, A, x, ones, a)
    apcg.apcg_vec_dot_async(x.h, ones.h, s, B)  # must wait for the whole chain on A
    assert apcg.apcg_scalar_get(s) == float(CHAIN) * N
    for h in (a, s):
        apcg.apcg_scalar_destroy(h)
    apcg.apcg_ctx_synchronize(A)
    apcg.apcg_ctx_destroy(A)
    apcg.apcg_ctx_destroy(B)


def test_write_write_ordered_by_call_order(apcg, vecs):
    x, ones = vecs
    A, B = apcg.apcg_ctx_create(0), apcg.apcg_ctx_create(0)
    a = apcg.apcg_scalar_create(A)
    apcg.apcg_scalar_set(a, 1.0, A)
    apcg.apcg_vec_set_async(ones.h, 1.0, A)
    _chain(apcg, A, x, ones, a)
    apcg.apcg_vec_set_async(x.h, -3.0, B)  # the later write wins
    out = x.numpy()
    assert np.all(out == -3.0)
    apcg.apcg_scalar_destroy(a)
    apcg.apcg_ctx_destroy(A)
    apcg.apcg_ctx_destroy(B)


def test_read_then_write_on_another_context(apcg, vecs):
    x, ones = vecs
    A, B = apcg.apcg_ctx_create(0), apcg.apcg_ctx_create(0)
    a = apcg.apcg_scalar_create(A)
    s = apcg.apcg_scalar_create(A)
    apcg.apcg_scalar_set(a, 1.0, A)
    apcg.apcg_vec_set_async(ones.h, 1.0, A)
    _chain(apcg, A, x, ones, a)
    apcg.apcg_vec_dot_async(x.h, ones.h, s, A)  # reads x (value CHAIN) ...
    apcg.apcg_vec_set_async(x.h, 0.0, B)         # ... before B overwrites it
    assert apcg.apcg_scalar_get(s) == float(CHAIN) * N
    assert np.all(x.numpy() == 0.0)
    for h in (a, s):
        apcg.apcg_scalar_destroy(h)
    apcg.apcg_ctx_destroy(A)
    apcg.apcg_ctx_destroy(B)


def test_reads_are_not_ordered(apcg, vecs):
    """Two contexts reading the same vector insert no cross-context wait."""
    x, ones = vecs
    A, B = apcg.apcg_ctx_create(0), apcg.apcg_ctx_create(0)
    apcg.apcg_vec_set_async(x.h, 2.0, A)
    apcg.apcg_vec_set_async(ones.h, 1.0, A)
    apcg.apcg_ctx_synchronize(A)
    sa, sb = apcg.apcg_scalar_create(A), apcg.apcg_scalar_create(B)
    apcg.apcg_ctx_synchronize(B)
    apcg.apcg_counters_reset()
    apcg.apcg_vec_dot_async(x.h, ones.h, sa, A)
    apcg.apcg_vec_dot_async(x.h, ones.h, sb, B)
    # the read on B waits once for each of A's last writes (x and ones); the
    # read on A waits for nothing; no read waits for another read
    waits = apcg.apcg_counters_get()["stream_waits"]
    assert waits <= 2
    assert apcg.apcg_scalar_get(sa) == apcg.apcg_scalar_get(sb) == 2.0 * N
    apcg.apcg_counters_reset()
    apcg.apcg_vec_dot_async(x.h, ones.h, sa, A)
    apcg.apcg_vec_dot_async(x.h, ones.h, sb, B)
    assert apcg.apcg_counters_get()["stream_waits"] == 0
    for h in (sa, sb):
        apcg.apcg_scalar_destroy(h)
    apcg.apcg_ctx_destroy(A)
    apcg.apcg_ctx_destroy(B)


def test_fork_join(apcg):
    from paper_2306_17801_amd.device import DeviceVec

    P0 = apcg.apcg_ctx_create(0)
    vs = [DeviceVec.zeros(1 << 22) for _ in range(3)]
    for v in vs:
        apcg.apcg_vec_set_async(v.h, 1.0, P0)
    kids = apcg.apcg_ctx_fork(P0, 3)
    for i, (k, v) in enumerate(zip(kids, vs)):
        a = apcg.apcg_scalar_create(k)
        apcg.apcg_scalar_set(a, float(i + 2), k)
        apcg.apcg_vec_scale_async(v.h, a, k)
        apcg.apcg_scalar_destroy(a)  # destroyed before the scale ran: still safe
    apcg.apcg_ctx_join(P0, kids, apcg.APCG_JOIN_DESTROY)
    s = apcg.apcg_scalar_create(P0)
    for i, v in enumerate(vs):
        apcg.apcg_vec_norm2_async(v.h, s, P0)
        assert apcg.apcg_scalar_get(s) == pytest.approx((i + 2) * np.sqrt(v.n), rel=1e-14)
    apcg.apcg_scalar_destroy(s)
    apcg.apcg_ctx_destroy(P0)


def test_join_sync_and_no_sync(apcg):
    P0 = apcg.apcg_ctx_create(0)
    kids = apcg.apcg_ctx_fork(P0, 2)
    apcg.apcg_ctx_join(P0, kids, apcg.APCG_JOIN_SYNC)
    assert all(apcg.apcg_ctx_query_idle(k) for k in kids)
    apcg.apcg_ctx_join(P0, kids, apcg.APCG_JOIN_NO_SYNC)
    apcg.apcg_ctx_join(P0, kids, apcg.APCG_JOIN_DESTROY)
    apcg.apcg_ctx_destroy(P0)


def test_global_blocking_context_completes_before_return(apcg, vecs):
    x, ones = vecs
    G = apcg.apcg_ctx_create(0, apcg.APCG_STREAM_GLOBAL_BLOCKING)
    assert apcg.apcg_ctx_get_stream_type(G) == apcg.APCG_STREAM_GLOBAL_BLOCKING
    A = apcg.apcg_ctx_create(0)
    a = apcg.apcg_scalar_create(A)
    apcg.apcg_scalar_set(a, 1.0, A)
    apcg.apcg_vec_set_async(ones.h, 1.0, A)
    _chain(apcg, A, x, ones, a)
    s = apcg.apcg_scalar_create(G)
    apcg.apcg_vec_dot_async(x.h, ones.h, s, G)  # waits for A's chain, done on return
    assert apcg.apcg_ctx_query_idle(G) and apcg.apcg_ctx_query_idle(A)
    apcg.apcg_counters_reset()
    assert apcg.apcg_scalar_get(s) == float(CHAIN) * N
    assert apcg.apcg_counters_get()["host_syncs"] <= 1
    # NULL context = the per-device globally blocking context (Eval without a context)
    t = apcg.apcg_scalar_create(None)
    apcg.apcg_vec_dot_async(x.h, ones.h, t, None)
    assert apcg.apcg_scalar_get(t) == float(CHAIN) * N
    for h in (a, s, t):
        apcg.apcg_scalar_destroy(h)
    apcg.apcg_ctx_destroy(A)
    apcg.apcg_ctx_destroy(G)
    with pytest.raises(apcg.ApcgError):
        apcg.apcg_ctx_create(0, 7)


def test_destroy_before_idle_is_safe(apcg, vecs):
    x, ones = vecs
    A = apcg.apcg_ctx_create(0)
    a = apcg.apcg_scalar_create(A)
    apcg.apcg_scalar_set(a, 1.0, A)
    apcg.apcg_vec_set_async(ones.h, 1.0, A)
    _chain(apcg, A, x, ones, a)
    apcg.apcg_scalar_destroy(a)  # still used by queued work
    apcg.apcg_ctx_destroy(A)     # stream still busy
    # a new context and scalars reuse released resources only after the work ended
    B = apcg.apcg_ctx_create(0)
    ss = [apcg.apcg_scalar_create(B) for _ in range(8)]
    for i, s in enumerate(ss):
        apcg.apcg_scalar_set(s, float(i), B)
    assert [apcg.apcg_scalar_get(s) for s in ss] == [float(i) for i in range(8)]
    assert np.all(x.numpy() == float(CHAIN))
    for s in ss:
        apcg.apcg_scalar_destroy(s)
    apcg.apcg_ctx_destroy(B)


def test_solve_has_no_per_iteration_host_wait(apcg):
    """Graph mode: no stream/device synchronisation inside the solve; the
    host only polls an event queued one graph earlier (at most one poll per
    K iterations).  The host-check mode, the synchronous shape, syncs after
    every kernel."""
    from paper_2306_17801_amd import problems as P
    from paper_2306_17801_amd.device import DeviceCSR, DeviceVec

    s = P.poisson2d_manufactured(64, 0)
    ctx = apcg.apcg_ctx_create(0)
    A, b, x = DeviceCSR(s.A), DeviceVec(s.b), DeviceVec.zeros(s.A.n)
    info = apcg.apcg_info_create(0, 1)
    for mode, K in ((apcg.APCG_MODE_GRAPH, 16), (apcg.APCG_MODE_STREAM, 16), (apcg.APCG_MODE_HOST_CHECK, 16)):
        opts = apcg.apcg_solve_opts_default(x0_is_zero=1, mode=mode, iters_per_graph=K)
        apcg.apcg_counters_reset()
        apcg.apcg_ksp_solve(ctx, A.h, b.h, x.h, 1e-10, 10000, opts, info, 0)
        c = apcg.apcg_counters_get()
        its = apcg.apcg_info_get(info, 0)["iterations"]
        if mode == apcg.APCG_MODE_HOST_CHECK:
            assert c["host_syncs"] >= 2 * its
        else:
            assert c["host_syncs"] == 0
            assert c["host_polls"] <= its // K + 2
            if mode == apcg.APCG_MODE_GRAPH:
                assert c["kernel_launches"] <= 4 and c["graph_launches"] <= its // K + 3
    apcg.apcg_info_destroy(info)
    apcg.apcg_ctx_destroy(ctx)
