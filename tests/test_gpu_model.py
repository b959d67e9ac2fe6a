"""The programming model beyond the solvers, on the GPU and through the C
ABI: scalar expressions (Section 3.2.1: Eval / Execute, MultiEval) against
the oracle's evaluator, and dependency marking of the caller's own work on
registered memory and on library objects (Section 3.1.2)."""
import math

import numpy as np
import pytest

from oracle import expr as OX

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


def scalars(apcg, ctx, values):
    out = []
    for v in values:
        s = apcg.apcg_scalar_create(ctx)
        apcg.apcg_scalar_set(s, float(v), ctx)
        out.append(s)
    return out


def programs():
    from paper_2306_17801_amd.expr import Sym, const, cos, exp, fabs, log, maximum, minimum, recip, sin, sqrt

    x, y, z = Sym.inputs(3)
    exact = {
        "paper_example": [sqrt(fabs(((x + y) / z) * z)) + 15.0],
        "cg_scalars": [x / y, y / z, -(x / y), recip(z) * x],
        "shared": [(x - y) * (x - y) + (x - y), minimum(x, y) - maximum(y, z), x * 1.0 + (z - 0.0)],
        "folded": [(const(3.0) * 7.0 - 1.0) / x, sqrt(const(2.0)) * y],
    }
    transcendental = {
        "trig": [sin(x) * sin(x) + cos(x) * cos(x), sin(((x + y) / z) * z) + 15.0],
        "explog": [exp(log(fabs(y))) - fabs(y), log(fabs(x) + 1.0) * exp(-fabs(z))],
    }
    return exact, transcendental


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_expr_matches_oracle(apcg, ctx, seed):
    """Every output equals the oracle's postfix evaluation: bit for bit for
    the correctly rounded operations (CSE, folding and the exact rewrites
    change nothing), within 4 ulp for exp/log/sin/cos."""
    from paper_2306_17801_amd.expr import Eval

    rng = np.random.default_rng(seed)
    vals = list(rng.uniform(-3, 3, 3))
    ins = scalars(apcg, ctx, vals)
    exact, trans = programs()
    for group, tol_ulp in ((exact, 0), (trans, 4)):
        for name, outs in group.items():
            print(f"case expr {name} seed={seed}", flush=True)
            e = Eval(outs, ninputs=3)
            res = scalars(apcg, ctx, [0.0] * len(outs))
            e.execute(ctx, ins, res)
            got = [apcg.apcg_scalar_get(r) for r in res]
            want = OX.eval_postfix(e.tokens, vals, len(outs))
            for g, w in zip(got, want):
                if tol_ulp == 0:
                    assert g == w or (math.isnan(g) and math.isnan(w)), (name, g, w)
                else:
                    assert abs(g - w) <= tol_ulp * np.spacing(max(abs(w), 1e-300)) + 1e-15, (name, g, w)
            for r in res:
                apcg.apcg_scalar_destroy(r)
            e.close()
    for s in ins:
        apcg.apcg_scalar_destroy(s)


def test_expr_one_launch_and_in_place(apcg, ctx):
    """A multi-output program is one kernel launch; an output may be one of
    the inputs (x <- 2x + y, three times in a row on the device)."""
    from paper_2306_17801_amd.expr import Eval, Sym

    x, y = Sym.inputs(2)
    sx, sy = scalars(apcg, ctx, [1.5, 0.25])
    o1, o2, o3 = scalars(apcg, ctx, [0.0, 0.0, 0.0])
    e3 = Eval([x * y, x + y, x - y], 2)
    apcg.apcg_ctx_synchronize(ctx)
    before = apcg.apcg_counters_get()["kernel_launches"]
    e3.execute(ctx, [sx, sy], [o1, o2, o3])
    assert apcg.apcg_counters_get()["kernel_launches"] - before == 1
    assert [apcg.apcg_scalar_get(o) for o in (o1, o2, o3)] == [1.5 * 0.25, 1.75, 1.25]
    step = Eval([2.0 * x + y], 2)
    for _ in range(3):
        step.execute(ctx, [sx, sy], [sx])
    v = 1.5
    for _ in range(3):
        v = 2.0 * v + 0.25
    assert apcg.apcg_scalar_get(sx) == v
    for h in (sx, sy, o1, o2, o3):
        apcg.apcg_scalar_destroy(h)


def test_expr_ordered_across_contexts(apcg):
    """A long reduction on context A writes a scalar; an expression on
    context B reads it: B's kernel waits for A's (write-read order)."""
    import torch
    from paper_2306_17801_amd.expr import Eval, Sym

    a, b = apcg.apcg_ctx_create(0), apcg.apcg_ctx_create(0)
    n = 1 << 25
    u = torch.full((n,), 0.5, dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    hu = apcg.apcg_vec_wrap(u)
    d = apcg.apcg_scalar_create(a)
    out = apcg.apcg_scalar_create(b)
    (x,) = Sym.inputs(1)
    e = Eval([x / 4.0 + 1.0], 1)
    for _ in range(3):
        apcg.apcg_vec_dot_async(hu, hu, d, a)
    e.execute(b, [d], [out])
    assert apcg.apcg_scalar_get(out) == (0.25 * n) / 4.0 + 1.0
    apcg.apcg_ctx_synchronize(a)
    apcg.apcg_vec_destroy(hu)
    apcg.apcg_scalar_destroy(d)
    apcg.apcg_scalar_destroy(out)
    apcg.apcg_ctx_destroy(a)
    apcg.apcg_ctx_destroy(b)


def test_marking_registered_memory(apcg):
    """The caller's own kernels (torch on the contexts' streams) on a
    registered region: a write on A then a read on B (B copies the final
    values), and a read on B then a write on A (B copies the old values)."""
    import torch

    a, b = apcg.apcg_ctx_create(0), apcg.apcg_ctx_create(0)
    sa = torch.cuda.ExternalStream(apcg.apcg_ctx_get_stream(a))
    sb = torch.cuda.ExternalStream(apcg.apcg_ctx_get_stream(b))
    n = 1 << 24
    buf = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    rid = apcg.apcg_memory_register(0, buf.data_ptr(), buf.numel() * 8)
    assert apcg.apcg_memory_register(0, buf.data_ptr(), buf.numel() * 8) == rid
    assert apcg.apcg_memory_lookup(0, buf.data_ptr() + 8 * 1000) == (rid, buf.data_ptr(), n * 8)
    W, R = apcg.APCG_ACCESS_WRITE, apcg.APCG_ACCESS_READ
    # write on A (many passes), then read on B
    apcg.apcg_mark_intent_begin(a, rid, W, "fill")
    with torch.cuda.stream(sa):
        for _ in range(40):
            buf.add_(1.0)
    apcg.apcg_mark_intent_end(a, rid, W, "fill")
    apcg.apcg_mark_intent_begin(b, rid, R, "copy")
    with torch.cuda.stream(sb):
        snap = buf.clone()
    apcg.apcg_mark_intent_end(b, rid, R, "copy")
    torch.cuda.synchronize()
    assert bool(torch.all(snap == 40.0))
    # read on B (several copies), then a write on A
    apcg.apcg_mark_intent_begin(b, rid, R, "copies")
    with torch.cuda.stream(sb):
        snaps = [buf.clone() for _ in range(8)]
    apcg.apcg_mark_intent_end(b, rid, R, "copies")
    apcg.apcg_mark_intent_begin(a, rid, W, "overwrite")
    with torch.cuda.stream(sa):
        buf.fill_(-1.0)
    apcg.apcg_mark_intent_end(a, rid, W, "overwrite")
    torch.cuda.synchronize()
    assert all(bool(torch.all(s == 40.0)) for s in snaps)
    assert bool(torch.all(buf == -1.0))
    # overlapping registration, unknown ids and modes are rejected
    with pytest.raises(apcg.ApcgError):
        apcg.apcg_memory_register(0, buf.data_ptr() + 64, 128)
    with pytest.raises(apcg.ApcgError):
        apcg.apcg_mark_intent_begin(a, rid + 10**6, R, "unknown")
    with pytest.raises(apcg.ApcgError):
        apcg.apcg_mark_intent_begin(a, rid, 7, "bad mode")
    apcg.apcg_memory_unregister(rid)
    with pytest.raises(apcg.ApcgError):
        apcg.apcg_memory_lookup(0, buf.data_ptr())
    apcg.apcg_ctx_synchronize(a)
    apcg.apcg_ctx_synchronize(b)
    apcg.apcg_ctx_destroy(a)
    apcg.apcg_ctx_destroy(b)


def test_marking_library_objects(apcg):
    """A vector's id orders the caller's own write (torch on A's stream)
    before the library's read of the vector on B (a dot product)."""
    import torch

    a, b = apcg.apcg_ctx_create(0), apcg.apcg_ctx_create(0)
    sa = torch.cuda.ExternalStream(apcg.apcg_ctx_get_stream(a))
    n = 1 << 24
    t = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    v = apcg.apcg_vec_wrap(t)
    vid = apcg.apcg_vec_get_id(v)
    assert apcg.apcg_vec_get_id(v) == vid
    apcg.apcg_mark_intent_begin(a, vid, apcg.APCG_ACCESS_WRITE, "user fill")
    with torch.cuda.stream(sa):
        for _ in range(30):
            t.add_(0.5)
    apcg.apcg_mark_intent_end(a, vid, apcg.APCG_ACCESS_WRITE, "user fill")
    s = apcg.apcg_scalar_create(b)
    apcg.apcg_vec_dot_async(v, v, s, b)
    assert apcg.apcg_scalar_get(s) == 225.0 * n
    apcg.apcg_scalar_destroy(s)
    apcg.apcg_vec_destroy(v)
    apcg.apcg_ctx_synchronize(a)
    apcg.apcg_ctx_destroy(a)
    apcg.apcg_ctx_destroy(b)
